"""GPU parity of the learned form: proposal-network forward and gradients
(bfloat16 matrix cores vs the oracle's bfloat16 emulation), Adam, features,
and the proposal -> refinement -> threshold -> fallback sequence."""
import math
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
import scenegen
from parity import assert_parity, axial_angle, compare

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _native():
    from paper_2604_05794_amd import native
    native.lib()
    return native


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for (W, b) in oracle.mlp_split(np.zeros(oracle.mlp_n_params())):
        parts.append(rng.normal(0, 1.0 / math.sqrt(W.shape[0]), W.size))
        parts.append(rng.normal(0, 0.1, b.size))
    return np.concatenate(parts).astype(np.float32)


def _rand_feats(seed, B):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (B, 112)).astype(np.float32)
    return oracle.round_bf16(x)


def _bf16_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV).to(torch.bfloat16)


def test_forward_matches_bfloat16_oracle():
    nat = _native()
    p = _rand_params(1)
    x = _rand_feats(1, 1000)
    net = nat.MLP(seed=0)
    net.set_params(p)
    y = net.forward(_bf16_dev(x))
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    yo = oracle.mlp_forward(p.astype(np.float64), x, bf16=True)
    ang = np.arccos(np.clip(np.sum(y * yo, 1), -1, 1))
    print("forward angle median", np.median(ang), "max", ang.max(), flush=True)
    assert np.median(ang) <= 1e-3 and ang.max() <= 1e-2
    assert np.allclose(np.linalg.norm(y, axis=1), 1, atol=1e-5)


def test_forward_ragged_batches():
    nat = _native()
    p = _rand_params(2)
    net = nat.MLP(seed=0)
    net.set_params(p)
    x = _rand_feats(2, 300)
    full = net.forward(_bf16_dev(x))
    torch.cuda.synchronize()
    for B in (1, 5, 127, 128, 129, 255):
        part = net.forward(_bf16_dev(x[:B]))
        torch.cuda.synchronize()
        assert torch.equal(part, full[:B]), B


@pytest.mark.parametrize("batch", [64, 352, 1024])
def test_gradient_matches_bfloat16_oracle(batch):
    """Whole (64) and ragged (352) chunks of the gradient column sums, and
    (1024) the weight-gradient products in four K slices."""
    nat = _native()
    p = _rand_params(3)
    x = _rand_feats(3, batch)
    rng = np.random.default_rng(3)
    t = rng.normal(size=(batch, 3))
    t = (t / np.linalg.norm(t, axis=1, keepdims=True)).astype(np.float32)
    net = nat.MLP(seed=0)
    net.set_params(p)
    loss, grad = net.loss_grad(_bf16_dev(x), torch.from_numpy(t).to(DEV))
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    lo, go = oracle.mlp_loss_grad(p.astype(np.float64), x, t, bf16=True)
    assert abs(float(loss.item()) - lo) <= 1e-3 * max(1.0, abs(lo))
    off = 0
    rels = []
    for (W, b) in oracle.mlp_split(np.zeros(oracle.mlp_n_params())):
        for size in (W.size, b.size):
            a, r = g[off:off + size], go[off:off + size]
            rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            print("tensor at", off, "rel-L2", rel, "norms", np.linalg.norm(a), np.linalg.norm(r),
                  "cos", float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r) + 1e-30)), flush=True)
            rels.append(rel)
            off += size
    assert max(rels) <= 1e-2, rels


def test_adam_step_matches_oracle():
    nat = _native()
    p = _rand_params(4)
    x = _rand_feats(4, 64)
    rng = np.random.default_rng(4)
    t = rng.normal(size=(64, 3))
    t = (t / np.linalg.norm(t, axis=1, keepdims=True)).astype(np.float32)
    net = nat.MLP(seed=0)
    net.set_params(p)
    _, grad = net.loss_grad(_bf16_dev(x), torch.from_numpy(t).to(DEV))
    g = grad.cpu().numpy().astype(np.float32)
    net.train_step(_bf16_dev(x), torch.from_numpy(t).to(DEV), lr=1e-3)
    torch.cuda.synchronize()
    w = p.copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    oracle.adam_step(w, m, v, g, 1, 1e-3)
    got = net.get_params()
    assert np.max(np.abs(got - w)) <= 1e-6


def test_training_reduces_the_loss():
    nat = _native()
    rng = np.random.default_rng(5)
    # a learnable map: the target is a fixed smooth function of the input
    B = 256
    A = rng.normal(size=(112, 3))
    net = nat.MLP(seed=5)
    losses = []
    for step in range(150):
        x = oracle.round_bf16(rng.normal(0, 1, (B, 112)).astype(np.float32))
        t = x.astype(np.float64) @ A
        t = (t / np.linalg.norm(t, axis=1, keepdims=True)).astype(np.float32)
        loss = torch.empty(1, device=DEV)
        net.train_step(_bf16_dev(x), torch.from_numpy(t).to(DEV), lr=2e-3, loss=loss)
        losses.append(float(loss.item()))
    print("loss first/last", losses[:3], losses[-3:], flush=True)
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])


def test_checkpoint_round_trip_and_resume():
    nat = _native()
    rng = np.random.default_rng(6)
    data = []
    for _ in range(6):
        x = oracle.round_bf16(rng.normal(0, 1, (64, 112)).astype(np.float32))
        t = rng.normal(size=(64, 3))
        t = (t / np.linalg.norm(t, axis=1, keepdims=True)).astype(np.float32)
        data.append((_bf16_dev(x), torch.from_numpy(t).to(DEV)))
    a = nat.MLP(seed=11)
    for x, t in data:
        a.train_step(x, t, lr=1e-3)
    b = nat.MLP(seed=11)
    for x, t in data[:3]:
        b.train_step(x, t, lr=1e-3)
    b.set_calibration(0.05, 0.2)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.fdmlp")
        b.save(path)
        c = nat.MLP(seed=99, path=path)
    assert c.calibration() == pytest.approx((0.05, 0.2))
    for x, t in data[3:]:
        c.train_step(x, t, lr=1e-3)
    torch.cuda.synchronize()
    assert np.array_equal(a.get_params(), c.get_params())


@pytest.mark.parametrize("depth", [False, True])
def test_features_match_oracle(depth):
    nat = _native()
    rec = dict(scenegen.RECIPES["tiny"])
    rec["n_points"] = 2000
    rec["n_views"] = 24
    rec["arc_deg"] = 360.0
    sc = scenegen.make_scene(rec, 3)
    head = np.array([0.0, 0.0, 0.02], np.float32)
    pts = torch.from_numpy(sc.points).to(DEV)
    dm = torch.from_numpy(sc.depth).to(DEV) if depth else None
    f = nat.features(pts, torch.from_numpy(sc.cams).to(DEV), torch.from_numpy(sc.theta).to(DEV),
                     torch.from_numpy(sc.conf).to(DEV), head_centre=head, depth_maps=dm)
    torch.cuda.synchronize()
    f = f.float().cpu().numpy().astype(np.float64)
    fo = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=1,
                       depth=sc.depth if depth else None).features(sc.points, head)
    fo_q = oracle.round_bf16(fo.astype(np.float32)).astype(np.float64)
    # slot validity and view choice are exact; values within a bfloat16 step
    valid_g = f[:, 6::7]
    valid_o = fo[:, 6::7]
    assert np.array_equal(valid_g, valid_o)
    err = np.abs(f - fo_q)
    tol = 2.0 ** -7 * np.abs(fo) + 1e-5
    bad = err > tol
    print("features: max err", err.max(), "bad", bad.sum(), flush=True)
    assert bad.sum() <= 1e-4 * bad.size


def _dev_scene(sc):
    return (torch.from_numpy(sc.points).to(DEV), torch.from_numpy(sc.cams).to(DEV),
            torch.from_numpy(sc.theta).to(DEV), torch.from_numpy(sc.conf).to(DEV))


def _tiny(n=3000):
    rec = dict(scenegen.RECIPES["tiny"])
    rec["n_points"] = n
    return scenegen.make_scene(rec, 7)


KW = dict(patch=3, n_candidates=48, refine_iters=8, top_k=5)


def test_learned_with_tau_minus_infinity_is_the_plain_method():
    nat = _native()
    sc = _tiny()
    pts, cams, th, cf = _dev_scene(sc)
    ctx = nat.Context(max_points=sc.n_points)
    d0, c0 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, **KW)
    prop = torch.from_numpy(sc.gt).to(DEV)
    d1, c1 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                                 proposal=nat.FD_PROPOSAL_GIVEN, proposal_dirs=prop,
                                 fallback_cost=-math.inf, learned_iters=2, **KW)
    torch.cuda.synchronize()
    assert ctx.fallback_count() == sc.n_points
    assert torch.equal(d0, d1) and torch.equal(c0, c1)


def test_nan_proposals_all_fall_back():
    nat = _native()
    sc = _tiny()
    pts, cams, th, cf = _dev_scene(sc)
    ctx = nat.Context(max_points=sc.n_points)
    d0, c0 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, **KW)
    d1, c1 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                                 proposal=nat.FD_PROPOSAL_NAN, fallback_cost=math.inf, **KW)
    torch.cuda.synchronize()
    assert ctx.fallback_count() == sc.n_points
    assert torch.equal(d0, d1) and torch.equal(c0, c1)
    # an invalid given proposal (NaN or zero vector) falls back too
    prop = torch.from_numpy(sc.gt).to(DEV).clone()
    prop[::2] = float("nan")
    prop[1::4] = 0.0
    d2, c2 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                                 proposal=nat.FD_PROPOSAL_GIVEN, proposal_dirs=prop,
                                 fallback_cost=math.inf, **KW)
    torch.cuda.synchronize()
    n_bad = len(range(0, sc.n_points, 2)) + len(range(1, sc.n_points, 4))
    assert ctx.fallback_count() >= n_bad
    assert torch.equal(d2[::2], d0[::2]) and torch.equal(d2[1::4], d0[1::4])


@pytest.mark.parametrize("tau,depth", [(math.inf, False), (0.25, False), (0.1, False),
                                       (0.25, True)])
def test_given_proposal_parity_with_oracle(tau, depth):
    nat = _native()
    sc = _tiny(2500)
    pts, cams, th, cf = _dev_scene(sc)
    extra = dict(depth_maps=torch.from_numpy(sc.depth).to(DEV)) if depth else {}
    rng = np.random.default_rng(8)
    # ground-truth tangents perturbed by ~3 degrees: a realistic proposal
    prop = sc.gt.astype(np.float64) + rng.normal(0, 0.05, sc.gt.shape)
    prop32 = prop.astype(np.float32)
    ctx = nat.Context(max_points=sc.n_points)
    step0 = 0.05
    d, c = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                               proposal=nat.FD_PROPOSAL_GIVEN,
                               proposal_dirs=torch.from_numpy(prop32).to(DEV),
                               fallback_cost=tau, learned_iters=2, learned_step0=step0,
                               **extra, **KW)
    torch.cuda.synchronize()
    n_fb = ctx.fallback_count()
    listed, in_place = ctx.fallback_split()
    assert listed + in_place == n_fb
    d = d.cpu().numpy()
    c = c.cpu().numpy()
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth if depth else None, **KW)
    do, co, fb = orc.fuse_learned(sc.points, prop32.astype(np.float64), 2, step0, tau)
    res = compare(orc, sc.points, d, c, do, co)
    print("learned tau", tau, "depth", depth, {k: v for k, v in res.items() if not k.endswith("_idx")},
          "fallbacks gpu", n_fb, f"({listed} listed, {in_place} in place)", "oracle",
          int(fb.sum()), flush=True)
    assert_parity(res)
    # the fallback decision is a threshold on a float cost: equal up to the
    # points whose refined cost lies within rounding of tau
    assert abs(n_fb - int(fb.sum())) <= max(3, 0.002 * sc.n_points)


def test_trained_network_gains_over_the_method_without_it():
    """The committed checkpoint on a scene it has neither been trained nor
    calibrated on (realistic recipe, seed 1200, depth test on): its proposals lie closer to the plain result than
    an untrained network's, more of its refined results are kept below the
    calibrated threshold, and the kept results stay within the error budget
    of the calibration.  Without the network (NaN proposals) every point
    takes the full search."""
    import os
    nat = _native()
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2604_05794_amd", "weights", "proposal_mlp.fdmlp")
    rec = dict(scenegen.RECIPES["realistic"])
    rec["n_points"] = 100_000
    sc = scenegen.make_scene(rec, 1200)
    pts, cams, th, cf = _dev_scene(sc)
    dm = torch.from_numpy(sc.depth).to(DEV)
    kw = dict(patch=5, n_candidates=128, refine_iters=8, top_k=5, depth_maps=dm)
    ctx = nat.Context(max_points=sc.n_points)
    dp, cp = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, **kw)
    fin = torch.isfinite(cp)
    feats = nat.features(pts, cams, th, cf, head_centre=sc.head_centre, depth_maps=dm)
    trained = nat.MLP(path=path)
    untrained = nat.MLP(seed=11)
    step0, tau = trained.calibration()

    def axial(a, b):
        return torch.rad2deg(torch.atan2(torch.linalg.norm(torch.cross(a, b, dim=1), dim=1),
                                         torch.abs((a * b).sum(1))))

    stats = {}
    for name, net in (("trained", trained), ("untrained", untrained)):
        prop = net.forward(feats)
        d, c = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                                   mlp=net, learned_iters=2, learned_step0=step0,
                                   fallback_cost=tau, head_centre=sc.head_centre, **kw)
        torch.cuda.synchronize()
        kept = 1.0 - ctx.fallback_count() / sc.n_points
        stats[name] = dict(proposal_median_deg=float(axial(prop[fin], dp[fin]).median()),
                           kept=kept, mean_err_vs_plain_deg=float(axial(d[fin], dp[fin]).mean()))
    d0, c0 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                                 proposal=nat.FD_PROPOSAL_NAN, fallback_cost=tau, **kw)
    torch.cuda.synchronize()
    assert ctx.fallback_count() == sc.n_points
    print("network gain", stats, flush=True)
    t, u = stats["trained"], stats["untrained"]
    assert t["proposal_median_deg"] < 0.6 * u["proposal_median_deg"]
    assert t["kept"] > u["kept"] + 0.02
    assert t["mean_err_vs_plain_deg"] <= 2.0


def test_network_against_a_fibonacci_proposal_at_equal_budget():
    """What the trained network gains over the method without it at equal
    refinement budget: on a scene neither trained nor calibrated on
    (realistic recipe, seed 1200, depth test), the network proposal and a
    proposal from a 16-direction Fibonacci lattice (the plain search with
    16 candidates and no refinement, which takes about as long as the
    network's features and forward pass) are each refined by the same 2
    iterations from the same step and held to the same threshold.  Measured
    (bench.py --workload gains): the two keep the same share of points
    within a few percent and both stay within the calibrated error budget;
    the network gains nothing here that a small lattice does not.  The test
    holds that finding: both forms within budget, kept shares within 5
    percentage points of each other."""
    import os
    nat = _native()
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2604_05794_amd", "weights", "proposal_mlp.fdmlp")
    rec = dict(scenegen.RECIPES["realistic"])
    rec["n_points"] = 100_000
    sc = scenegen.make_scene(rec, 1200)
    pts, cams, th, cf = _dev_scene(sc)
    dm = torch.from_numpy(sc.depth).to(DEV)
    kw = dict(patch=5, n_candidates=128, refine_iters=8, top_k=5, depth_maps=dm)
    ctx = nat.Context(max_points=sc.n_points)
    dp, cp = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, **kw)
    fin = torch.isfinite(cp)
    net = nat.MLP(path=path)
    step0, tau = net.calibration()

    def axial(a, b):
        return torch.rad2deg(torch.atan2(torch.linalg.norm(torch.cross(a, b, dim=1), dim=1),
                                         torch.abs((a * b).sum(1))))

    d, _ = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED, mlp=net,
                               learned_iters=2, learned_step0=step0, fallback_cost=tau,
                               head_centre=sc.head_centre, **kw)
    torch.cuda.synchronize()
    kept_net = 1.0 - ctx.fallback_count() / sc.n_points
    err_net = float(axial(d[fin], dp[fin]).mean())
    dq, _ = nat.fuse_directions(pts, cams, th, cf, ctx=ctx,
                                **dict(kw, n_candidates=16, refine_iters=0))
    d2, _ = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, mode=nat.FD_MODE_LEARNED,
                                proposal=nat.FD_PROPOSAL_GIVEN, proposal_dirs=dq,
                                learned_iters=2, learned_step0=step0, fallback_cost=tau, **kw)
    torch.cuda.synchronize()
    kept_fib = 1.0 - ctx.fallback_count() / sc.n_points
    err_fib = float(axial(d2[fin], dp[fin]).mean())
    print(f"network: kept {kept_net:.4f}, mean angle to plain {err_net:.3f} deg; "
          f"16-direction lattice: kept {kept_fib:.4f}, {err_fib:.3f} deg", flush=True)
    assert err_net <= 2.0 and err_fib <= 2.0
    assert kept_net > 0.02 and kept_fib > 0.02
    assert abs(kept_net - kept_fib) <= 0.05


@pytest.mark.parametrize("views", [64, 136])
def test_features_inside_the_learned_search_equal_the_features_entry_point(views):
    """With the network, the learned form makes the feature rows inside its
    view selection (two kernels for scenes of at most 128 views, one pass
    above that) and in processing order.  Handed instead the network's
    proposals for the rows of the standalone features entry point (one
    pass, point order), it must give the same bits, per scene and
    batched: the rows are the same whichever kernels make them."""
    nat = _native()
    rec = dict(scenegen.RECIPES["realistic"])
    rec.update(n_points=8000, n_strands=800, n_views=views, res=256)
    sc = scenegen.make_scene(rec, 21)
    net = nat.MLP(path=os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                    "paper_2604_05794_amd", "weights", "proposal_mlp.fdmlp"))
    step0, tau = net.calibration()
    pts, cams, th, cf = _dev_scene(sc)
    dm = torch.from_numpy(sc.depth).to(DEV)
    kw = dict(patch=5, n_candidates=64, refine_iters=8, top_k=5)
    lk = dict(mode=nat.FD_MODE_LEARNED, learned_iters=2, learned_step0=step0,
              fallback_cost=tau)
    ctx = nat.Context(max_points=sc.n_points)
    d1, c1 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, depth_maps=dm,
                                 head_centre=sc.head_centre, mlp=net, **lk, **kw)
    prop = net.forward(nat.features(pts, cams, th, cf, head_centre=sc.head_centre,
                                    depth_maps=dm))
    d2, c2 = nat.fuse_directions(pts, cams, th, cf, ctx=ctx, depth_maps=dm,
                                 head_centre=sc.head_centre, proposal=nat.FD_PROPOSAL_GIVEN,
                                 proposal_dirs=prop, **lk, **kw)
    torch.cuda.synchronize()
    kept = int((~(torch.all(d1 == nat.fuse_directions(
        pts, cams, th, cf, ctx=ctx, depth_maps=dm, **kw)[0], dim=1))).sum())
    print(f"{views} views: {sc.n_points} points, {kept} not equal to the plain result",
          flush=True)
    assert torch.equal(d1, d2) and torch.equal(c1, c2)
    scene = dict(points=pts, cams=cams, orient_maps=th, conf_maps=cf, depth_maps=dm,
                 head_centre=sc.head_centre, dirs=torch.empty_like(d1),
                 costs=torch.empty_like(c1))
    bctx = nat.Context(max_points=sc.n_points, max_views=sc.n_views, max_scenes=1)
    nat.fuse_batched([scene], bctx, mlp=net, **lk, **kw)
    torch.cuda.synchronize()
    assert torch.equal(scene["dirs"], d1) and torch.equal(scene["costs"], c1)
