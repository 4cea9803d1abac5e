"""Pins of the oracle's learned-proposal parts: network, optimiser, features,
and the learned search with its fallback to the plain search."""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for (W, b) in oracle.mlp_split(np.zeros(oracle.mlp_n_params())):
        k = W.shape[0]
        parts.append(rng.normal(0, scale / math.sqrt(k), W.size))
        parts.append(rng.normal(0, 0.1, b.size))
    return np.concatenate(parts)


def test_parameter_count():
    assert oracle.mlp_n_params() == 112 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 3 + 3


def test_gelu_known_value_through_a_single_path():
    """Route one input through one unit per layer: the output direction and
    its scale follow the tanh-form GELU, gelu(1) = 0.8411919906."""
    p = np.zeros(oracle.mlp_n_params())
    layers = oracle.mlp_split(p)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = layers
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    W3[0, 0] = 1.0
    W4[0, 0] = 1.0
    b4[1] = 0.5
    x = np.zeros((1, 112), np.float32)
    x[0, 0] = 1.0
    y = oracle.mlp_forward(p, x)[0]
    g = 0.8411919906082768
    g2 = 0.5 * g * (1 + math.tanh(math.sqrt(2 / math.pi) * (g + 0.044715 * g ** 3)))
    g3 = 0.5 * g2 * (1 + math.tanh(math.sqrt(2 / math.pi) * (g2 + 0.044715 * g2 ** 3)))
    want = np.array([g3, 0.5, 0.0]) / math.hypot(g3, 0.5)
    assert np.allclose(y, want, atol=1e-12)
    assert g == pytest.approx(0.5 * (1 + math.tanh(math.sqrt(2 / math.pi) * 1.044715)),
                              abs=1e-12)


def test_gradient_matches_central_differences():
    params = _rand_params(1)
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, (6, 112)).astype(np.float32)
    t = rng.normal(size=(6, 3))
    t = (t / np.linalg.norm(t, axis=1, keepdims=True)).astype(np.float32)
    loss, g = oracle.mlp_loss_grad(params, x, t)
    n = len(params)
    # a spread of weights and biases from every layer
    idx = np.unique(np.concatenate([rng.integers(0, n, 60),
                                    [0, 112 * 256, 112 * 256 + 5, n - 1, n - 4, n - 10]]))
    h = 1e-6
    for i in idx:
        pp = params.copy()
        pp[i] += h
        lp, _ = oracle.mlp_loss_grad(pp, x, t)
        pp[i] -= 2 * h
        lm, _ = oracle.mlp_loss_grad(pp, x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_loss_is_axial_and_zero_at_target():
    params = _rand_params(2)
    rng = np.random.default_rng(2)
    x = rng.normal(0, 1, (5, 112)).astype(np.float32)
    y = oracle.mlp_forward(params, x)
    l1, _ = oracle.mlp_loss_grad(params, x, y.astype(np.float32))
    l2, _ = oracle.mlp_loss_grad(params, x, (-y).astype(np.float32))
    assert l1 < 1e-7 and l2 < 1e-7


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.round_bf16(x)
    assert np.array_equal(got, want)
    got_c = np.array([oracle.lib().fdo_round_bf16(float(v)) for v in x[:500]], np.float32)
    assert np.array_equal(got_c, want[:500])


def test_bf16_emulation_is_close_to_fp64():
    params = _rand_params(4)
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (64, 112)).astype(np.float32)
    y64 = oracle.mlp_forward(params, x, bf16=False)
    y16 = oracle.mlp_forward(params, x, bf16=True)
    ang = np.arccos(np.clip(np.sum(y64 * y16, 1), -1, 1))
    assert np.median(ang) < 2e-2 and ang.max() < 0.2
    assert not np.array_equal(y64, y16)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves w by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    n = 1000
    g = rng.normal(0, 1, n).astype(np.float32)
    g[:10] = 0.0
    w = rng.normal(0, 1, n).astype(np.float32)
    w0 = w.astype(np.float64).copy()
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    lr, eps = 1e-3, 1e-8
    for step in range(1, 6):
        oracle.adam_step(w, m, v, g, step, lr, eps=eps)
        want = w0 - step * lr * g.astype(np.float64) / (np.abs(g.astype(np.float64)) + eps)
        assert np.allclose(w, want, rtol=0, atol=2e-6)
    assert np.array_equal(w[:10], w0[:10].astype(np.float32))


# ---- features ---------------------------------------------------------------

def test_features_rank_frontal_views_and_describe_them():
    sc = scenegen.random_direction_field_scene(20, n_points=30, n_views=12, res=64,
                                               arc_deg=330.0)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=1)
    head = np.array([0.0, 0.0, -0.05], np.float32)
    S = 4
    F = o.features(sc.points, head, n_slots=S)
    assert F.shape == (30, 7 * S)
    cams = sc.cams.astype(np.float64)
    for i, p in enumerate(sc.points.astype(np.float64)):
        # brute force ranking on the float64 scores (well separated here)
        sc_v = []
        for v in range(len(cams)):
            R = cams[v, 4:13].reshape(3, 3)
            t = cams[v, 13:16]
            Xc = R @ p + t
            if Xc[2] <= 1e-3:
                continue
            u = cams[v, 0] * Xc[0] / Xc[2] + cams[v, 2]
            w = cams[v, 1] * Xc[1] / Xc[2] + cams[v, 3]
            if not (0 <= u <= 63 and 0 <= w <= 63):
                continue
            c = -R.T @ t
            a = c - p
            b = p - head
            sc_v.append((-(a @ b) / np.linalg.norm(a), v, a / np.linalg.norm(a), (u, w)))
        sc_v.sort()
        for j in range(S):
            f = F[i, 7 * j:7 * j + 7]
            if j >= len(sc_v):
                assert not f.any()
                continue
            _, v, vd, (u, w) = sc_v[j]
            assert f[6] == 1.0
            assert np.allclose(f[3:6], vd, atol=1e-6)
            s = oracle.sample(sc.theta[v], sc.conf[v], u, w)
            assert f[2] == pytest.approx(s[0], abs=1e-5)
            mag = math.hypot(f[0], f[1])
            assert mag <= f[2] + 1e-12
            if not s[2]:
                assert mag == 0.0


def _plane_normal(f):
    """Normal of the plane a feature slot describes: line of sight v and the
    direction at angle psi across it (frame e1 = z x v, e2 = v x e1)."""
    v = np.asarray(f[3:6], np.float64)
    e1 = np.cross([0.0, 0.0, 1.0], v)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(v, e1)
    psi = 0.5 * math.atan2(f[1], f[0])
    t = math.cos(psi) * e1 + math.sin(psi) * e2
    n = np.cross(v, t)
    return n / np.linalg.norm(n)


def test_feature_planes_contain_the_true_direction():
    """On a noise-free straight strand every observed slot describes a plane
    through the line of sight that contains the strand direction."""
    sc = scenegen.straight_strand_scene(seed=21, n_points=30, n_views=24, res=256,
                                        arc_deg=330.0)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=1)
    F = o.features(sc.points, np.zeros(3, np.float32), n_slots=16)
    checked = 0
    for i in range(len(sc.points)):
        d = sc.gt[i].astype(np.float64)
        for j in range(16):
            f = F[i, 7 * j:7 * j + 7]
            if f[6] == 0 or math.hypot(f[0], f[1]) < 0.05:
                continue
            assert abs(_plane_normal(f) @ d) < 1e-4
            checked += 1
    assert checked >= 60
    # and a wrong direction is not in those planes
    rng = np.random.default_rng(21)
    far = 0
    for i in range(5):
        q = rng.normal(size=3)
        q /= np.linalg.norm(q)
        for j in range(16):
            f = F[i, 7 * j:7 * j + 7]
            if f[6] and math.hypot(f[0], f[1]) >= 0.05:
                far += abs(_plane_normal(f) @ q) > 1e-2
    assert far > 0


# ---- learned search and fallback --------------------------------------------

def _tiny_scene():
    r = dict(scenegen.RECIPES["tiny"])
    r["n_points"] = 300
    return scenegen.make_scene(r, 0)


def test_learned_with_tau_minus_infinity_is_the_plain_method():
    sc = _tiny_scene()
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=8)
    d, c = o.fuse(sc.points)
    rng = np.random.default_rng(0)
    prop = rng.normal(size=(len(sc.points), 3))
    dl, cl, fb = o.fuse_learned(sc.points, prop, 2, 0.05, -math.inf)
    assert fb.all()
    assert np.array_equal(d, dl) and np.array_equal(c, cl)


def test_nan_proposals_always_fall_back():
    sc = _tiny_scene()
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=8)
    d, c = o.fuse(sc.points)
    prop = np.full((len(sc.points), 3), np.nan)
    prop[::3] = 0.0
    dl, cl, fb = o.fuse_learned(sc.points, prop, 2, 0.05, math.inf)
    assert fb.all()
    assert np.array_equal(d, dl) and np.array_equal(c, cl)


def test_ground_truth_proposal_is_no_worse_than_the_plain_search():
    sc = _tiny_scene()
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=8)
    d, c = o.fuse(sc.points)
    dl, cl, fb = o.fuse_learned(sc.points, sc.gt.astype(np.float64), 2, 0.05, math.inf)
    fin = np.isfinite(c)
    assert not fb[fin].any()
    gt = sc.gt[fin].astype(np.float64)

    def err(a):
        return np.arctan2(np.linalg.norm(np.cross(a, gt), axis=1), np.abs(np.sum(a * gt, 1)))

    assert err(dl[fin]).mean() <= err(d[fin]).mean()
    # tau = +inf keeps every refined proposal; a finite tau sends the worse
    # ones to the plain search and never keeps a cost above it
    tau = float(np.median(cl[fin]))
    dl2, cl2, fb2 = o.fuse_learned(sc.points, sc.gt.astype(np.float64), 2, 0.05, tau)
    keep = fin & (fb2 == 0)
    assert (cl2[keep] <= tau).all()
    assert np.array_equal(dl2[fin & (fb2 == 1)], d[fin & (fb2 == 1)])
