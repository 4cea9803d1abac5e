"""Batched persistent launch (fd_fuse_directions_batched): bit-identical to
per-scene calls, graph replay, autotuned shapes, learned form."""
import math
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
import scenegen
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
KW = dict(patch=3, n_candidates=48, refine_iters=6, top_k=5)


def _native():
    from paper_2604_05794_amd import native
    native.lib()
    return native


def _uneven_scenes(dtype=np.float16):
    """Uneven point counts, view counts and map sizes (one empty scene)."""
    out = []
    specs = [(1500, 10, 96, 0), (0, 6, 64, 1), (4097, 16, 128, 2), (333, 7, 80, 3),
             (2600, 12, 112, 4)]
    for n, V, res, seed in specs:
        rec = dict(scenegen.RECIPES["tiny"])
        rec.update(n_points=max(n, 1), n_views=V, res=res, arc_deg=300.0, n_strands=120,
                   dtype="f16" if dtype == np.float16 else "f32", outliers=0.1)
        sc = scenegen.make_scene(rec, 50 + seed)
        if n == 0:
            sc.points = sc.points[:0]
            sc.gt = sc.gt[:0]
        out.append(sc)
    return out


def _dev_scene(sc, depth=False):
    n = sc.n_points
    d = dict(points=torch.from_numpy(np.ascontiguousarray(sc.points)).to(DEV),
             cams=torch.from_numpy(sc.cams).to(DEV),
             orient_maps=torch.from_numpy(sc.theta).to(DEV),
             conf_maps=torch.from_numpy(sc.conf).to(DEV),
             dirs=torch.full((n, 3), 9.0, device=DEV),
             costs=torch.full((n,), 9.0, device=DEV),
             head_centre=sc.head_centre)
    if depth:
        d["depth_maps"] = torch.from_numpy(np.ascontiguousarray(sc.depth)).to(DEV)
    return d


def _single(nat, d, **kw):
    if "depth_maps" in d:
        kw = dict(kw, depth_maps=d["depth_maps"])
    return nat.fuse_directions(d["points"], d["cams"], d["orient_maps"], d["conf_maps"], **kw)


@pytest.mark.parametrize("depth", [False, True])
def test_batched_plain_is_bitwise_per_scene(depth):
    nat = _native()
    scenes = _uneven_scenes()
    # with depth: every other scene brings depth maps, the rest run without
    devs = [_dev_scene(s, depth and k % 2 == 0) for k, s in enumerate(scenes)]
    total = sum(s.n_points for s in scenes)
    ctx = nat.Context(max_points=total, max_scenes=len(scenes))
    nat.fuse_batched(devs, ctx, **KW)
    torch.cuda.synchronize()
    for d in devs:
        if d["points"].shape[0] == 0:
            continue
        d1, c1 = _single(nat, d, **KW)
        torch.cuda.synchronize()
        assert torch.equal(d1, d["dirs"]) and torch.equal(c1, d["costs"])
    # one scene against the oracle, through the batched launch
    sc, d = scenes[2], devs[2]
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth if depth else None, **KW)
    do, co = orc.fuse(sc.points)
    res = compare(orc, sc.points, d["dirs"].cpu().numpy(), d["costs"].cpu().numpy(), do, co)
    print("batched vs oracle", {k: v for k, v in res.items() if not k.endswith("_idx")})
    assert_parity(res)


def test_graph_replay_follows_new_input_values():
    nat = _native()
    scenes = _uneven_scenes()
    devs = [_dev_scene(s) for s in scenes]
    total = sum(s.n_points for s in scenes)
    ctx = nat.Context(max_points=total, max_scenes=len(scenes))
    nat.fuse_batched(devs, ctx, **KW)
    first = [d["dirs"].clone() for d in devs]
    for rep in range(3):
        # eager work between the replays, then replay over shifted points
        # (same buffers, new values)
        for d in devs:
            d["costs"].fill_(-1.0)
        devs[0]["points"].add_(0.001 if rep == 1 else 0.0)
        nat.fuse_batched(devs, ctx, **KW)
        torch.cuda.synchronize()
        d1, c1 = _single(nat, devs[0], **KW)
        torch.cuda.synchronize()
        assert torch.equal(d1, devs[0]["dirs"]) and torch.equal(c1, devs[0]["costs"])
        for k in range(2, len(devs)):
            assert torch.equal(first[k], devs[k]["dirs"])


def test_autotuned_shapes_do_not_change_results():
    nat = _native()
    scenes = _uneven_scenes()
    devs = [_dev_scene(s) for s in scenes]
    total = sum(s.n_points for s in scenes)
    ctx = nat.Context(max_points=total, max_scenes=len(scenes))
    nat.fuse_batched(devs, ctx, **KW)
    torch.cuda.synchronize()
    ref = [d["dirs"].clone() for d in devs]
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.json")
        nat.autotune(devs, ctx, cache_path=path, **KW)
        txt = open(path).read()
        import json
        cache = json.loads(txt)
        assert len(cache) == 1
        (key, val), = cache.items()
        assert val["chunk"] >= 1 and (val["grid"] >= 1 or val["grid"] == -1)
        ctx2 = nat.Context(max_points=total, max_scenes=len(scenes))
        nat.autotune(devs, ctx2, cache_path=path, **KW)   # read from the cache
        nat.fuse_batched(devs, ctx2, **KW)
        torch.cuda.synchronize()
        for r, d in zip(ref, devs):
            assert torch.equal(r, d["dirs"])


@pytest.mark.parametrize("depth", [False, True])
def test_batched_learned_is_bitwise_per_scene(depth):
    nat = _native()
    scenes = _uneven_scenes()
    devs = [_dev_scene(s, depth and k % 2 == 0) for k, s in enumerate(scenes)]
    total = sum(s.n_points for s in scenes)
    ctx = nat.Context(max_points=total, max_scenes=len(scenes))
    net = nat.MLP(seed=3)
    kw = dict(KW, mode=nat.FD_MODE_LEARNED, mlp=net, learned_iters=2, learned_step0=0.05,
              fallback_cost=0.3)
    nat.fuse_batched(devs, ctx, **kw)
    torch.cuda.synchronize()
    for d in devs:
        if d["points"].shape[0] == 0:
            continue
        d1, c1 = _single(nat, d, head_centre=d["head_centre"], **kw)
        torch.cuda.synchronize()
        assert torch.equal(d1, d["dirs"]) and torch.equal(c1, d["costs"])


def test_batched_errors():
    nat = _native()
    scenes = _uneven_scenes()[:2]
    devs = [_dev_scene(s) for s in scenes]
    total = sum(s.n_points for s in scenes)
    small = nat.Context(max_points=10, max_scenes=2)
    with pytest.raises(nat.FdError) as e:
        nat.fuse_batched(devs, small, **KW)
    assert e.value.code == nat.FD_E_NOMEM
    no_scenes = nat.Context(max_points=total)
    with pytest.raises(nat.FdError) as e:
        nat.fuse_batched(devs, no_scenes, **KW)
    assert e.value.code == nat.FD_E_NOMEM
    ctx = nat.Context(max_points=total, max_scenes=2)
    with pytest.raises(nat.FdError) as e:
        nat.fuse_batched(devs * 17, ctx, **KW)
    assert e.value.code == nat.FD_E_INVAL
    torch.cuda.synchronize()
    assert (devs[0]["dirs"] == 9.0).all()


def test_reserve_after_capture_and_a_shared_context():
    """A captured graph never keeps workspace pointers that a later reserve
    freed, nor another call's lattice or the learned step it was captured
    with: after each of these, the batched results still equal the per-scene
    ones."""
    nat = _native()
    scenes = _uneven_scenes()
    devs = [_dev_scene(s) for s in scenes]
    total = sum(s.n_points for s in scenes)
    ctx = nat.Context(max_points=total, max_scenes=len(scenes))

    def check(**kw):
        for d in devs:
            d["dirs"].fill_(9.0)
            d["costs"].fill_(9.0)
        nat.fuse_batched(devs, ctx, **kw)
        torch.cuda.synchronize()
        for d in devs:
            if d["points"].shape[0] == 0:
                continue
            d1, c1 = _single(nat, d, head_centre=d["head_centre"], **kw)
            torch.cuda.synchronize()
            assert torch.equal(d1, d["dirs"]) and torch.equal(c1, d["costs"])

    check(**KW)
    # the per-point buffers move: the next batched call must not replay the
    # old graph
    ctx.reserve(4 * total + 1000, max_scenes=len(scenes))
    check(**KW)
    # a single-scene call through the same context with another lattice
    d = devs[2]
    nat.fuse_directions(d["points"], d["cams"], d["orient_maps"], d["conf_maps"], ctx=ctx,
                        **dict(KW, n_candidates=128))
    check(**KW)
    # the learned form's first step from the network's calibration
    net = nat.MLP(seed=5)
    kw = dict(KW, mode=nat.FD_MODE_LEARNED, mlp=net, learned_iters=2, fallback_cost=0.3)
    net.set_calibration(0.05, 0.3)
    check(**kw)
    net.set_calibration(0.2, 0.3)
    check(**kw)
