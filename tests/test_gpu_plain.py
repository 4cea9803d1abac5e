"""GPU parity of the plain fusion path (fd_fuse_directions, FD_MODE_PLAIN)
against the CPU oracle, through the C ABI."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from parity import assert_parity, axial_angle, compare

pytestmark = pytest.mark.gpu


def _native():
    from paper_2604_05794_amd import native
    native.lib()
    return native


def _dev(sc):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(sc.points)).to(dev),
            torch.from_numpy(np.ascontiguousarray(sc.cams)).to(dev),
            torch.from_numpy(np.ascontiguousarray(sc.theta)).to(dev),
            torch.from_numpy(np.ascontiguousarray(sc.conf)).to(dev))


def _gpu_fuse(sc, depth=False, **kw):
    nat = _native()
    pts, cams, th, cf = _dev(sc)
    if depth:
        kw["depth_maps"] = torch.from_numpy(np.ascontiguousarray(sc.depth)).to(th.device)
    d, c = nat.fuse_directions(pts, cams, th, cf, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), c.cpu().numpy()


def _log(tag, res):
    print(tag, {k: v for k, v in res.items() if not k.endswith("_idx")}, flush=True)


_cache = {}


def _scene(name, seed=0):
    key = (name, seed)
    if key not in _cache:
        _cache[key] = scenegen.make_scene(name, seed)
    return _cache[key]


@pytest.mark.parametrize("depth", [False, True])
def test_tiny_workload_all_points(depth):
    """10k points, 200 helices, 12 views at 256^2 float32, P = 3, 48
    candidates; with and without the depth visibility test."""
    sc = _scene("tiny")
    kw = dict(patch=3, n_candidates=48, refine_iters=8, top_k=5)
    d, c = _gpu_fuse(sc, depth=depth, **kw)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth if depth else None, **kw)
    do, co = orc.fuse(sc.points)
    res = compare(orc, sc.points, d, c, do, co)
    _log(f"tiny depth={depth}", res)
    assert_parity(res)


@pytest.mark.parametrize("depth", [True, False])
def test_realistic_workload_sampled_points(depth):
    """500k points, 64 views at 1024^2 float16 (binary16 depth maps), P = 5,
    128 candidates + 8 iterations: the full launch on the GPU, every 97th
    point by the oracle."""
    sc = _scene("realistic")
    kw = dict(patch=5, n_candidates=128, refine_iters=8, top_k=5)
    d, c = _gpu_fuse(sc, depth=depth, **kw)
    idx = np.arange(0, sc.n_points, 97)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth if depth else None, **kw)
    do, co = orc.fuse(sc.points[idx])
    res = compare(orc, sc.points[idx], d[idx], c[idx], do, co)
    _log(f"realistic depth={depth}", res)
    assert_parity(res)
    # every point of the launch: finite cost in [0, 1] with a unit direction,
    # or +inf with a zero direction
    fin = np.isfinite(c)
    assert np.all((c[fin] >= -1e-6) & (c[fin] <= 1 + 1e-6))
    assert np.allclose(np.linalg.norm(d[fin], axis=1), 1, atol=1e-5)
    assert not d[~fin].any()


@pytest.mark.parametrize("patch,top_k,n_cand,iters", [(1, 1, 16, 0), (3, 8, 64, 4),
                                                      (5, 5, 128, 8), (7, 3, 32, 12)])
def test_parameter_grid(patch, top_k, n_cand, iters):
    sc = scenegen.random_direction_field_scene(30 + patch, n_points=701, n_views=10, res=96,
                                               arc_deg=300.0, smooth=True)
    kw = dict(patch=patch, n_candidates=n_cand, refine_iters=iters, top_k=top_k)
    d, c = _gpu_fuse(sc, **kw)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, **kw)
    do, co = orc.fuse(sc.points)
    res = compare(orc, sc.points, d, c, do, co)
    _log(f"grid P{patch} K{top_k}", res)
    assert_parity(res)


def test_float16_non_square_maps():
    sc = scenegen.random_direction_field_scene(40, n_points=333, n_views=7, res=64,
                                               arc_deg=200.0, dtype=np.float16)
    # crop to a non-square image (cx, cy stay those of the 64 x 64 camera)
    sc.theta = np.ascontiguousarray(sc.theta[:, :48, :])
    sc.conf = np.ascontiguousarray(sc.conf[:, :48, :])
    kw = dict(patch=5, n_candidates=64, refine_iters=6, top_k=4)
    d, c = _gpu_fuse(sc, **kw)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, **kw)
    do, co = orc.fuse(sc.points)
    res = compare(orc, sc.points, d, c, do, co)
    _log("f16 non-square", res)
    assert_parity(res)


def _misaligned(t):
    """A copy of t whose data starts 2 bytes past a 4-byte boundary."""
    flat = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
    v = flat[1:].view(t.shape)
    v.copy_(t)
    assert v.data_ptr() % 4 == 2
    return v


def test_maps_not_4_byte_aligned_take_single_texel_loads():
    """Binary16 maps whose base is only 2-byte aligned (or of odd width)
    cannot take the paired texel loads; the results are bitwise those of
    the aligned maps, in the plain search and the proposal features."""
    nat = _native()
    rec = dict(scenegen.RECIPES["realistic"])
    rec["n_points"] = 3000
    rec["n_views"] = 16
    rec["res"] = 256
    sc = scenegen.make_scene(rec, 21)
    pts, cams, th, cf = _dev(sc)
    dm = torch.from_numpy(sc.depth).to(th.device)
    kw = dict(patch=5, n_candidates=64, refine_iters=6, top_k=5, depth_maps=dm)
    d0, c0 = nat.fuse_directions(pts, cams, th, cf, **kw)
    f0 = nat.features(pts, cams, th, cf, head_centre=sc.head_centre, depth_maps=dm)
    kw["depth_maps"] = _misaligned(dm)
    d1, c1 = nat.fuse_directions(pts, cams, _misaligned(th), _misaligned(cf), **kw)
    f1 = nat.features(pts, cams, _misaligned(th), _misaligned(cf), head_centre=sc.head_centre,
                      depth_maps=kw["depth_maps"])
    torch.cuda.synchronize()
    assert torch.equal(d0, d1) and torch.equal(c0, c1)
    assert torch.equal(f0, f1)


@pytest.mark.parametrize("n", [1, 2, 11, 12, 13, 47, 48, 49, 61])
def test_ragged_sizes(n):
    sc = _scene("tiny")
    kw = dict(patch=3, n_candidates=48, refine_iters=8, top_k=5)
    pts = sc.points[1000:1000 + n]
    sub = scenegen.Scene(pts, sc.gt[1000:1000 + n], sc.cams, sc.theta, sc.conf, None,
                         sc.head_centre, {})
    d, c = _gpu_fuse(sub, **kw)
    full_d, full_c = _gpu_fuse(sc, **kw)
    # each point is fused independently of the others in the launch
    assert np.array_equal(d, full_d[1000:1000 + n]) and np.array_equal(c, full_c[1000:1000 + n])


def test_empty_input_is_a_no_op():
    nat = _native()
    sc = _scene("tiny")
    pts, cams, th, cf = _dev(sc)
    d, c = nat.fuse_directions(pts[:0], cams, th, cf, patch=3, n_candidates=48)
    torch.cuda.synchronize()
    assert d.shape == (0, 3) and c.shape == (0,)


def test_points_without_views_get_infinite_cost():
    sc = _scene("tiny")
    pts = sc.points[:64].copy()
    pts[::2] = np.array([50.0, 50.0, 50.0], np.float32)       # outside every image
    pts[1::4] = np.array([0.6, 0.0, 0.16], np.float32)         # at a camera centre
    sub = scenegen.Scene(pts, sc.gt[:64], sc.cams, sc.theta, sc.conf, None, sc.head_centre, {})
    kw = dict(patch=3, n_candidates=48, refine_iters=8, top_k=5)
    d, c = _gpu_fuse(sub, **kw)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, **kw)
    do, co = orc.fuse(pts)
    assert np.array_equal(np.isinf(c), np.isinf(co))
    assert np.isinf(c[::2]).all() and not d[::2].any()
    # zero confidence everywhere: nothing is eligible
    zero = np.zeros_like(sc.conf)
    sub2 = scenegen.Scene(sc.points[:100], sc.gt[:100], sc.cams, sc.theta, zero, None,
                          sc.head_centre, {})
    d2, c2 = _gpu_fuse(sub2, **kw)
    assert np.isinf(c2).all() and not d2.any()


def test_permutation_equivariance_and_determinism():
    sc = _scene("tiny")
    kw = dict(patch=3, n_candidates=48, refine_iters=8, top_k=5)
    d1, c1 = _gpu_fuse(sc, **kw)
    d1b, c1b = _gpu_fuse(sc, **kw)
    assert np.array_equal(d1, d1b) and np.array_equal(c1, c1b)
    perm = np.random.default_rng(0).permutation(sc.n_points)
    sub = scenegen.Scene(sc.points[perm], sc.gt[perm], sc.cams, sc.theta, sc.conf, None,
                         sc.head_centre, {})
    d2, c2 = _gpu_fuse(sub, **kw)
    assert np.array_equal(d1[perm], d2) and np.array_equal(c1[perm], c2)


def test_invalid_arguments_are_rejected_before_launch():
    nat = _native()
    sc = _scene("tiny")
    pts, cams, th, cf = _dev(sc)
    d = torch.full((sc.n_points, 3), 7.0, device=pts.device)
    c = torch.full((sc.n_points,), 7.0, device=pts.device)
    for bad in (dict(patch=4), dict(patch=9), dict(top_k=0), dict(top_k=9), dict(top_k=13),
                dict(n_candidates=0), dict(refine_iters=-1), dict(refine_iters=99),
                dict(mode=7), dict(z_near=-1.0)):
        kw = dict(patch=3, n_candidates=48)
        kw.update(bad)
        with pytest.raises(nat.FdError) as e:
            nat.fuse_directions(pts, cams, th, cf, dirs=d, costs=c, **kw)
        assert e.value.code == nat.FD_E_INVAL, bad
    torch.cuda.synchronize()
    assert (d == 7.0).all() and (c == 7.0).all()
    ctx = nat.Context(max_points=100)
    with pytest.raises(nat.FdError) as e:
        nat.fuse_directions(pts, cams, th, cf, dirs=d, costs=c, ctx=ctx, patch=3,
                            n_candidates=48)
    assert e.value.code == nat.FD_E_NOMEM
    torch.cuda.synchronize()
    assert (d == 7.0).all()


def test_explicit_context_matches_default():
    nat = _native()
    sc = _scene("tiny")
    kw = dict(patch=3, n_candidates=48, refine_iters=8, top_k=5)
    d1, c1 = _gpu_fuse(sc, **kw)
    ctx = nat.Context(max_points=sc.n_points)
    d2, c2 = _gpu_fuse(sc, ctx=ctx, **kw)
    assert np.array_equal(d1, d2) and np.array_equal(c1, c2)
