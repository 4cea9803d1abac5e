"""GPU parity of the paper-literal candidate mode (FD_MODE_FPMVO: Sec.
3.1.1-3.1.2, Eqs. 1-7, scored by Eq. 12) against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
FP = dict(lam=3.0, n_samples=5, delta=5e-3)


def _native():
    from paper_2604_05794_amd import native
    native.lib()
    return native


def _gpu(sc, **kw):
    nat = _native()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    d, c = nat.fuse_directions(t(sc.points), t(sc.cams), t(sc.theta), t(sc.conf),
                               depth_maps=t(sc.depth), mode=nat.FD_MODE_FPMVO,
                               fpmvo_lambda=FP["lam"], fpmvo_samples=FP["n_samples"],
                               fpmvo_delta=FP["delta"], **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), c.cpu().numpy()


def _check(tag, sc, idx, kw):
    d, c = _gpu(sc, **kw)
    orc = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth, **kw)
    do, co = orc.fpmvo(sc.points[idx], **FP)
    res = compare(orc, sc.points[idx], d[idx], c[idx], do, co)
    print(tag, {k: v for k, v in res.items() if not k.endswith("_idx")}, flush=True)
    assert_parity(res)
    return d, c


def test_tiny_scene_all_points():
    sc = scenegen.make_scene("tiny", 0)
    _check("fpmvo tiny", sc, np.arange(sc.n_points), dict(patch=3, top_k=5))


def test_realistic_scene_sampled_points():
    sc = scenegen.make_scene("realistic", 0)
    d, c = _check("fpmvo realistic", sc, np.arange(0, sc.n_points, 97), dict(patch=5, top_k=5))
    fin = np.isfinite(c)
    assert fin.mean() > 0.99
    assert np.allclose(np.linalg.norm(d[fin], axis=1), 1, atol=1e-5)
    assert not d[~fin].any()


def test_isolated_strands_match_the_oracle():
    for seed in range(4):
        sc = scenegen.straight_strand_scene(seed, n_points=40, n_views=8, res=256,
                                            arc_deg=120.0)
        _check(f"fpmvo strand {seed}", sc, np.arange(sc.n_points), dict(patch=3, top_k=5))


@pytest.mark.parametrize("n", [1, 13, 61])
def test_ragged_sizes_equal_the_full_launch(n):
    sc = scenegen.make_scene("tiny", 0)
    kw = dict(patch=3, top_k=5)
    full_d, full_c = _gpu(sc, **kw)
    sub = scenegen.Scene(sc.points[500:500 + n], sc.gt[500:500 + n], sc.cams, sc.theta, sc.conf,
                         sc.depth, sc.head_centre, {})
    d, c = _gpu(sub, **kw)
    assert np.array_equal(d, full_d[500:500 + n]) and np.array_equal(c, full_c[500:500 + n])


def test_invalid_arguments():
    nat = _native()
    sc = scenegen.make_scene("tiny", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    pts, cams, th, cf, dm = t(sc.points), t(sc.cams), t(sc.theta), t(sc.conf), t(sc.depth)
    with pytest.raises(nat.FdError) as e:   # no depth maps
        nat.fuse_directions(pts, cams, th, cf, mode=nat.FD_MODE_FPMVO)
    assert e.value.code == nat.FD_E_INVAL
    for bad in (dict(fpmvo_samples=0), dict(fpmvo_samples=17), dict(fpmvo_lambda=0.0),
                dict(fpmvo_delta=-1.0), dict(fpmvo_lambda=float("nan"))):
        with pytest.raises(nat.FdError) as e:
            nat.fuse_directions(pts, cams, th, cf, depth_maps=dm, mode=nat.FD_MODE_FPMVO, **bad)
        assert e.value.code == nat.FD_E_INVAL
    ctx = nat.Context(max_points=sc.n_points, max_scenes=1)
    scene = dict(points=pts, cams=cams, orient_maps=th, conf_maps=cf, depth_maps=dm,
                 dirs=torch.empty((sc.n_points, 3), device=DEV),
                 costs=torch.empty((sc.n_points,), device=DEV))
    with pytest.raises(nat.FdError) as e:
        nat.fuse_batched([scene], ctx, mode=nat.FD_MODE_FPMVO)
    assert e.value.code == nat.FD_E_INVAL
