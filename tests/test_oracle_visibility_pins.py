"""Pins of the oracle's visibility test (Sec. 3.1.1, the score V_i^v): a view
takes part for a point only when the point's camera-space depth agrees with
the rendered depth at its projection.

The pins reduce the test to cases with a known answer: a view whose depth
map hides the point behaves exactly as if the camera were not there; depth
equal to the point's own depth changes nothing; the tolerance and the
nearest-texel rule switch visibility where they say; and on generated
scenes the oracle's count of visible views agrees with the scene
generator's own visibility count (a separate implementation in double
precision).
"""
import math

import numpy as np
import pytest

import oracle
import scenegen


def _z64(cam, p):
    cam = np.asarray(cam, np.float64)
    return float(cam[10:13] @ np.asarray(p, np.float64) + cam[15])


def _u64(cam, p):
    cam = np.asarray(cam, np.float64)
    R = cam[4:13].reshape(3, 3)
    X = R @ np.asarray(p, np.float64) + cam[13:16]
    return np.array([cam[0] * X[0] / X[2] + cam[2], cam[1] * X[1] / X[2] + cam[3]])


def _depth_for(cams, p, shape, visible):
    """Constant depth map per view: the point's own depth where `visible`,
    an occluder 5 cm in front of it elsewhere."""
    V, H, W = shape
    d = np.empty((V, H, W), np.float32)
    for v in range(V):
        z = _z64(cams[v], p)
        d[v] = z if visible[v] else z - 0.05
    return d


def _scene(V=9, W=48, H=40, seed=0):
    rng = np.random.default_rng(seed)
    cams = scenegen.orbit_cameras(V, W, H, 200.0)
    theta = rng.uniform(0, math.pi, (V, H, W)).astype(np.float32)
    conf = rng.uniform(0.05, 1.0, (V, H, W)).astype(np.float32)
    return cams, theta, conf


def _points(n, seed):
    rng = np.random.default_rng(100 + seed)
    return rng.uniform(-0.05, 0.05, (n, 3)).astype(np.float32)


KW = dict(patch=3, n_candidates=64, refine_iters=4, top_k=5)


def test_own_depth_changes_nothing():
    cams, theta, conf = _scene()
    o0 = oracle.Oracle(cams, theta, conf, **KW)
    for i, p in enumerate(_points(12, 0)):
        dep = _depth_for(cams, p, theta.shape, [True] * len(cams))
        o1 = oracle.Oracle(cams, theta, conf, depth=dep, **KW)
        ids0, u0 = o0.select_views(p)
        ids1, u1 = o1.select_views(p)
        assert list(ids0) == list(ids1) and np.array_equal(u0, u1)
        d0, c0 = o0.fuse(p[None])
        d1, c1 = o1.fuse(p[None])
        assert np.array_equal(d0, d1) and np.array_equal(c0, c1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hidden_views_act_as_absent_cameras(seed):
    cams, theta, conf = _scene(seed=seed)
    V = len(cams)
    rng = np.random.default_rng(seed)
    for p in _points(6, seed):
        vis = rng.uniform(size=V) < 0.55
        vis[rng.integers(V)] = True
        keep = np.flatnonzero(vis)
        dep = _depth_for(cams, p, theta.shape, vis)
        o1 = oracle.Oracle(cams, theta, conf, depth=dep, **KW)
        sub = oracle.Oracle(cams[keep], theta[keep], conf[keep], **KW)
        ids1, u1 = o1.select_views(p)
        ids2, u2 = sub.select_views(p)
        assert list(ids1) == [int(keep[j]) for j in ids2]
        assert np.array_equal(u1, u2)
        d1, c1 = o1.fuse(p[None])
        d2, c2 = sub.fuse(p[None])
        assert np.array_equal(d1, d2) and np.array_equal(c1, c2)
        # the objective at any direction likewise
        dd = np.array([0.3, -0.5, 0.81])
        assert o1.objective(p, dd) == sub.objective(p, dd)
        # proposal features: the frontal slots only ever hold visible views
        hc = np.zeros(3, np.float32)
        f1 = o1.features(p[None], hc)
        f2 = sub.features(p[None], hc)
        assert np.array_equal(f1, f2)


def test_no_visible_view_gives_no_result():
    cams, theta, conf = _scene()
    p = _points(1, 3)[0]
    dep = _depth_for(cams, p, theta.shape, [False] * len(cams))
    o = oracle.Oracle(cams, theta, conf, depth=dep, **KW)
    ids, _ = o.select_views(p)
    assert len(ids) == 0
    d, c = o.fuse(p[None])
    assert c[0] == math.inf and not d.any()
    assert not o.features(p[None], np.zeros(3, np.float32)).any()


def test_tolerance_and_background():
    cams, theta, conf = _scene(V=3)
    p = _points(1, 4)[0]
    tau = 4e-3
    o_ref = oracle.Oracle(cams, theta, conf, **KW)
    full, _ = o_ref.select_views(p)
    assert len(full) == 3
    for off, want in [(0.0, True), (0.9 * tau, True), (-0.9 * tau, True), (1.1 * tau, False),
                      (-1.1 * tau, False), (math.inf, False), (math.nan, False)]:
        dep = np.empty(theta.shape, np.float32)
        for v in range(3):
            dep[v] = _z64(cams[v], p) + (off if v == 1 else 0.0)
        o = oracle.Oracle(cams, theta, conf, depth=dep, vis_tau=tau, **KW)
        ids, _ = o.select_views(p)
        assert (1 in ids) == want, (off, ids)
        assert len(ids) == (3 if want else 2)


def test_nearest_texel_rule():
    """A depth step between columns c and c+1: a point is visible while its
    projection rounds to column c and hidden once it rounds to c+1."""
    W, H = 64, 48
    cams = scenegen.orbit_cameras(1, W, H, 360.0)
    cam = cams[0]
    theta = np.zeros((1, H, W), np.float32)
    conf = np.ones((1, H, W), np.float32)
    R = cam[4:13].reshape(3, 3).astype(np.float64)
    p0 = np.array([0.0, 0.0, 0.0])
    u0 = _u64(cam, p0)
    z0 = _z64(cam, p0)
    c = int(math.floor(u0[0])) + 3
    dep = np.full((1, H, W), z0, np.float32)
    dep[0, :, c + 1:] = z0 - 0.05
    o = oracle.Oracle(cams, theta, conf, depth=dep, **KW)
    # moving along the camera's x axis keeps Z, and moves u by fx * dx / Z
    for frac, want in [(0.30, True), (0.45, True), (0.55, False), (0.80, False),
                       (-0.45, True)]:
        dx = (c + frac - u0[0]) * z0 / cam[0]
        p = (p0 + dx * R[0]).astype(np.float32)
        u = _u64(cam, p)
        assert abs(u[0] - (c + frac)) < 1e-3
        ids, _ = o.select_views(p)
        assert (len(ids) == 1) == want, (frac, u)


def test_visible_count_agrees_with_the_generator():
    """The scene generator keeps its own visibility count (double precision,
    separate code); the oracle's eligible-view count with uniform confidence
    and K = V must match it except where rounding sits on a boundary."""
    rec = dict(scenegen.RECIPES["tiny"])
    rec.update(n_points=600, n_views=8, res=160, arc_deg=360.0, kappa=None, outliers=0.0,
               outer=False)
    sc = scenegen.make_scene(rec, 7)
    V = sc.n_views
    conf = np.ones_like(sc.conf)
    o = oracle.Oracle(sc.cams, sc.theta, conf, depth=sc.depth, top_k=8, patch=1,
                      vis_tau=scenegen.VIS_TAU)
    gen = scenegen.visible_views(sc.points, sc.cams, sc.depth, tau=scenegen.VIS_TAU)
    got = np.array([len(o.select_views(p)[0]) for p in sc.points])
    assert V == 8
    assert gen.max() > 1 and (gen == 0).any()          # both cases occur
    assert (got == gen).mean() > 0.99
