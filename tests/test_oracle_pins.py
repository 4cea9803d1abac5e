"""Pins of the CPU oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, brute force, special cases with known answers, invariances, an
independent library routine.  EfficientMonoHair Sec. 3.1, Eqs. (4), (8)-(12).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import scenegen


def _proj64(cam, x):
    """Pinhole projection in float64 straight from the 16-float record."""
    cam = np.asarray(cam, np.float64)
    R = cam[4:13].reshape(3, 3)
    t = cam[13:16]
    Xc = R @ np.asarray(x, np.float64) + t
    return np.array([cam[0] * Xc[0] / Xc[2] + cam[2], cam[1] * Xc[1] / Xc[2] + cam[3]])


def _image_angle(cam, p, d, eps=1e-4):
    """Angle of the image of the 3D line through p along d (a perspective map
    sends lines to lines, so two projected points give its direction)."""
    a = _proj64(cam, p)
    b = _proj64(cam, np.asarray(p, np.float64) + eps * np.asarray(d, np.float64))
    return math.atan2(b[1] - a[1], b[0] - a[0])


def _axial(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    c = np.cross(a, b)
    return np.arctan2(np.linalg.norm(np.atleast_2d(c), axis=-1),
                      np.abs(np.sum(np.atleast_2d(a) * np.atleast_2d(b), axis=-1)))


def _uniform_maps(cams, p, d_star, res):
    V = len(cams)
    th = np.empty((V, res, res), np.float32)
    for v in range(V):
        th[v] = np.mod(_image_angle(cams[v], p, d_star), math.pi)
    return th, np.ones((V, res, res), np.float32)


# ---- map decoding and the sampler -------------------------------------------

def test_half_to_float_matches_numpy_for_every_code():
    codes = np.arange(65536, dtype=np.uint16)
    ref = codes.view(np.float16).astype(np.float32)
    got = np.array([oracle.half_to_float(int(c)) for c in codes[::7]], np.float32)
    r = ref[::7]
    fin = np.isfinite(r)
    assert np.array_equal(got[fin], r[fin])
    assert np.array_equal(np.isnan(got), np.isnan(r))


def test_sampler_returns_texel_at_texel_centres():
    rng = np.random.default_rng(1)
    th = rng.uniform(0, math.pi, (9, 11)).astype(np.float32)
    c = rng.uniform(0.1, 1, (9, 11)).astype(np.float32)
    c[4, 5] = 0.0
    for (y, x) in [(0, 0), (3, 7), (8, 10), (4, 5), (2, 2)]:
        s = oracle.sample(th, c, x, y)
        assert s[0] == pytest.approx(float(c[y, x]), abs=1e-15)
        if c[y, x] == 0:
            assert s[2] == 0.0
        else:
            assert s[2] == 1.0
            # axial: compare doubled angles
            assert abs(math.remainder(2 * s[1] - 2 * float(th[y, x]), 2 * math.pi)) < 1e-12


def test_sampler_midpoint_is_axial_mean():
    th = np.zeros((1, 2), np.float32)
    c = np.ones((1, 2), np.float32)
    # 0.1 and pi - 0.1 are the lines at +-0.1 rad: their axial mean is 0, where a
    # plain angle average would give pi/2
    th[0] = [0.1, math.pi - 0.1]
    s = oracle.sample(th, c, 0.5, 0.0)
    assert abs(s[1]) < 1e-7 and s[2] == 1.0
    assert s[0] == pytest.approx(1.0, abs=1e-15)
    th[0] = [0.2, 0.4]
    s = oracle.sample(th, c, 0.5, 0.0)
    assert s[1] == pytest.approx(0.3, abs=1e-7)
    # confidence-weighted: C = (1, 3) pulls the mean three times harder
    c[0] = [1.0, 3.0]
    th[0] = [0.0, 0.2]
    s = oracle.sample(th, c, 0.5, 0.0)
    expect = 0.5 * math.atan2(3 * math.sin(0.4), 1 + 3 * math.cos(0.4))
    assert s[1] == pytest.approx(expect, abs=1e-7)
    assert s[0] == pytest.approx(2.0, abs=1e-15)


def test_sampler_background_does_not_move_orientation():
    th = np.zeros((3, 3), np.float32)
    c = np.zeros((3, 3), np.float32)
    th[1, 1] = 0.7
    c[1, 1] = 1.0
    th[1, 2] = 2.9   # background texel with a stray angle: C = 0, must not count
    for (x, y) in [(1.2, 1.3), (0.6, 1.0), (1.9, 0.8)]:
        s = oracle.sample(th, c, x, y)
        w = max(0, 1 - abs(x - 1)) * max(0, 1 - abs(y - 1))
        assert s[0] == pytest.approx(w, abs=1e-15)
        assert s[2] == 1.0 and s[1] == pytest.approx(0.7, abs=1e-7)
    s = oracle.sample(th, c, 2.5, 2.5)   # all four texels background / outside
    assert s[0] == 0.0 and s[2] == 0.0


# ---- Eq. (4) view selection -------------------------------------------------

def test_top_k_brute_force_and_ties():
    Wd, Ht = 40, 24       # non-square, so cx != cy
    cams = scenegen.orbit_cameras(6, Wd, Ht, 150.0)
    cams = np.concatenate([cams, cams[2:3]], 0)       # view 6 duplicates view 2
    V = len(cams)
    levels = np.array([0.3, 0.9, 0.6, 0.0, 0.75, 0.45, 0.6], np.float32)
    conf = np.broadcast_to(levels[:, None, None], (V, Ht, Wd)).copy()
    theta = np.zeros((V, Ht, Wd), np.float32)
    p = np.array([0.01, -0.02, 0.03], np.float32)
    for K in (1, 3, 5, 7):
        o = oracle.Oracle(cams, theta, conf, patch=1, top_k=K)
        ids, u = o.select_views(p)
        # brute force: eligible views (C > 0, all points in front and inside),
        # stable sort by descending confidence (ties keep the lower index)
        elig = [v for v in range(V) if levels[v] > 0]
        order = sorted(elig, key=lambda v: (-levels[v], v))
        assert list(ids) == order[:K]
        for j, v in enumerate(ids):
            assert np.allclose(u[j], _proj64(cams[v], p), atol=1e-9, rtol=0)
    # the duplicated view ties with view 2 and must come after it
    o = oracle.Oracle(cams, theta, conf, patch=1, top_k=7)
    ids, _ = o.select_views(p)
    assert list(ids).index(2) < list(ids).index(6)


def test_view_eligibility_front_and_inside():
    res = 16
    cams = scenegen.orbit_cameras(4, res, res, 360.0)
    conf = np.ones((4, res, res), np.float32)
    theta = np.zeros_like(conf)
    o = oracle.Oracle(cams, theta, conf, patch=1, top_k=4)
    # a point on the far side of the orbit's first camera, well outside the
    # field of view of the opposite camera's frustum
    ids, _ = o.select_views(np.array([0.0, 0.0, 0.0], np.float32))
    assert sorted(ids) == [0, 1, 2, 3]
    far = np.array([5.0, 0.0, 0.0], np.float32)     # behind camera 0, outside others
    ids, _ = o.select_views(far)
    for v in ids:
        u = _proj64(cams[v], far)
        R = cams[v][4:13].reshape(3, 3).astype(np.float64)
        Z = R[2] @ far + cams[v][15]
        assert Z > 0 and 0 <= u[0] <= res - 1 and 0 <= u[1] <= res - 1
    assert 0 not in ids
    J = o.objective(np.array([50.0, 50.0, 50.0], np.float32), np.array([0, 0, 1.0]))
    assert J == math.inf


# ---- objective: closed forms ------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_uniform_field_closed_form(seed):
    """Maps constant per view at the image angle of d* through p, C = 1:
    J(d*) = 0 and J(d) = 1 - mean_v |cos(phi_v(d) - phi_v(d*))| with phi from
    two-point projection (Eq. 8 with a finite offset), for every patch size."""
    rng = np.random.default_rng(seed)
    res = 64
    cams = scenegen.orbit_cameras(5, res, res, 160.0)
    p = rng.normal(0, 0.02, 3).astype(np.float32)
    d_star = rng.normal(size=3)
    d_star /= np.linalg.norm(d_star)
    th, c = _uniform_maps(cams, p, d_star, res)
    for P in (1, 3, 5):
        o = oracle.Oracle(cams, th, c, patch=P, top_k=5)
        assert o.objective(p, d_star) < 1e-12
        for _ in range(20):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            want = 1 - np.mean([abs(math.cos(_image_angle(cams[v], p, d) -
                                             _image_angle(cams[v], p, d_star)))
                                for v in range(5)])
            assert o.objective(p, d) == pytest.approx(want, abs=1e-7)


def test_two_view_triangulation():
    """P = 1, two views with constant observed image lines: the minimiser is
    the intersection of the two back-projected planes, d* = n1 x n2."""
    res = 128
    cams = scenegen.orbit_cameras(2, res, res, 80.0)
    p = np.array([0.01, 0.02, -0.01], np.float32)
    angles = [0.4, 2.1]
    th = np.stack([np.full((res, res), a, np.float32) for a in angles])
    c = np.ones((2, res, res), np.float32)
    normals = []
    for v in range(2):
        cam = cams[v].astype(np.float64)
        Kinv = np.linalg.inv(np.array([[cam[0], 0, cam[2]], [0, cam[1], cam[3]], [0, 0, 1]]))
        R = cam[4:13].reshape(3, 3)
        u = _proj64(cam, p)
        o = np.array([math.cos(angles[v]), math.sin(angles[v])])
        a = Kinv @ np.array([u[0], u[1], 1.0])
        b = Kinv @ np.array([u[0] + o[0], u[1] + o[1], 1.0])
        normals.append(R.T @ np.cross(a, b))
    d_star = np.cross(normals[0], normals[1])
    d_star /= np.linalg.norm(d_star)
    o = oracle.Oracle(cams, th, c, patch=1, n_candidates=48, refine_iters=20, top_k=2)
    assert o.objective(p, d_star) < 1e-9
    dirs, costs = o.fuse(p[None, :])
    assert _axial(dirs[0], d_star)[0] <= 1e-3
    assert costs[0] < 1e-6


def test_single_view_minimisers_lie_in_the_plane():
    res = 128
    cams = scenegen.orbit_cameras(1, res, res, 0.0)
    p = np.array([0.0, 0.01, 0.02], np.float32)
    ang = 1.1
    th = np.full((1, res, res), ang, np.float32)
    c = np.ones((1, res, res), np.float32)
    cam = cams[0].astype(np.float64)
    Kinv = np.linalg.inv(np.array([[cam[0], 0, cam[2]], [0, cam[1], cam[3]], [0, 0, 1]]))
    R = cam[4:13].reshape(3, 3)
    u = _proj64(cam, p)
    a = Kinv @ np.array([u[0], u[1], 1.0])
    b = Kinv @ np.array([u[0] + math.cos(ang), u[1] + math.sin(ang), 1.0])
    n = R.T @ np.cross(a, b)
    n /= np.linalg.norm(n)
    o = oracle.Oracle(cams, th, c, patch=1, n_candidates=48, refine_iters=16, top_k=1)
    dirs, costs = o.fuse(p[None, :])
    assert abs(float(n @ dirs[0])) <= 1e-3
    assert costs[0] < 1e-6


# ---- objective: structure of Eqs. (9)-(11) -----------------------------------

def test_patch_max_is_monotone_in_patch_size():
    sc = scenegen.random_direction_field_scene(3, n_points=12, n_views=6, res=48)
    rng = np.random.default_rng(3)
    o1, o3, o5 = (oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=P, top_k=5)
                  for P in (1, 3, 5))
    for p in sc.points:
        for _ in range(10):
            d = rng.normal(size=3)
            j1, j3, j5 = o1.objective(p, d), o3.objective(p, d), o5.objective(p, d)
            if math.isinf(j1):
                continue
            assert j5 <= j3 + 1e-15 and j3 <= j1 + 1e-15


def test_confidence_scaling_scales_consistency():
    sc = scenegen.random_direction_field_scene(4, n_points=10, n_views=6, res=48)
    half = (sc.conf * np.float32(0.5)).astype(np.float32)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, top_k=4)
    oh = oracle.Oracle(sc.cams, sc.theta, half, patch=3, top_k=4)
    rng = np.random.default_rng(4)
    for p in sc.points:
        d = rng.normal(size=3)
        J, Jh = o.objective(p, d), oh.objective(p, d)
        if math.isinf(J):
            continue
        assert (1 - Jh) == pytest.approx(0.5 * (1 - J), abs=1e-15)


def test_direction_sign_does_not_matter():
    sc = scenegen.random_direction_field_scene(5, n_points=10, n_views=6, res=48)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, top_k=5)
    rng = np.random.default_rng(5)
    for p in sc.points:
        d = rng.normal(size=3)
        J = o.objective(p, d)
        if math.isinf(J):
            continue
        assert o.objective(p, -d) == pytest.approx(J, abs=1e-14)
        assert o.objective(p, 3.7 * d) == pytest.approx(J, abs=1e-14)


def _transform_scene(cams, pts, Q, t0):
    cams2 = cams.astype(np.float64).copy()
    for v in range(len(cams)):
        R = cams[v, 4:13].reshape(3, 3).astype(np.float64)
        t = cams[v, 13:16].astype(np.float64)
        R2 = R @ Q.T
        cams2[v, 4:13] = R2.ravel()
        cams2[v, 13:16] = t - R2 @ t0
    pts2 = pts.astype(np.float64) @ Q.T + t0
    return cams2.astype(np.float32), pts2.astype(np.float32)


def _rotation(rng):
    A = rng.normal(size=(3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def _signed_permutation_rotations():
    """The 24 rotations that map coordinate axes to coordinate axes: their
    entries are 0 and +-1, so they act exactly on binary32 data."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            Q = np.zeros((3, 3))
            for i, j in enumerate(perm):
                Q[i, j] = signs[i]
            if np.linalg.det(Q) > 0:
                out.append(Q)
    return out


def test_joint_rigid_transform_is_exact():
    """p' = Q p + t0, R'_v = R_v Q^T, t'_v = t_v - R'_v t0 leaves every
    camera-space point, and R'_v Q d = R_v d, unchanged, so J'(Q d) = J(d).
    Cameras on a 2^-16 grid, points on a 2^-20 grid, t0 on a 2^-8 grid and
    axis-permuting rotations make the transformed binary32 inputs exact; the
    binary64 objective then agrees to 1e-12 (observed: 2e-16)."""
    sc = scenegen.random_direction_field_scene(17, n_points=24, n_views=6, res=64, smooth=True)
    cams = sc.cams.astype(np.float64).copy()
    cams[:, 4:16] = np.round(cams[:, 4:16] * 2.0 ** 16) / 2.0 ** 16
    pts = np.round(sc.points.astype(np.float64) * 2.0 ** 20) / 2.0 ** 20
    rng = np.random.default_rng(17)
    o = oracle.Oracle(cams.astype(np.float32), sc.theta, sc.conf, patch=3, top_k=4)
    rots = _signed_permutation_rotations()
    assert len(rots) == 24
    n_checked = 0
    for Q in rots[1:9]:
        t0 = np.round(rng.uniform(-0.1, 0.1, 3) * 2.0 ** 8) / 2.0 ** 8
        cams2 = cams.copy()
        for v in range(len(cams)):
            R2 = cams[v, 4:13].reshape(3, 3) @ Q.T
            cams2[v, 4:13] = R2.ravel()
            cams2[v, 13:16] = cams[v, 13:16] - R2 @ t0
        pts2 = pts @ Q.T + t0
        # the transformed scene is exactly representable in binary32
        assert np.array_equal(cams2.astype(np.float32).astype(np.float64), cams2)
        assert np.array_equal(pts2.astype(np.float32).astype(np.float64), pts2)
        o2 = oracle.Oracle(cams2.astype(np.float32), sc.theta, sc.conf, patch=3, top_k=4)
        for i in range(len(pts)):
            p, p2 = pts[i].astype(np.float32), pts2[i].astype(np.float32)
            ids, u = o.select_views(p)
            ids2, u2 = o2.select_views(p2)
            assert list(ids) == list(ids2)
            assert np.allclose(u, u2, atol=1e-9, rtol=0)
            for _ in range(5):
                d = rng.normal(size=3)
                J = o.objective(p, d)
                if math.isinf(J):
                    continue
                assert abs(o2.objective(p2, Q @ d) - J) <= 1e-12
                n_checked += 1
    assert n_checked >= 400
    # a transposed rotation (a typical slip) breaks it
    Q = next(q for q in rots if not np.array_equal(q, q.T))
    cams2 = cams.copy()
    for v in range(len(cams)):
        cams2[v, 4:13] = (cams[v, 4:13].reshape(3, 3) @ Q.T).ravel()
    o2 = oracle.Oracle(cams2.astype(np.float32), sc.theta, sc.conf, patch=3, top_k=4)
    bad = 0
    for i in range(8):
        p, p2 = pts[i].astype(np.float32), (pts[i] @ Q.T).astype(np.float32)
        d = rng.normal(size=3)
        J = o.objective(p, d)
        if not math.isinf(J):
            bad += abs(o2.objective(p2, Q.T @ d) - J) > 1e-3
    assert bad >= 1


def test_joint_rigid_transform_general_rotation():
    """The same invariance under a general rotation and translation: the
    transformed cameras are rounded to binary32, which moves J by ~1e-7."""
    sc = scenegen.random_direction_field_scene(6, n_points=16, n_views=6, res=64, smooth=True)
    rng = np.random.default_rng(6)
    Q = _rotation(rng)
    t0 = rng.normal(0, 0.05, 3)
    cams2, pts2 = _transform_scene(sc.cams, sc.points, Q, t0)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, top_k=4)
    o2 = oracle.Oracle(cams2, sc.theta, sc.conf, patch=3, top_k=4)
    n_checked = 0
    for i, p in enumerate(sc.points):
        assert o.select_views(p)[0].tolist() == o2.select_views(pts2[i])[0].tolist()
        for _ in range(5):
            d = rng.normal(size=3)
            J = o.objective(p, d)
            if math.isinf(J):
                continue
            assert o2.objective(pts2[i], Q @ d) == pytest.approx(J, abs=1e-6)
            n_checked += 1
    assert n_checked >= 40


def test_world_scaling_by_two_is_exact():
    sc = scenegen.random_direction_field_scene(7, n_points=24, n_views=6, res=48)
    cams2 = sc.cams.copy()
    cams2[:, 13:16] *= 2
    pts2 = sc.points * np.float32(2)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, top_k=4)
    o2 = oracle.Oracle(cams2, sc.theta, sc.conf, patch=3, n_candidates=48, top_k=4)
    d1, c1 = o.fuse(sc.points)
    d2, c2 = o2.fuse(pts2)
    assert np.array_equal(d1, d2) and np.array_equal(c1, c2)


def test_point_permutation_permutes_outputs():
    sc = scenegen.random_direction_field_scene(8, n_points=40, n_views=6, res=48)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, top_k=4)
    perm = np.random.default_rng(8).permutation(40)
    d1, c1 = o.fuse(sc.points)
    d2, c2 = o.fuse(sc.points[perm])
    assert np.array_equal(d1[perm], d2) and np.array_equal(c1[perm], c2)


def test_search_is_rotation_equivariant_up_to_the_lattice():
    sc = scenegen.random_direction_field_scene(9, n_points=16, n_views=6, res=64, smooth=True)
    rng = np.random.default_rng(9)
    Q = _rotation(rng)
    cams2, pts2 = _transform_scene(sc.cams, sc.points, Q, np.zeros(3))
    kw = dict(patch=3, n_candidates=48, refine_iters=8, top_k=4)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, **kw)
    o2 = oracle.Oracle(cams2, sc.theta, sc.conf, **kw)
    d1, c1 = o.fuse(sc.points)
    d2, c2 = o2.fuse(pts2)
    aT = oracle.default_step0(48) / 2 ** 8
    for i in range(len(d1)):
        if math.isinf(c1[i]):
            continue
        ang = _axial(Q @ d1[i], d2[i])[0]
        # the lattice is fixed to the world, so the search lands in the same
        # minimum only approximately: same direction or equally good
        assert ang <= 2 * aT or abs(c1[i] - c2[i]) <= 1e-5 or \
            abs(o2.objective(pts2[i], Q @ d1[i]) - c2[i]) <= 1e-3


# ---- search -----------------------------------------------------------------

def test_lattice_is_a_uniform_hemisphere():
    for n in (48, 128, 1000):
        L = oracle.lattice(n)
        assert np.allclose(np.linalg.norm(L, axis=1), 1, atol=1e-15)
        assert (L[:, 2] > 0).all()
        # equal-area bands: z quantiles of a uniform hemisphere are uniform
        assert np.allclose(np.sort(L[:, 2]), (np.arange(n) + 0.5) / n, atol=1e-12)
    L = oracle.lattice(4000)
    # every axial direction has a lattice point within a small angle
    rng = np.random.default_rng(10)
    q = rng.normal(size=(300, 3))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    worst = np.max(np.min(np.arccos(np.clip(np.abs(q @ L.T), 0, 1)), axis=1))
    assert worst < 2.5 * math.sqrt(2 * math.pi / 4000)


def test_onb_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        e1, e2 = oracle.onb(n)
        M = np.stack([e1, e2, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(e1, e2), n, atol=1e-12)


def test_no_refinement_returns_the_exact_lattice_argmin():
    sc = scenegen.random_direction_field_scene(12, n_points=10, n_views=6, res=48)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=0,
                      top_k=4)
    L = oracle.lattice(48)
    dirs, costs = o.fuse(sc.points)
    for i, p in enumerate(sc.points):
        J = o.objective_many(p, L)
        if math.isinf(J[0]):
            assert math.isinf(costs[i]) and not dirs[i].any()
            continue
        k = int(np.argmin(J))          # first minimum
        assert costs[i] == J[k]
        assert np.allclose(dirs[i], L[k], atol=0)


def test_refinement_never_increases_cost():
    sc = scenegen.random_direction_field_scene(13, n_points=20, n_views=6, res=48)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=8,
                      top_k=4)
    for p in sc.points:
        d, tr, lb, k = o.trace(p)
        if k == 0:
            continue
        assert np.all(np.diff(tr) <= 0)
        assert tr[-1] == pytest.approx(o.objective(p, d), abs=1e-15)


def test_search_matches_dense_brute_force_on_a_clean_strand():
    sc = scenegen.straight_strand_scene(seed=14, n_points=12, n_views=4, res=64)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=8,
                      top_k=4)
    dense = oracle.lattice(100_000)
    dirs, costs = o.fuse(sc.points)
    ok = 0
    n = 0
    for i, p in enumerate(sc.points):
        if math.isinf(costs[i]):
            continue
        n += 1
        J = o.objective_many(p, dense)
        ok += costs[i] <= J.min() + 1e-4
    assert n >= 8 and ok == n


def test_noise_free_strand_recovers_ground_truth():
    sc = scenegen.straight_strand_scene(seed=15, n_points=40, n_views=8, res=256)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=12,
                      top_k=5)
    dirs, costs = o.fuse(sc.points)
    fin = np.isfinite(costs)
    assert fin.sum() >= 30
    err = _axial(dirs[fin], sc.gt[fin])
    assert err.max() <= 1e-3


def test_search_reaches_the_brute_force_optimum_on_a_clean_strand():
    """Dense hemisphere lattice of 10^6 directions (spacing about 2.5e-3 rad):
    on a noise-free single strand (4 views, 64^2) every point's search result
    is within 1e-4 of the brute-force minimum of J."""
    sc = scenegen.straight_strand_scene(seed=21, n_points=40, n_views=4, res=64)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, refine_iters=8,
                      top_k=4)
    dense = oracle.lattice(1_000_000)
    dirs, costs = o.fuse(sc.points)
    n = ok = 0
    for i, p in enumerate(sc.points):
        if math.isinf(costs[i]):
            continue
        n += 1
        ok += costs[i] <= o.objective_many(p, dense).min() + 1e-4
    assert n >= 30 and ok == n


def _golden_gt():
    with open(os.path.join(os.path.dirname(__file__), "golden", "gt_regression.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["bf_noise_free", "bf_noisy"])
def test_brute_force_fraction_on_helices(name):
    """The same brute force on 100 points of 40 helices (4 views, 64^2, zero
    jitter; noise-free and kappa = 50): the search is a heuristic, so the
    fraction of points at the dense optimum (within 1e-4) is reported and held
    to its first value (tests/golden/gt_regression.json)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_gt_regression", os.path.join(os.path.dirname(__file__), "golden",
                                           "make_gt_regression.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    got = mk.run_bf(name)
    want = _golden_gt()[name]
    print(name, got)
    assert got["n"] == want["n"]
    assert got["frac_at_optimum"] >= want["frac_at_optimum"] - 0.02


@pytest.mark.parametrize("name", ["helix_noise_free", "helix_noisy"])
def test_helical_ground_truth_regression(name):
    """Error against the generator's ground-truth tangents on 4000 points of
    the helical tiny recipe, noise-free with zero jitter and as specified
    (kappa = 50, 2 mm jitter): regression thresholds set from the oracle's
    first run, 2% slack."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_gt_regression", os.path.join(os.path.dirname(__file__), "golden",
                                           "make_gt_regression.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    got = mk.run_gt(name)
    want = _golden_gt()[name]
    print(name, got)
    assert abs(got["n"] - want["n"]) <= 2
    assert got["mean_deg"] <= 1.02 * want["mean_deg"]
    assert got["median_deg"] <= 1.02 * want["median_deg"]


def test_canonical_sign():
    sc = scenegen.random_direction_field_scene(16, n_points=30, n_views=6, res=48)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, n_candidates=48, top_k=4)
    dirs, costs = o.fuse(sc.points)
    for d, c in zip(dirs, costs):
        if math.isinf(c):
            assert not d.any()
            continue
        assert np.linalg.norm(d) == pytest.approx(1, abs=1e-14)
        assert d[2] > 0 or (d[2] == 0 and (d[1] > 0 or (d[1] == 0 and d[0] >= 0)))


def test_paper_hyperparameters_fixture():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "paper_hyperparameters.json")))
    assert g["top_k"] == 5 and g["patch"] == 5 and g["depth_range_mm"] == 10.0
