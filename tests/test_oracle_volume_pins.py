"""Pins of the oracle's occupancy / orientation volume (the fusion of the
oriented points into one volume that opens Sec. 3.2; the rule is a reading,
stated in oracle/volume.c).

Checked against what the mathematics fixes: the 3x3 eigen-solver against
LAPACK (numpy.linalg.eigh), the voxel rule against a brute-force binary32
evaluation, rank-one tensors (one direction), cones (closed-form
eigenvalues), even in-plane spreads (coherence 0), axial and weight-scale
invariance, order independence and counts.
"""
import math

import numpy as np
import pytest

import oracle


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _canon(d):
    d = np.array(d, np.float64)
    s = d[2] if d[2] != 0 else (d[1] if d[1] != 0 else d[0])
    return -d if s < 0 else d


def test_eigen_solver_against_lapack():
    rng = np.random.default_rng(11)
    mats = []
    for _ in range(150):
        B = rng.normal(size=(3, 3))
        mats.append(B @ B.T)              # positive semidefinite
        mats.append(B + B.T)              # indefinite
    Q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    mats += [np.diag([3.0, 1.0, 1.0]), np.zeros((3, 3)), np.eye(3) * 2.5,
             Q @ np.diag([2.0, 2.0, 0.5]) @ Q.T, Q @ np.diag([1.0, 0.0, 0.0]) @ Q.T,
             np.diag([0.0, 5.0, 1.0])]
    for A in mats:
        lam, V = oracle.sym3_eigen(A)
        ref = np.linalg.eigvalsh(A)[::-1]
        scale = max(1.0, np.abs(ref).max())
        assert np.allclose(lam, ref, atol=1e-12 * scale)
        assert np.allclose(V.T @ V, np.eye(3), atol=1e-12)
        assert np.allclose(A @ V, V * lam, atol=1e-11 * scale)


def test_voxel_rule_against_binary32_brute_force():
    rng = np.random.default_rng(12)
    o = np.array([-0.1, -0.05, 0.02], np.float32)
    h = np.float32(0.002)
    dims = np.array([40, 30, 20], np.int32)
    pts = (o + rng.uniform(-0.01, 0.09, (4000, 3))).astype(np.float32)
    for p in pts:
        q = (p - o) / h                                 # numpy binary32
        ok = np.all((q >= 0) & (q < dims.astype(np.float32)))
        i = np.floor(q).astype(np.int64)
        want = (i[2] * dims[1] + i[1]) * dims[0] + i[0] if ok else -1
        assert oracle.voxel_of(p, o, h, dims) == want
    # faces go to the upper voxel; the far face and non-finite points are out
    o0 = np.zeros(3, np.float32)
    h0 = np.float32(0.5)
    d0 = np.array([4, 4, 4], np.int32)
    assert oracle.voxel_of([0.5, 0.0, 1.0], o0, h0, d0) == (2 * 4 + 0) * 4 + 1
    assert oracle.voxel_of([2.0, 0.0, 0.0], o0, h0, d0) == -1
    assert oracle.voxel_of([-1e-9, 0.0, 0.0], o0, h0, d0) == -1
    assert oracle.voxel_of([np.nan, 0.0, 0.0], o0, h0, d0) == -1
    assert oracle.voxel_of([np.inf, 0.0, 0.0], o0, h0, d0) == -1


def _grid():
    return np.zeros(3, np.float32), np.float32(0.25), np.array([4, 4, 4], np.int32)


def test_one_direction_gives_itself_with_coherence_one():
    rng = np.random.default_rng(13)
    o, h, dims = _grid()
    for _ in range(50):
        d = _unit(rng.normal(size=3)).astype(np.float32)
        w = np.float32(rng.uniform(0.1, 1.0))
        k = int(rng.integers(1, 6))
        pts = np.tile(np.array([[0.3, 0.6, 0.1]], np.float32), (k, 1))
        r = oracle.volume(pts, np.tile(d, (k, 1)), o, h, dims, weights=np.full(k, w))
        v = (0 * 4 + 2) * 4 + 1
        assert r["occ"].ravel()[v] == k and r["occ"].sum() == k and r["inside"] == k
        dd = d.astype(np.float64)
        T = r["tensor"].reshape(-1, 6)[v]
        want = k * float(w) * np.array([dd[0] ** 2, dd[1] ** 2, dd[2] ** 2, dd[0] * dd[1],
                                        dd[0] * dd[2], dd[1] * dd[2]])
        assert np.allclose(T, want, atol=1e-14)
        assert np.allclose(r["dir"].reshape(-1, 3)[v], _canon(dd / np.linalg.norm(dd)),
                           atol=1e-7)
        assert abs(r["coherence"].ravel()[v] - 1.0) < 1e-9


def test_cone_has_the_closed_form_eigenvalues():
    """M directions at angle alpha around axis a, azimuths 2 pi k / M:
    T = M (cos^2 a a a^T + sin^2 a / 2 (u u^T + v v^T)), so the orientation
    is a and the coherence 1 - tan^2(alpha) / 2 (for tan^2 < 2)."""
    rng = np.random.default_rng(14)
    o, h, dims = _grid()
    for alpha in (0.1, 0.4, 0.7, 0.9):
        a = _unit(rng.normal(size=3))
        u = _unit(np.cross(a, [0.3, 0.5, 0.7]))
        v = np.cross(a, u)
        M = 12
        phi = 2 * math.pi * np.arange(M) / M
        D = (math.cos(alpha) * a + math.sin(alpha) * (np.cos(phi)[:, None] * u +
                                                      np.sin(phi)[:, None] * v))
        D32 = D.astype(np.float32)
        pts = np.full((M, 3), 0.4, np.float32)
        r = oracle.volume(pts, D32, o, h, dims)
        vox = (1 * 4 + 1) * 4 + 1
        # binary32 inputs: the closed form holds to the inputs' rounding
        assert abs(r["coherence"].ravel()[vox] - (1 - math.tan(alpha) ** 2 / 2)) < 1e-6
        ang = math.acos(min(1.0, abs(float(r["dir"].reshape(-1, 3)[vox] @ a))))
        assert ang < 1e-6


def test_even_spread_in_a_plane_has_no_coherence():
    rng = np.random.default_rng(15)
    o, h, dims = _grid()
    n = _unit(rng.normal(size=3))
    u = _unit(np.cross(n, [1.0, 0.2, 0.1]))
    v = np.cross(n, u)
    for M in (3, 4, 7):
        phi = math.pi * np.arange(M) / M
        D = np.cos(phi)[:, None] * u + np.sin(phi)[:, None] * v
        r = oracle.volume(np.full((M, 3), 0.9, np.float32), D.astype(np.float32), o, h, dims)
        vox = (3 * 4 + 3) * 4 + 3
        assert r["coherence"].ravel()[vox] < 1e-6
        assert abs(float(r["dir"].reshape(-1, 3)[vox] @ n)) < 1e-6   # in the plane


def test_axial_weight_scale_and_order_invariance():
    rng = np.random.default_rng(16)
    o = np.array([-0.05, -0.05, -0.05], np.float32)
    h = np.float32(0.01)
    dims = np.array([10, 10, 10], np.int32)
    n = 5000
    pts = rng.uniform(-0.06, 0.06, (n, 3)).astype(np.float32)
    D = _unit(rng.normal(size=(n, 3))).astype(np.float32)
    w = rng.uniform(0, 1, n).astype(np.float32)
    r = oracle.volume(pts, D, o, h, dims, weights=w)
    # d and -d: every product d_a d_b is unchanged, so the volume is identical
    sg = np.where(rng.uniform(size=n) < 0.5, -1, 1).astype(np.float32)[:, None]
    r2 = oracle.volume(pts, D * sg, o, h, dims, weights=w)
    for k in ("occ", "tensor", "dir", "coherence"):
        assert np.array_equal(r[k], r2[k])
    # weights x 4 (exact in binary32): tensor x 4, orientation unchanged
    r3 = oracle.volume(pts, D, o, h, dims, weights=w * 4)
    assert np.allclose(r3["tensor"], 4 * r["tensor"], atol=1e-12)
    assert np.allclose(r3["coherence"], r["coherence"], atol=1e-9)
    busy = r["coherence"] > 1e-3
    assert np.all(np.abs(np.sum(r3["dir"] * r["dir"], -1))[busy] > 1 - 1e-9)
    # point order changes only the rounding of the sums
    perm = rng.permutation(n)
    r4 = oracle.volume(pts[perm], D[perm], o, h, dims, weights=w[perm])
    assert np.array_equal(r4["occ"], r["occ"])
    assert np.allclose(r4["tensor"], r["tensor"], atol=1e-12)


def test_counts_and_tensors_against_brute_force():
    rng = np.random.default_rng(17)
    o = np.array([0.0, 0.0, 0.0], np.float32)
    h = np.float32(0.02)
    dims = np.array([6, 5, 4], np.int32)
    n = 3000
    pts = rng.uniform(-0.02, 0.14, (n, 3)).astype(np.float32)
    D = _unit(rng.normal(size=(n, 3))).astype(np.float32)
    w = rng.uniform(0, 1, n).astype(np.float32)
    r = oracle.volume(pts, D, o, h, dims, weights=w)
    q = (pts - o) / h
    ok = np.all((q >= 0) & (q < dims.astype(np.float32)), axis=1)
    i = np.floor(q[ok]).astype(np.int64)
    lin = (i[:, 2] * dims[1] + i[:, 1]) * dims[0] + i[:, 0]
    nv = int(np.prod(dims))
    assert r["inside"] == ok.sum()
    assert np.array_equal(r["occ"].ravel(), np.bincount(lin, minlength=nv))
    d64 = D[ok].astype(np.float64)
    w64 = w[ok].astype(np.float64)
    outer = w64[:, None, None] * d64[:, :, None] * d64[:, None, :]
    T = np.zeros((nv, 3, 3))
    np.add.at(T, lin, outer)
    six = np.stack([T[:, 0, 0], T[:, 1, 1], T[:, 2, 2], T[:, 0, 1], T[:, 0, 2], T[:, 1, 2]], -1)
    assert np.allclose(r["tensor"].reshape(-1, 6), six, atol=1e-12)
    # orientation: the top eigenvector of each voxel's tensor (LAPACK)
    for v in np.flatnonzero(r["occ"].ravel() > 0)[:60]:
        lam, V = np.linalg.eigh(T[v])
        if lam[2] - lam[1] < 1e-9 * lam[2]:
            continue
        got = r["dir"].reshape(-1, 3)[v]
        assert abs(abs(got @ V[:, 2]) - 1) < 1e-9
        assert abs(r["coherence"].ravel()[v] - (lam[2] - lam[1]) / lam[2]) < 1e-9


def test_zero_weight_and_zero_direction_count_but_carry_no_orientation():
    o, h, dims = _grid()
    pts = np.array([[0.1, 0.1, 0.1], [0.1, 0.1, 0.1], [0.6, 0.1, 0.1]], np.float32)
    D = np.array([[0, 0, 1], [0, 0, 0], [1, 0, 0]], np.float32)
    r = oracle.volume(pts, D, o, h, dims, weights=np.array([0.0, 1.0, 0.0], np.float32))
    assert r["occ"].ravel()[0] == 2 and r["occ"].ravel()[2] == 1
    assert not r["tensor"].any() and not r["dir"].any() and not r["coherence"].any()


def test_a_straight_strand_fills_its_voxels_with_its_direction():
    rng = np.random.default_rng(18)
    o = np.array([-0.1, -0.1, -0.1], np.float32)
    h = np.float32(0.004)
    dims = np.array([50, 50, 50], np.int32)
    d = _unit([0.3, -0.5, 0.8])
    t = rng.uniform(0, 0.15, 2000)
    pts = (np.array([-0.05, 0.04, -0.07]) + t[:, None] * d).astype(np.float32)
    r = oracle.volume(pts, np.tile(d.astype(np.float32), (len(t), 1)), o, h, dims)
    busy = r["occ"] > 0
    assert busy.sum() >= 0.15 / 0.004
    assert np.all(np.abs(r["dir"][busy] @ d) > 1 - 1e-7)
    assert np.all(r["coherence"][busy] > 1 - 1e-7)
