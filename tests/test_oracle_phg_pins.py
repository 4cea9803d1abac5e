"""Pins of the oracle's parallel hair growing (Sec. 3.2.1 guide strands with
deferred occupancy, Sec. 3.2.2 segment linking by Eq. 13; the stopping and
conflict rules are readings, stated in oracle/phg.c).

Checked against what the rules fix on fields with known answers: straight
traces in a uniform field leave the grid where the geometry says, the sign
follows the reference, a 90-degree turn stops a trace at the turn, empty /
incoherent voxels stop it, a voxel cap with batches of 1 blocks a second
strand that a single batch of 2 lets through, crossing counts add up to the
steps, and the linking rule against a brute-force evaluation and on chains
and conflicts built by hand.
"""
import math

import numpy as np
import pytest

import oracle

COS30 = math.cos(math.radians(30.0))


def _uniform(dims, u, coh=1.0):
    nx, ny, nz = dims
    occ = np.ones((nz, ny, nx), np.uint32)
    d = np.broadcast_to(np.asarray(u, np.float32), (nz, ny, nx, 3)).copy()
    c = np.full((nz, ny, nx), coh, np.float32)
    return dict(occ=occ, dir=d, coherence=c)


def _grid(dims, h=0.01):
    return np.zeros(3, np.float32), np.float32(h), np.asarray(dims, np.int32)


def test_uniform_field_traces_a_straight_line_to_the_border():
    dims = (20, 20, 20)
    grid = _grid(dims)
    u = np.array([0.0, 0.0, 1.0], np.float32)
    vol = _uniform(dims, u)
    seeds = np.array([[0.055, 0.105, 0.0125], [0.031, 0.017, 0.19]], np.float32)
    r = oracle.grow(vol, grid, seeds, np.tile(u, (2, 1)), step=0.004, max_steps=200,
                    voxel_cap=0)
    for i, s in enumerate(seeds):
        n = r["n_verts"][i]
        v = r["verts"][i, :n].astype(np.float64)
        # every vertex on the line; the last one left the grid (z >= 0.2)
        assert np.allclose(v[:, :2], s[:2], atol=0)
        assert np.all(np.diff(v[:, 2]) > 0)
        assert v[-2, 2] < 0.2 and v[-1, 2] >= 0.2 - 1e-7
        want = math.ceil((0.2 - s[2]) / 0.004 - 1e-6)
        assert abs((n - 1) - want) <= 1
        assert np.array_equal(r["last_dir"][i], u)


def test_direction_sign_follows_the_reference():
    dims = (10, 10, 10)
    grid = _grid(dims)
    u = np.array([1.0, 0.0, 0.0], np.float32)
    vol = _uniform(dims, u)
    seed = np.array([[0.05, 0.05, 0.05]], np.float32)
    a = oracle.grow(vol, grid, seed, -u[None], step=0.01, voxel_cap=0)
    n = a["n_verts"][0]
    # 0.05, 0.04, ...: the last vertex is the first one outside (x < 0)
    assert n in (6, 7)
    assert a["verts"][0, n - 1, 0] < 0 <= a["verts"][0, n - 2, 0]
    assert np.all(np.diff(a["verts"][0, :n, 0]) < 0)
    assert np.array_equal(a["last_dir"][0], -u)


def test_a_sharp_turn_stops_the_trace_at_the_turn():
    dims = (10, 10, 10)
    grid = _grid(dims)
    vol = _uniform(dims, [0.0, 0.0, 1.0])
    vol["dir"][6:, :, :] = np.array([1.0, 0.0, 0.0], np.float32)   # z >= 0.06: along x
    seed = np.array([[0.05, 0.05, 0.005]], np.float32)
    r = oracle.grow(vol, grid, seed, np.array([[0, 0, 1]], np.float32), step=0.01,
                    voxel_cap=0, max_bend_cos=COS30)
    n = r["n_verts"][0]
    assert r["verts"][0, n - 1, 2] >= 0.06 - 1e-7 and r["verts"][0, n - 2, 2] < 0.06
    # a loose bend limit lets it turn
    r2 = oracle.grow(vol, grid, seed, np.array([[0, 0, 1]], np.float32), step=0.01,
                     voxel_cap=0, max_bend_cos=-1.0)
    assert r2["n_verts"][0] > n and r2["verts"][0, r2["n_verts"][0] - 1, 0] > 0.06


def test_the_first_step_takes_any_angle_to_the_seed_direction():
    """A root's reference is the scalp normal, which the hair may leave at a
    steep angle: only the sign comes from it, the bend limit starts after
    the first step."""
    dims = (10, 10, 10)
    grid = _grid(dims)
    u = np.array([1.0, 0.0, 0.0], np.float32)
    vol = _uniform(dims, u)
    normal = np.array([[0.5, 0.0, math.sqrt(0.75)]], np.float32)     # 60 deg from u
    r = oracle.grow(vol, grid, np.array([[0.005, 0.05, 0.05]], np.float32), normal,
                    step=0.01, voxel_cap=0, max_bend_cos=COS30)
    assert r["n_verts"][0] == 11 and np.array_equal(r["last_dir"][0], u)


def test_empty_incoherent_and_outside_voxels_stop():
    dims = (10, 1, 1)
    grid = _grid(dims)
    u = np.array([1.0, 0.0, 0.0], np.float32)
    vol = _uniform(dims, u)
    vol["occ"][0, 0, 5] = 0
    seed = np.array([[0.005, 0.005, 0.005]], np.float32)
    r = oracle.grow(vol, grid, seed, u[None], step=0.01, voxel_cap=0)
    assert r["n_verts"][0] == 6          # voxels 0..4 stepped through, 5 empty
    vol["occ"][0, 0, 5] = 1
    vol["coherence"][0, 0, 3] = 0.1
    r = oracle.grow(vol, grid, seed, u[None], step=0.01, voxel_cap=0, min_coherence=0.2)
    assert r["n_verts"][0] == 4
    r = oracle.grow(vol, grid, np.array([[-0.001, 0.005, 0.005]], np.float32), u[None],
                    step=0.01, voxel_cap=0)
    assert r["n_verts"][0] == 1 and not r["last_dir"].any()
    r = oracle.grow(_uniform(dims, u), grid, seed, u[None], step=0.01, voxel_cap=0,
                    max_steps=3)
    assert r["n_verts"][0] == 4


def test_deferred_occupancy_and_crossing_counts():
    dims = (10, 4, 4)
    grid = _grid(dims)
    u = np.array([1.0, 0.0, 0.0], np.float32)
    vol = _uniform(dims, u)
    seeds = np.array([[0.005, 0.015, 0.015], [0.005, 0.015, 0.015], [0.005, 0.025, 0.025]],
                     np.float32)
    dirs = np.tile(u, (3, 1))
    # one batch: no strand sees another, all grow to the border
    a = oracle.grow(vol, grid, seeds, dirs, step=0.01, voxel_cap=1, batch=3)
    assert list(a["n_verts"]) == [11, 11, 11]
    # batches of one: the second strand starts in a voxel the first crossed
    b = oracle.grow(vol, grid, seeds, dirs, step=0.01, voxel_cap=1, batch=1)
    assert list(b["n_verts"]) == [11, 1, 11]
    # every step counts once in the voxel it read
    for r in (a, b):
        assert r["crossings"].sum() == int(np.sum(r["n_verts"] - 1))
    assert a["crossings"].reshape(4, 4, 10)[1, 1].tolist() == [2] * 10
    # counts carried in from an earlier call block as well
    c = oracle.grow(vol, grid, seeds[:1], dirs[:1], step=0.01, voxel_cap=2,
                    crossings=a["crossings"])
    assert c["n_verts"][0] == 1


def test_seed_modes_take_the_volume_direction():
    dims = (10, 10, 10)
    grid = _grid(dims)
    u = np.array([0.0, 1.0, 0.0], np.float32)
    vol = _uniform(dims, u)
    seed = np.array([[0.05, 0.065, 0.05]], np.float32)
    centre = (0.05, 0.05, 0.05)            # the seed lies at +y of the centre
    f = oracle.grow(vol, grid, seed, seed_mode=1, centre=centre, step=0.01, voxel_cap=0)
    b = oracle.grow(vol, grid, seed, seed_mode=2, centre=centre, step=0.01, voxel_cap=0)
    assert np.all(np.diff(f["verts"][0, :f["n_verts"][0], 1]) > 0)   # away: +y
    assert np.all(np.diff(b["verts"][0, :b["n_verts"][0], 1]) < 0)   # towards: -y
    assert np.array_equal(f["last_dir"][0], u)
    # the backward trace reports the segment's own direction (root to tip)
    assert np.array_equal(b["last_dir"][0], u)


def _link_brute(S, SD, E, ED, flags, dmax, cmin):
    n = len(S)
    d2max = np.float32(dmax) * np.float32(dmax)
    prop = -np.ones(n, int)
    pd = np.zeros(n)
    for i in range(n):
        if not flags[i] & 1:
            continue
        for j in range(n):
            if j == i or (flags[j] & 3) != 3:
                continue
            d = E[i].astype(np.float64) - S[j]
            d2 = float(d @ d)
            if d2 < d2max and float(ED[i].astype(np.float64) @ SD[j]) > cmin:
                if prop[i] < 0 or d2 < pd[i]:
                    prop[i], pd[i] = j, d2
    succ = -np.ones(n, int)
    win = {}
    for i in range(n):
        j = prop[i]
        if j >= 0 and (j not in win or pd[i] < pd[win[j]]):
            win[j] = i
    for j, i in win.items():
        succ[i] = j
    return succ


def test_linking_against_brute_force():
    rng = np.random.default_rng(21)
    for n in (1, 7, 300):
        S = rng.uniform(0, 0.05, (n, 3)).astype(np.float32)
        E = rng.uniform(0, 0.05, (n, 3)).astype(np.float32)
        SD = rng.normal(size=(n, 3))
        SD = (SD / np.linalg.norm(SD, axis=1, keepdims=True)).astype(np.float32)
        ED = rng.normal(size=(n, 3))
        ED = (ED / np.linalg.norm(ED, axis=1, keepdims=True)).astype(np.float32)
        flags = rng.choice([0, 1, 3, 3, 3], n).astype(np.uint8)
        got = oracle.link(S, SD, E, ED, flags, 0.01, 0.3)
        assert np.array_equal(got, _link_brute(S, SD, E, ED, flags, 0.01, 0.3))
        # a link is always a compatible pair and no start is taken twice
        ok = got >= 0
        assert len(set(got[ok].tolist())) == ok.sum()
        for i in np.flatnonzero(ok):
            j = got[i]
            assert np.linalg.norm(E[i] - S[j]) < 0.0101 and ED[i] @ SD[j] > 0.3 - 1e-6


def test_chains_conflicts_and_ties():
    z = np.array([0.0, 0.0, 1.0], np.float32)
    # pieces 0..3 along z, each end 1 mm below the next start
    S = np.array([[0, 0, 0.00], [0, 0, 0.011], [0, 0, 0.022], [0, 0, 0.033]], np.float32)
    E = S + np.array([0, 0, 0.010], np.float32)
    D = np.tile(z, (4, 1))
    flags = np.array([1, 3, 3, 3], np.uint8)        # piece 0 is a root strand
    assert oracle.link(S, D, E, D, flags, 0.003, COS30).tolist() == [1, 2, 3, -1]
    # a perpendicular start does not continue a strand
    D2 = D.copy()
    D2[2] = [1.0, 0.0, 0.0]
    assert oracle.link(S, D2, E, D, flags, 0.003, COS30).tolist() == [1, -1, 3, -1]
    # two ends near one start: the nearer wins; equal distances: the lower index
    S3 = np.array([[0, 0, 0.05], [0, 0, 0.05], [0, 0, 0.0]], np.float32)
    E3 = np.array([[0, 0, -0.002], [0, 0, -0.001], [0, 0, 0.03]], np.float32)
    D3 = np.tile(z, (3, 1))
    f3 = np.array([1, 1, 3], np.uint8)
    assert oracle.link(S3, D3, E3, D3, f3, 0.003, COS30).tolist() == [-1, 2, -1]
    E4 = np.array([[0.001, 0, 0.0], [-0.001, 0, 0.0], [0, 0, 0.03]], np.float32)
    assert oracle.link(S3, D3, E4, D3, f3, 0.003, COS30).tolist() == [2, -1, -1]
    # a piece never continues itself
    assert oracle.link(S[:1], D[:1], S[:1], D[:1], np.array([3], np.uint8), 0.003,
                       COS30).tolist() == [-1]


def _trace(points, S):
    v = np.zeros((S, 3), np.float32)
    v[:len(points)] = points
    return v


def test_assembly_concatenates_a_chain_root_to_tip():
    S = 6
    z = lambda a, b: np.array([[0, 0, t] for t in np.arange(a, b, 0.001)], np.float32)
    guide = dict(verts=_trace(z(0.0, 0.004), S)[None], n_verts=np.array([4], np.int32))
    # segment 0 from seed 0.0065: backward to 0.0045, forward to 0.0075;
    # segment 1 from seed 0.0095: backward 0.0085, forward 0.0105
    b0 = np.array([[0, 0, 0.0065], [0, 0, 0.0055], [0, 0, 0.0045]], np.float32)
    f0 = np.array([[0, 0, 0.0065], [0, 0, 0.0075]], np.float32)
    b1 = np.array([[0, 0, 0.0095], [0, 0, 0.0085]], np.float32)
    f1 = np.array([[0, 0, 0.0095], [0, 0, 0.0105]], np.float32)
    fwd = dict(verts=np.stack([_trace(f0, S), _trace(f1, S)]), n_verts=np.array([2, 2], np.int32))
    bwd = dict(verts=np.stack([_trace(b0, S), _trace(b1, S)]), n_verts=np.array([3, 2], np.int32))
    off, verts, pieces = oracle.assemble(guide, fwd, bwd, np.array([1, 2, -1], np.int32))
    want = np.concatenate([z(0.0, 0.004), b0[:0:-1], f0, b1[:0:-1], f1])
    assert off.tolist() == [0, len(want)] and pieces.tolist() == [3]
    assert np.array_equal(verts, want)
    assert np.all(np.diff(verts[:, 2]) > 0)          # root to tip, no repeated seed
    # an unlinked guide strand is its own trace; a chain stops at a guide piece
    off, verts, pieces = oracle.assemble(guide, fwd, bwd, np.array([-1, 2, -1], np.int32))
    assert off.tolist() == [0, 4] and pieces.tolist() == [1]
    off, verts, pieces = oracle.assemble(guide, fwd, bwd, np.array([1, 0, -1], np.int32))
    assert pieces.tolist() == [2] and off[-1] == 4 + 2 + 2


def test_assembled_strands_are_continuous_on_a_traced_volume():
    """Grow, link and assemble on a uniform field: inside a piece every step
    has the step length; at a joint the gap is within the link distance."""
    dims = (40, 10, 10)
    grid = _grid(dims, h=0.005)
    u = np.array([1.0, 0.0, 0.0], np.float32)
    vol = _uniform(dims, u)
    roots = np.array([[0.001, 0.025, 0.025]], np.float32)
    g = oracle.grow(vol, grid, roots, u[None], step=0.004, max_steps=10, voxel_cap=0)
    seeds = np.array([[0.0495, 0.025, 0.025], [0.0775, 0.025, 0.025]], np.float32)
    f = oracle.grow(vol, grid, seeds, seed_mode=1, centre=(-1.0, 0.025, 0.025), step=0.004,
                    max_steps=5, voxel_cap=0)
    b = oracle.grow(vol, grid, seeds, seed_mode=2, centre=(-1.0, 0.025, 0.025), step=0.004,
                    max_steps=1, voxel_cap=0)
    ng = 1
    S_ = np.concatenate([roots, b["verts"][np.arange(2), b["n_verts"] - 1]])
    SD = np.concatenate([u[None], b["last_dir"]])
    E = np.concatenate([g["verts"][np.arange(1), g["n_verts"] - 1],
                        f["verts"][np.arange(2), f["n_verts"] - 1]])
    ED = np.concatenate([g["last_dir"], f["last_dir"]])
    F = np.array([1, 3, 3], np.uint8)
    succ = oracle.link(S_, SD, E, ED, F, 0.006, COS30)
    assert succ.tolist() == [1, 2, -1]
    off, verts, pieces = oracle.assemble(g, f, b, succ)
    assert pieces.tolist() == [3]
    d = np.linalg.norm(np.diff(verts.astype(np.float64), axis=0), axis=1)
    assert np.all((np.abs(d - 0.004) < 1e-6) | (d < 0.006))
    assert np.all(np.diff(verts[:, 0]) > 0)
