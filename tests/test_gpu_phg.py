"""GPU parity of parallel hair growing (fd_grow_strands: Sec. 3.2.1;
fd_link_segments: Sec. 3.2.2, Eq. 13) against the CPU oracle.

Both sides read the same binary32 volume (the GPU's own fd_fuse_volume
output, copied to the host for the oracle) and take every decision with the
same binary32 operations, so traces must be identical bit for bit (vertices,
lengths, last directions), crossing counts identical, and links identical.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
COS30 = math.cos(math.radians(30.0))
T = dict(step=1e-3, max_steps=200, min_coherence=0.2, max_bend_cos=COS30, voxel_cap=8)


def _native():
    from paper_2604_05794_amd import native
    native.lib()
    return native


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _volume(recipe, seed, n, voxel):
    nat = _native()
    pts, dirs, w, _ = scenegen.make_oriented_points(recipe, seed, n)
    origin, h, dims = scenegen.head_grid(pts, voxel)
    occ, D, C = nat.fuse_volume(_t(pts), _t(dirs), origin, h, dims, weights=_t(w))
    torch.cuda.synchronize()
    host = dict(occ=occ.cpu().numpy().view(np.uint32), dir=D.cpu().numpy(),
                coherence=C.cpu().numpy())
    return (origin, h, dims), (occ, D, C), host


def _grow_both(grid, dev_vol, host_vol, seeds, seed_dirs, crossings_dev, crossings_host, **kw):
    nat = _native()
    prm = dict(T)
    prm.update(kw)
    origin, h, dims = grid
    v, n, last = nat.grow_strands(*dev_vol, origin, h, dims, _t(seeds),
                                  None if seed_dirs is None else _t(seed_dirs),
                                  crossings=crossings_dev, **prm)
    torch.cuda.synchronize()
    o = oracle.grow(host_vol, grid, seeds, seed_dirs, crossings=crossings_host,
                    **{k: v_ for k, v_ in prm.items() if k != "centre" and k != "seed_mode"},
                    seed_mode=prm.get("seed_mode", 0), centre=prm.get("centre", (0, 0, 0)))
    v, n, last = v.cpu().numpy(), n.cpu().numpy(), last.cpu().numpy()
    assert np.array_equal(n, o["n_verts"])
    for i in range(len(seeds)):
        assert np.array_equal(v[i, :n[i]], o["verts"][i, :n[i]]), i
    assert np.array_equal(last, o["last_dir"])
    assert np.array_equal(crossings_dev.cpu().numpy().view(np.uint32), o["crossings"])
    return v, n, last, o["crossings"]


def test_guide_strands_and_segments_match_the_oracle():
    nat = _native()
    grid, dev_vol, host_vol = _volume("tiny", 0, 100_000, 0.004)
    roots, normals = scenegen.scalp_seeds("tiny", 0)
    # more seeds than the 200 roots: hair points with their noisy directions
    pts, dirs, _, _ = scenegen.make_oriented_points("tiny", 5, 3000)
    seeds = np.concatenate([roots, pts])
    sdirs = np.concatenate([normals, dirs])
    nv = int(np.prod(grid[2]))
    cr = torch.zeros(nv, dtype=torch.int32, device=DEV)
    v, n, last, crh = _grow_both(grid, dev_vol, host_vol, seeds, sdirs, cr, None, step=2e-3,
                                 batch=64, voxel_cap=3)
    print("guide traces: mean steps", float(np.mean(n - 1)), "stopped at once",
          int(np.sum(n == 1)), flush=True)
    # the roots grow (the extra seeds crowd their voxels past the cap)
    assert np.mean(n[:len(roots)] - 1) > 3
    # interior segments, forward and backward, continuing the counts
    lat = scenegen.lattice_seeds(*grid, 3)
    f = _grow_both(grid, dev_vol, host_vol, lat, None, cr, crh, step=2e-3, batch=512,
                   voxel_cap=3, seed_mode=nat.FD_SEED_AWAY, centre=(0.0, 0.0, 0.0))
    b = _grow_both(grid, dev_vol, host_vol, lat, None, cr, f[3], step=2e-3, batch=512,
                   voxel_cap=3, seed_mode=nat.FD_SEED_TOWARDS, centre=(0.0, 0.0, 0.0))
    assert np.sum((f[1] > 1) & (b[1] > 1)) > 100


@pytest.mark.parametrize("batch", [1, 7, 4096])
def test_batch_sizes(batch):
    grid, dev_vol, host_vol = _volume("tiny", 1, 50_000, 0.004)
    roots, normals = scenegen.scalp_seeds("tiny", 1)
    nv = int(np.prod(grid[2]))
    cr = torch.zeros(nv, dtype=torch.int32, device=DEV)
    _grow_both(grid, dev_vol, host_vol, roots, normals, cr, None, step=2e-3, batch=batch,
               voxel_cap=2)


def test_full_size_guide_strands():
    """The benchmark's growing: 20k roots of the realistic hairstyle through
    the 2 mm volume of 2M oriented points, batches of 4096."""
    grid, dev_vol, host_vol = _volume("realistic", 0, 2_000_000, 0.002)
    roots, normals = scenegen.scalp_seeds("realistic", 0)
    nv = int(np.prod(grid[2]))
    cr = torch.zeros(nv, dtype=torch.int32, device=DEV)
    v, n, last, _ = _grow_both(grid, dev_vol, host_vol, roots, normals, cr, None, batch=4096)
    print("realistic guide strands:", len(roots), "mean steps", float(np.mean(n - 1)), flush=True)


def _pieces(g, f, b, roots, normals):
    """Guide strands (no predecessor) then segments (backward half reversed,
    then forward half)."""
    gv, gn, gl = g[:3]
    fv, fn, fl = f[:3]
    bv, bn, bl = b[:3]
    ng, ns = len(gn), len(fn)
    ar_g, ar_s = np.arange(ng), np.arange(ns)
    starts = np.concatenate([roots, bv[ar_s, bn - 1]])
    sdirs = np.concatenate([normals, bl])
    ends = np.concatenate([gv[ar_g, gn - 1], fv[ar_s, fn - 1]])
    edirs = np.concatenate([gl, fl])
    flags = np.concatenate([np.where(gn > 1, 1, 0),
                            np.where((fn > 1) & (bn > 1), 3, 0)]).astype(np.uint8)
    return starts, sdirs, ends, edirs, flags


def test_links_match_the_oracle():
    nat = _native()
    grid, dev_vol, host_vol = _volume("tiny", 2, 100_000, 0.004)
    roots, normals = scenegen.scalp_seeds("tiny", 2)
    nv = int(np.prod(grid[2]))
    cr = torch.zeros(nv, dtype=torch.int32, device=DEV)
    g = _grow_both(grid, dev_vol, host_vol, roots, normals, cr, None, step=2e-3, batch=64)
    lat = scenegen.lattice_seeds(*grid, 3)
    f = _grow_both(grid, dev_vol, host_vol, lat, None, cr, g[3], step=2e-3, max_steps=20,
                   seed_mode=nat.FD_SEED_AWAY)
    b = _grow_both(grid, dev_vol, host_vol, lat, None, cr, f[3], step=2e-3, max_steps=20,
                   seed_mode=nat.FD_SEED_TOWARDS)
    S, SD, E, ED, F = _pieces(g, f, b, roots, normals)
    counts = []
    for dmax, cmin in ((0.003, COS30), (0.006, 0.5), (0.0015, 0.95)):
        succ = nat.link_segments(_t(S), _t(SD), _t(E), _t(ED), _t(F), dmax, cmin)
        torch.cuda.synchronize()
        want = oracle.link(S, SD, E, ED, F, dmax, cmin)
        got = succ.cpu().numpy()
        assert np.array_equal(got, want)
        counts.append(int((got >= 0).sum()))
        print("links", dmax, cmin, counts[-1], "of", len(S), flush=True)
    assert counts[1] > 50


def test_links_on_random_pieces_and_edge_cases():
    nat = _native()
    rng = np.random.default_rng(31)
    for n in (1, 2, 100, 20000):
        S = rng.uniform(-0.05, 0.05, (n, 3)).astype(np.float32)
        E = rng.uniform(-0.05, 0.05, (n, 3)).astype(np.float32)
        SD = rng.normal(size=(n, 3))
        SD = (SD / np.linalg.norm(SD, axis=1, keepdims=True)).astype(np.float32)
        ED = rng.normal(size=(n, 3))
        ED = (ED / np.linalg.norm(ED, axis=1, keepdims=True)).astype(np.float32)
        F = rng.choice([0, 1, 3, 3, 3], n).astype(np.uint8)
        dmax = 0.004 if n > 100 else 0.05
        got = nat.link_segments(_t(S), _t(SD), _t(E), _t(ED), _t(F), dmax, 0.2).cpu().numpy()
        assert np.array_equal(got, oracle.link(S, SD, E, ED, F, dmax, 0.2))
    # equal distances: the lowest proposer wins; a start exactly at d_max is out
    z = np.array([0, 0, 1], np.float32)
    S = np.array([[0, 0, 0.01], [9, 9, 9], [9, 9, 9]], np.float32)
    E = np.array([[9, 9, 9], [0.001, 0, 0.01], [-0.001, 0, 0.01]], np.float32)
    D = np.tile(z, (3, 1))
    F = np.array([3, 1, 1], np.uint8)
    got = nat.link_segments(_t(S), _t(D), _t(E), _t(D), _t(F), 0.003, 0.5).cpu().numpy()
    assert got.tolist() == [-1, 0, -1]
    got = nat.link_segments(_t(S), _t(D), _t(E), _t(D), _t(F), 0.001, 0.5).cpu().numpy()
    assert np.array_equal(got, oracle.link(S, D, E, D, F, 0.001, 0.5))
    empty = torch.empty((0, 3), dtype=torch.float32, device=DEV)
    assert nat.link_segments(empty, empty, empty, empty,
                             torch.empty(0, dtype=torch.uint8, device=DEV), 0.01, 0.5).numel() == 0


def test_invalid_arguments():
    nat = _native()
    grid, dev_vol, host_vol = _volume("tiny", 0, 20_000, 0.004)
    origin, h, dims = grid
    nv = int(np.prod(dims))
    cr = torch.zeros(nv, dtype=torch.int32, device=DEV)
    s = _t(np.zeros((4, 3), np.float32))
    for bad in (dict(step=0.0), dict(step=float("nan")), dict(batch=0), dict(voxel_cap=-1),
                dict(seed_mode=3), dict(min_coherence=float("inf"))):
        with pytest.raises(nat.FdError) as e:
            nat.grow_strands(*dev_vol, origin, h, dims, s, s, crossings=cr, **bad)
        assert e.value.code == nat.FD_E_INVAL
    with pytest.raises(nat.FdError):
        nat.grow_strands(*dev_vol, origin, h, dims, s, s, crossings=cr, max_steps=0)
    with pytest.raises(nat.FdError) as e:          # FD_SEED_GIVEN without directions
        nat.grow_strands(*dev_vol, origin, h, dims, s, None, crossings=cr)
    assert e.value.code == nat.FD_E_INVAL
    with pytest.raises(ValueError):
        nat.grow_strands(*dev_vol, origin, h, dims, s, s, crossings=cr[:-1])
    f = torch.zeros(4, dtype=torch.uint8, device=DEV)
    for dmax, cmin in ((0.0, 0.5), (float("nan"), 0.5), (0.01, float("inf"))):
        with pytest.raises(nat.FdError) as e:
            nat.link_segments(s, s, s, s, f, dmax, cmin)
        assert e.value.code == nat.FD_E_INVAL


def test_assembled_strands_match_the_oracle():
    nat = _native()
    grid, dev_vol, host_vol = _volume("tiny", 2, 100_000, 0.004)
    roots, normals = scenegen.scalp_seeds("tiny", 2)
    nv = int(np.prod(grid[2]))
    cr = torch.zeros(nv, dtype=torch.int32, device=DEV)
    origin, h, dims = grid
    lat = scenegen.lattice_seeds(*grid, 3)
    prm = dict(T)
    prm.update(step=2e-3)
    g = nat.grow_strands(*dev_vol, origin, h, dims, _t(roots), _t(normals), crossings=cr,
                         batch=64, **prm)
    prm_s = dict(prm)
    prm_s.update(max_steps=20)
    f = nat.grow_strands(*dev_vol, origin, h, dims, _t(lat), None, crossings=cr,
                         seed_mode=nat.FD_SEED_AWAY, **prm_s)
    b = nat.grow_strands(*dev_vol, origin, h, dims, _t(lat), None, crossings=cr,
                         seed_mode=nat.FD_SEED_TOWARDS, **prm_s)
    host = lambda r: (r[0].cpu().numpy(), r[1].cpu().numpy(), r[2].cpu().numpy())
    gh, fh, bh = host(g), host(f), host(b)
    S, SD, E, ED, F = _pieces(gh, fh, bh, roots, normals)
    succ = nat.link_segments(_t(S), _t(SD), _t(E), _t(ED), _t(F), 0.006, 0.5)
    off, verts, pieces = nat.assemble_strands(g, f, b, succ)
    torch.cuda.synchronize()
    asdict = lambda r: dict(verts=r[0], n_verts=r[1])
    o_off, o_verts, o_pieces = oracle.assemble(asdict(gh), asdict(fh), asdict(bh),
                                               succ.cpu().numpy())
    assert np.array_equal(off.cpu().numpy(), o_off)
    assert np.array_equal(pieces.cpu().numpy(), o_pieces)
    assert np.array_equal(verts.cpu().numpy(), o_verts)
    print("strands", len(roots), "vertices", int(o_off[-1]), "with segments",
          int((o_pieces > 1).sum()), flush=True)
    assert (o_pieces > 1).sum() > 5
    # a short output buffer is filled up to its capacity and no further
    cap = int(o_off[-1]) // 2
    out = torch.full((cap + 8, 3), -7.0, dtype=torch.float32, device=DEV)
    lib = nat.lib()
    import ctypes
    rc = lib.fd_assemble_strands(
        ctypes.c_void_p(g[0].data_ptr()), ctypes.c_void_p(g[1].data_ptr()), len(roots),
        g[0].shape[1], ctypes.c_void_p(f[0].data_ptr()), ctypes.c_void_p(f[1].data_ptr()),
        f[0].shape[1], ctypes.c_void_p(b[0].data_ptr()), ctypes.c_void_p(b[1].data_ptr()),
        b[0].shape[1], len(lat), ctypes.c_void_p(succ.data_ptr()),
        ctypes.c_void_p(off.data_ptr()), cap, None, None, ctypes.c_void_p(out.data_ptr()))
    torch.cuda.synchronize()
    assert rc == 0
    o = out.cpu().numpy()
    assert np.array_equal(o[:cap], o_verts[:cap]) and np.all(o[cap:] == -7.0)
