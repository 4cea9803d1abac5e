"""CPU oracle for fusion-patch multi-view direction optimisation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2604_05794_amd``) never imports it and shares no code with it.

Thin ctypes marshalling over ``liboracle.so`` (built from ``fdo.c``,
``mlp.c`` and ``gabor.c`` by :func:`build`); all arithmetic is in the C sources, which cite the
paper (EfficientMonoHair, Sec. 3.1, Eqs. (4), (8)-(12)).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FD_ORACLE_LIB selects another build of the same sources (the sanitizer test)
_LIB_PATH = os.environ.get("FD_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SOURCES = ("fdo.c", "mlp.c", "gabor.c", "volume.c", "phg.c")


def build(out=None, sanitize=False) -> str:
    """Compile liboracle.so with gcc (binary64, OpenMP, no FP contraction);
    sanitize=True adds AddressSanitizer and UndefinedBehaviorSanitizer
    (aborting on the first report) for a build at `out`."""
    out = out or _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = out + ".tmp"
    san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", "-g"] if sanitize else [])
    cmd = (["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-Wall"] + san + ["-o", tmp] + srcs + ["-lm"])
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class TraceParams(ctypes.Structure):
    _fields_ = [("step", ctypes.c_float), ("max_steps", ctypes.c_int32),
                ("min_coherence", ctypes.c_float), ("max_bend_cos", ctypes.c_float),
                ("voxel_cap", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("seed_mode", ctypes.c_int32), ("centre", ctypes.c_float * 3)]


class Params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("map_dtype", ctypes.c_int32),
        ("patch", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("refine_step0", ctypes.c_double),
        ("top_k", ctypes.c_int32),
        ("z_near", ctypes.c_double),
        ("depth_maps", ctypes.c_void_p),
        ("vis_tau", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, dbl, flt = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
        pp = ctypes.POINTER(Params)
        sig = {
            "fdo_half_to_float": (flt, [ctypes.c_uint16]),
            "fdo_select_views": (i32, [P, P, i32, P, pp, P, P]),
            "fdo_sample": (None, [P, P, i32, i32, i32, dbl, dbl, P]),
            "fdo_objective": (dbl, [P, P, P, i32, P, P, pp]),
            "fdo_objective_many": (i32, [P, P, i64, P, i32, P, P, pp, P, i32]),
            "fdo_objective_each": (i32, [P, P, i64, P, i32, P, P, pp, P, i32]),
            "fdo_lattice": (None, [i32, P]),
            "fdo_onb": (None, [P, P, P]),
            "fdo_fuse_directions": (i32, [P, i64, P, i32, P, P, pp, P, P, i32]),
            "fdo_fuse_trace": (i32, [P, P, i32, P, P, pp, P, P, P]),
            "fdo_fuse_learned": (i32, [P, i64, P, i32, P, P, pp, P, i32, dbl, dbl,
                                       P, P, P, i32]),
            "fdo_features": (i32, [P, i64, P, i32, P, P, pp, P, i32, P, i32]),
            "fdo_fpmvo": (i32, [P, i64, P, i32, P, P, pp, dbl, i32, dbl, P, P, i32]),
            "fdo_fpmvo_trace": (i32, [P, P, i32, P, P, pp, dbl, i32, dbl, P, P, P, P, P, P,
                                      P, P, P, P]),
            "fdo_gabor_bank": (None, [i32, i32, dbl, dbl, dbl, P]),
            "fdo_gabor": (dbl, [P, i32, i32, i32, i32, P, P, P, P, P, i32]),
            "fdo_voxel_of": (i64, [P, P, flt, P]),
            "fdo_sym3_eigen": (None, [P, P, P]),
            "fdo_tensor_orientation": (None, [P, P, P]),
            "fdo_volume": (i64, [P, P, P, i64, P, flt, P, P, P, P, P, i32]),
            "fdo_grow": (i32, [P, flt, P, P, P, P, P, P, i32, ctypes.POINTER(TraceParams), P, P,
                               P, P]),
            "fdo_link": (None, [P, P, P, P, P, i32, flt, flt, P, i32]),
            "fdo_assemble": (i64, [P, P, i32, i32, P, P, i32, P, P, i32, i32, P, P, P, P]),
            "fdo_mlp_n_params": (i64, []),
            "fdo_mlp_forward": (i32, [P, P, i32, i32, P]),
            "fdo_mlp_loss_grad": (dbl, [P, P, P, i32, i32, P]),
            "fdo_adam_step": (None, [P, P, P, P, i64, i32, flt, flt, flt, flt]),
            "fdo_round_bf16": (flt, [flt]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def make_params(width, height, map_dtype=0, patch=5, n_candidates=128,
                refine_iters=8, refine_step0=0.0, top_k=5, z_near=1e-3,
                depth_ptr=None, vis_tau=5e-3) -> Params:
    return Params(int(width), int(height), int(map_dtype), int(patch),
                  int(n_candidates), int(refine_iters), float(refine_step0),
                  int(top_k), float(z_near), depth_ptr, float(vis_tau))


def _maps(scene_theta, scene_conf):
    t = np.ascontiguousarray(scene_theta)
    c = np.ascontiguousarray(scene_conf)
    if t.dtype == np.float16:
        return t.view(np.uint16), c.view(np.uint16), 1
    return _c(t, np.float32), _c(c, np.float32), 0


class Oracle:
    """Oracle bound to one scene: points (N,3) f32, cams (V,16) f32,
    theta/conf maps (V,H,W) f32 or f16; optional depth maps (V,H,W) of the
    same dtype switch on the visibility test with tolerance vis_tau."""

    # z_near and vis_tau default to the binary32 values the library's
    # parameter struct carries (1e-3 and 5e-3 rounded to binary32), so that
    # both sides are given the same thresholds
    def __init__(self, cams, theta, conf, patch=5, n_candidates=128,
                 refine_iters=8, refine_step0=0.0, top_k=5,
                 z_near=float(np.float32(1e-3)), depth=None,
                 vis_tau=float(np.float32(5e-3))):
        self.cams = _c(cams, np.float32)
        self.theta, self.conf, dt = _maps(theta, conf)
        V, H, W = self.theta.shape
        self.V = V
        self.depth = None
        if depth is not None:
            d = np.ascontiguousarray(depth)
            if d.shape != self.theta.shape:
                raise ValueError("depth maps must have the shape of the orientation maps")
            if dt == 1:
                self.depth = _c(d, np.float16).view(np.uint16)
            else:
                self.depth = _c(d, np.float32)
        self.prm = make_params(W, H, dt, patch, n_candidates, refine_iters,
                               refine_step0, top_k, z_near,
                               None if self.depth is None else self.depth.ctypes.data,
                               vis_tau)

    def with_params(self, **kw):
        o = Oracle.__new__(Oracle)
        o.cams, o.theta, o.conf, o.V = self.cams, self.theta, self.conf, self.V
        o.depth = self.depth
        fields = {f[0]: getattr(self.prm, f[0]) for f in Params._fields_}
        fields.update(kw)
        o.prm = Params(**fields)
        return o

    def select_views(self, p):
        p = _c(p, np.float32)
        ids = np.zeros(16, np.int32)
        u = np.zeros(32, np.float64)
        k = lib().fdo_select_views(_ptr(p), _ptr(self.cams), self.V, _ptr(self.conf),
                                   ctypes.byref(self.prm), _ptr(ids), _ptr(u))
        return ids[:k].copy(), u[:2 * k].reshape(k, 2).copy()

    def objective(self, p, d):
        p = _c(p, np.float32)
        d = _c(d, np.float64)
        return lib().fdo_objective(_ptr(p), _ptr(d), _ptr(self.cams), self.V,
                                   _ptr(self.theta), _ptr(self.conf), ctypes.byref(self.prm))

    def objective_many(self, p, dirs, n_threads=0):
        p = _c(p, np.float32)
        dirs = _c(dirs, np.float64).reshape(-1, 3)
        out = np.empty(len(dirs), np.float64)
        lib().fdo_objective_many(_ptr(p), _ptr(dirs), len(dirs), _ptr(self.cams), self.V,
                                 _ptr(self.theta), _ptr(self.conf), ctypes.byref(self.prm),
                                 _ptr(out), int(n_threads))
        return out

    def objective_each(self, points, dirs, n_threads=0):
        pts = _c(points, np.float32).reshape(-1, 3)
        d = _c(dirs, np.float64).reshape(-1, 3)
        out = np.empty(len(pts), np.float64)
        lib().fdo_objective_each(_ptr(pts), _ptr(d), len(pts), _ptr(self.cams), self.V,
                                 _ptr(self.theta), _ptr(self.conf), ctypes.byref(self.prm),
                                 _ptr(out), int(n_threads))
        return out

    def fuse(self, points, n_threads=0):
        pts = _c(points, np.float32).reshape(-1, 3)
        n = len(pts)
        dirs = np.empty((n, 3), np.float64)
        costs = np.empty(n, np.float64)
        lib().fdo_fuse_directions(_ptr(pts), n, _ptr(self.cams), self.V, _ptr(self.theta),
                                  _ptr(self.conf), ctypes.byref(self.prm), _ptr(dirs),
                                  _ptr(costs), int(n_threads))
        return dirs, costs

    def trace(self, p):
        p = _c(p, np.float32)
        d = np.zeros(3, np.float64)
        tr = np.zeros(self.prm.refine_iters + 1, np.float64)
        lb = np.zeros(1, np.int32)
        k = lib().fdo_fuse_trace(_ptr(p), _ptr(self.cams), self.V, _ptr(self.theta),
                                 _ptr(self.conf), ctypes.byref(self.prm), _ptr(d), _ptr(tr),
                                 _ptr(lb))
        return d, tr, int(lb[0]), k

    def fuse_learned(self, points, proposals, learned_iters, learned_step0, tau,
                     n_threads=0):
        pts = _c(points, np.float32).reshape(-1, 3)
        prop = _c(proposals, np.float64).reshape(-1, 3)
        n = len(pts)
        dirs = np.empty((n, 3), np.float64)
        costs = np.empty(n, np.float64)
        fb = np.empty(n, np.int32)
        lib().fdo_fuse_learned(_ptr(pts), n, _ptr(self.cams), self.V, _ptr(self.theta),
                               _ptr(self.conf), ctypes.byref(self.prm), _ptr(prop),
                               int(learned_iters), float(learned_step0), float(tau),
                               _ptr(dirs), _ptr(costs), _ptr(fb), int(n_threads))
        return dirs, costs, fb

    def fpmvo(self, points, lam=1.0, n_samples=5, delta=5e-3, n_threads=0):
        """Paper-literal candidates and medoid fusion (needs depth maps):
        (dirs (N,3), costs (N,))."""
        if self.depth is None:
            raise ValueError("fpmvo needs depth maps")
        pts = _c(points, np.float32).reshape(-1, 3)
        n = len(pts)
        d = np.zeros((n, 3))
        c = np.zeros(n)
        r = lib().fdo_fpmvo(_ptr(pts), n, _ptr(self.cams), self.V, _ptr(self.theta),
                            _ptr(self.conf), ctypes.byref(self.prm), float(lam),
                            int(n_samples), float(delta), _ptr(d), _ptr(c), int(n_threads))
        if r != 0:
            raise ValueError("fdo_fpmvo rejected its arguments")
        return d, c

    def fpmvo_trace(self, p, lam=1.0, n_samples=5, delta=5e-3):
        if self.depth is None:
            raise ValueError("fpmvo needs depth maps")
        p = _c(p, np.float32)
        S = int(n_samples)
        views = np.zeros(16, np.int32)
        cand = np.zeros((16, S, 3))
        ok = np.zeros((16, S), np.int32)
        w = np.zeros(16)
        medoid = np.zeros(S, np.int32)
        fused = np.zeros((S, 3))
        J = np.zeros(S)
        sb = np.zeros(1, np.int32)
        d = np.zeros(3)
        cost = np.zeros(1)
        k = lib().fdo_fpmvo_trace(_ptr(p), _ptr(self.cams), self.V, _ptr(self.theta),
                                  _ptr(self.conf), ctypes.byref(self.prm), float(lam), S,
                                  float(delta), _ptr(views), _ptr(cand), _ptr(ok), _ptr(w),
                                  _ptr(medoid), _ptr(fused), _ptr(J), _ptr(sb), _ptr(d),
                                  _ptr(cost))
        if k < 0:
            raise ValueError("fdo_fpmvo_trace rejected its arguments")
        return dict(views=views[:k].copy(), cand=cand[:k].copy(), ok=ok[:k].astype(bool),
                    w=w[:k].copy(), medoid=medoid.copy(), fused=fused, J=J, s_best=int(sb[0]),
                    dir=d, cost=float(cost[0]))

    def features(self, points, head_centre, n_slots=16, n_threads=0):
        pts = _c(points, np.float32).reshape(-1, 3)
        hc = _c(head_centre, np.float32)
        n = len(pts)
        f = np.empty((n, 7 * n_slots), np.float64)
        lib().fdo_features(_ptr(pts), n, _ptr(self.cams), self.V, _ptr(self.theta),
                           _ptr(self.conf), ctypes.byref(self.prm), _ptr(hc), int(n_slots),
                           _ptr(f), int(n_threads))
        return f


def sample(theta_map, conf_map, x, y):
    """Bilinear doubled-angle sample of one (H, W) map pair at (x, y)."""
    t, c, dt = _maps(theta_map, conf_map)
    H, W = t.shape
    out = np.zeros(3, np.float64)
    lib().fdo_sample(_ptr(t), _ptr(c), dt, W, H, float(x), float(y), _ptr(out))
    return out


def lattice(n):
    out = np.empty((n, 3), np.float64)
    lib().fdo_lattice(int(n), _ptr(out))
    return out


def onb(n):
    n = _c(n, np.float64)
    e1 = np.empty(3)
    e2 = np.empty(3)
    lib().fdo_onb(_ptr(n), _ptr(e1), _ptr(e2))
    return e1, e2


def half_to_float(h: int) -> float:
    return lib().fdo_half_to_float(int(h))


def default_step0(n_candidates: int) -> float:
    return 0.5 * math.sqrt(2.0 * math.pi / n_candidates)


# ---- proposal network -------------------------------------------------------

MLP_DIMS = (112, 256, 256, 256, 3)


def mlp_n_params() -> int:
    return int(lib().fdo_mlp_n_params())


def mlp_forward(params, x, bf16=False):
    params = _c(params, np.float64)
    x = _c(x, np.float32).reshape(-1, MLP_DIMS[0])
    y = np.empty((len(x), 3), np.float64)
    lib().fdo_mlp_forward(_ptr(params), _ptr(x), len(x), int(bool(bf16)), _ptr(y))
    return y


def mlp_loss_grad(params, x, targets, bf16=False):
    params = _c(params, np.float64)
    x = _c(x, np.float32).reshape(-1, MLP_DIMS[0])
    t = _c(targets, np.float32).reshape(-1, 3)
    g = np.empty(mlp_n_params(), np.float64)
    loss = lib().fdo_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(t), len(x), int(bool(bf16)),
                                   _ptr(g))
    return loss, g


def adam_step(w, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float32 arrays."""
    for a in (w, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    g = _c(g, np.float32)
    lib().fdo_adam_step(_ptr(w), _ptr(m), _ptr(v), _ptr(g), len(w), int(step), float(lr),
                        float(beta1), float(beta2), float(eps))


def round_bf16(x):
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def mlp_split(params):
    """Split a flat parameter vector into [(W (in,out), b), ...]."""
    out, o = [], 0
    for l in range(4):
        k, n = MLP_DIMS[l], MLP_DIMS[l + 1]
        W = params[o:o + k * n].reshape(k, n)
        o += k * n
        b = params[o:o + n]
        o += n
        out.append((W, b))
    return out


# ---- orientation and confidence maps (gabor.c) ------------------------------

GABOR_DEFAULTS = dict(n_orient=32, radius=8, sigma_along=2.4, sigma_across=1.8, wavelength=4.0)


def gabor_bank(n_orient=32, radius=8, sigma_along=2.4, sigma_across=1.8, wavelength=4.0):
    """(n_orient, 2r+1, 2r+1) zero-mean even Gabor kernels (see gabor.c)."""
    w = 2 * int(radius) + 1
    out = np.zeros((int(n_orient), w, w), np.float64)
    lib().fdo_gabor_bank(int(n_orient), int(radius), float(sigma_along), float(sigma_across),
                         float(wavelength), _ptr(out))
    return out


def gabor(image, bank, responses=False, n_threads=0):
    """Orientation (radians, [0, pi)) and confidence ([0, 1]) maps of one
    (H, W) image: (theta, conf, max raw confidence[, responses (H, W, N)])."""
    img = _c(image, np.float32)
    H, W = img.shape
    N, w, _ = bank.shape
    bk = _c(bank, np.float64)
    th = np.zeros((H, W))
    cf = np.zeros((H, W))
    rs = np.zeros((H, W, N)) if responses else None
    m = lib().fdo_gabor(_ptr(img), W, H, N, (w - 1) // 2, _ptr(bk), _ptr(th), _ptr(cf),
                        _ptr(rs) if responses else None, None, int(n_threads))
    return (th, cf, m, rs) if responses else (th, cf, m)


# ---- occupancy and orientation volume (volume.c) ----------------------------

def voxel_of(p, origin, voxel, dims):
    """Linear voxel index of one point, or -1 outside the grid."""
    return int(lib().fdo_voxel_of(_ptr(_c(p, np.float32)), _ptr(_c(origin, np.float32)),
                                  float(np.float32(voxel)), _ptr(_c(dims, np.int32))))


def sym3_eigen(A):
    """Eigenvalues (descending) and eigenvectors (columns) of a symmetric 3x3."""
    a = _c(A, np.float64).reshape(3, 3)
    lam = np.zeros(3)
    V = np.zeros((3, 3))
    lib().fdo_sym3_eigen(_ptr(a), _ptr(lam), _ptr(V))
    return lam, V


def tensor_orientation(T6):
    """(orientation, coherence) of one tensor (xx, yy, zz, xy, xz, yz)."""
    d = np.zeros(3)
    c = np.zeros(1)
    lib().fdo_tensor_orientation(_ptr(_c(T6, np.float64)), _ptr(d), _ptr(c))
    return d, float(c[0])


def volume(points, dirs, origin, voxel, dims, weights=None, n_threads=0):
    """Occupancy / orientation volume of oriented points: dict with occ
    (nz, ny, nx) uint32, tensor (nz, ny, nx, 6), dir (nz, ny, nx, 3),
    coherence (nz, ny, nx) and inside (points counted)."""
    pts = _c(points, np.float32)
    drs = _c(dirs, np.float32)
    n = len(pts)
    w = None if weights is None else _c(weights, np.float32)
    dims = np.asarray(dims, np.int32)
    nx, ny, nz = (int(x) for x in dims)
    occ = np.zeros((nz, ny, nx), np.uint32)
    T = np.zeros((nz, ny, nx, 6))
    D = np.zeros((nz, ny, nx, 3))
    C = np.zeros((nz, ny, nx))
    inside = lib().fdo_volume(_ptr(pts), _ptr(drs), _ptr(w) if w is not None else None, n,
                              _ptr(_c(origin, np.float32)), float(np.float32(voxel)),
                              _ptr(_c(dims, np.int32)), _ptr(occ), _ptr(T), _ptr(D), _ptr(C),
                              int(n_threads))
    return dict(occ=occ, tensor=T, dir=D, coherence=C, inside=int(inside))


# ---- parallel hair growing (phg.c) -------------------------------------------

TRACE_DEFAULTS = dict(step=1e-3, max_steps=200, min_coherence=0.2,
                      max_bend_cos=math.cos(math.radians(30.0)), voxel_cap=8, batch=4096)


def grow(volume, grid, seeds, seed_dirs=None, crossings=None, seed_mode=0,
         centre=(0.0, 0.0, 0.0), **kw):
    """Traces seeds through an occupancy / orientation volume (dict with occ
    (nz, ny, nx), dir (.., 3), coherence (..) in binary32); grid = (origin,
    voxel, dims).  Returns verts (n, max_steps + 1, 3), n_verts, last_dir
    and the crossing counts (updated copy of `crossings`)."""
    prm = dict(TRACE_DEFAULTS)
    prm.update(kw)
    origin, h, dims = grid
    dims = np.asarray(dims, np.int32)
    occ = _c(volume["occ"], np.uint32)
    vd = _c(volume["dir"], np.float32)
    coh = _c(volume["coherence"], np.float32)
    nv = int(np.prod(dims.astype(np.int64)))
    assert occ.size == nv and vd.size == 3 * nv and coh.size == nv
    sd = _c(seeds, np.float32).reshape(-1, 3)
    n = len(sd)
    dd = _c(seed_dirs, np.float32).reshape(-1, 3) if seed_dirs is not None else None
    if seed_mode == 0 and dd is None:
        raise ValueError("seed_mode 0 needs seed_dirs")
    cr = np.zeros(nv, np.uint32) if crossings is None else _c(crossings, np.uint32).reshape(-1).copy()
    p = TraceParams(float(prm["step"]), int(prm["max_steps"]), float(prm["min_coherence"]),
                    float(prm["max_bend_cos"]), int(prm["voxel_cap"]), int(prm["batch"]),
                    int(seed_mode), (ctypes.c_float * 3)(*[float(c) for c in centre]))
    S = int(prm["max_steps"]) + 1
    verts = np.zeros((n, S, 3), np.float32)
    nvt = np.zeros(n, np.int32)
    last = np.zeros((n, 3), np.float32)
    lib().fdo_grow(_ptr(_c(origin, np.float32)), float(np.float32(h)), _ptr(dims), _ptr(occ),
                   _ptr(vd), _ptr(coh), _ptr(sd), _ptr(dd) if dd is not None else None, n,
                   ctypes.byref(p), _ptr(cr), _ptr(verts), _ptr(nvt), _ptr(last))
    return dict(verts=verts, n_verts=nvt, last_dir=last, crossings=cr)


def link(starts, start_dirs, ends, end_dirs, flags, max_dist, min_cos, n_threads=0):
    """Eq. (13) links: succ[i] = the accepted successor piece of i, or -1."""
    s = _c(starts, np.float32).reshape(-1, 3)
    n = len(s)
    succ = np.full(n, -1, np.int32)
    lib().fdo_link(_ptr(s), _ptr(_c(start_dirs, np.float32)), _ptr(_c(ends, np.float32)),
                   _ptr(_c(end_dirs, np.float32)), _ptr(_c(flags, np.uint8)), n,
                   float(np.float32(max_dist)), float(np.float32(min_cos)), _ptr(succ),
                   int(n_threads))
    return succ


def assemble(guide, fwd, bwd, succ):
    """Strands from linked pieces: guide, fwd, bwd are grow() results (guide
    traces; forward and backward traces of the segment seeds); succ over
    the guide pieces then the segments.  Returns (offsets (n_guide + 1),
    verts (total, 3), pieces per strand)."""
    gv = _c(guide["verts"], np.float32)
    fv = _c(fwd["verts"], np.float32)
    bv = _c(bwd["verts"], np.float32)
    ng, ns = len(gv), len(fv)
    strides = (gv.shape[1], fv.shape[1], bv.shape[1])
    gn = _c(guide["n_verts"], np.int32)
    fn = _c(fwd["n_verts"], np.int32)
    bn = _c(bwd["n_verts"], np.int32)
    sc = _c(succ, np.int32)
    lens = np.zeros(ng, np.int64)
    pcs = np.zeros(ng, np.int32)
    args = (_ptr(gv), _ptr(gn), ng, strides[0], _ptr(fv), _ptr(fn), strides[1], _ptr(bv),
            _ptr(bn), strides[2], ns, _ptr(sc), _ptr(lens), _ptr(pcs))
    total = lib().fdo_assemble(*args, None)
    out = np.zeros((max(total, 1), 3), np.float32)
    lib().fdo_assemble(*args, _ptr(out))
    off = np.zeros(ng + 1, np.int64)
    off[1:] = np.cumsum(lens)
    return off, out[:total], pcs

