"""ctypes binding of libfusedir.so (include/fusedir.h).

Argument marshalling only: every step of the fusion runs in the library's HIP
kernels.  Tensors are torch CUDA (ROCm) tensors; torch provides device memory
and streams.  If the library is missing or fails to load, every call raises:
there is no other implementation behind these names.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfusedir.so")

FD_OK, FD_E_INVAL, FD_E_UNSUPPORTED, FD_E_HIP, FD_E_NOMEM = range(5)
FD_F32, FD_F16 = 0, 1
FD_MODE_PLAIN, FD_MODE_LEARNED, FD_MODE_FPMVO = 0, 1, 2
FD_PROPOSAL_MLP, FD_PROPOSAL_GIVEN, FD_PROPOSAL_NAN = 0, 1, 2
FD_MLP_N_PARAMS = 161283
FD_FEATURE_DIM = 112
FD_NOALLOC_MAX_POINTS = 524288

EXPORTS = (
    "fd_params_init", "fd_context_create", "fd_context_reserve", "fd_context_destroy",
    "fd_fuse_directions", "fd_fuse_directions_noalloc", "fd_last_fallback_count", "fd_last_fallback_split",
    "fd_fuse_directions_batched",
    "fd_mlp_create", "fd_mlp_set_params", "fd_mlp_get_params", "fd_mlp_set_calibration",
    "fd_mlp_get_calibration", "fd_mlp_save", "fd_mlp_load", "fd_mlp_forward",
    "fd_mlp_loss_grad", "fd_mlp_train_step", "fd_mlp_destroy", "fd_features", "fd_autotune",
    "fd_tuned_shape", "fd_set_tuned_shape", "fd_profile_enable", "fd_profile_read", "fd_gabor_params_init",
    "fd_orientation_maps", "fd_fuse_volume", "fd_grow_params_init", "fd_grow_strands",
    "fd_link_segments", "fd_strand_offsets", "fd_assemble_strands", "fd_probe_read",
    "fd_last_error",
)

FD_STAGE_TILING, FD_STAGE_TOPK, FD_STAGE_FUSE, FD_STAGE_FEATURES, FD_STAGE_MLP, \
    FD_STAGE_REFINE, FD_STAGE_FALLBACK, FD_STAGE_BATCHED, FD_STAGE_GABOR, \
    FD_STAGE_GABOR_NORM, FD_STAGE_VOLUME_CLEAR, FD_STAGE_VOLUME_SCATTER, \
    FD_STAGE_VOLUME_FINAL, FD_STAGE_GROW, FD_STAGE_GROW_CROSS, FD_STAGE_LINK = range(16)
FD_SEED_GIVEN, FD_SEED_AWAY, FD_SEED_TOWARDS = 0, 1, 2
FD_MAX_GROW_STEPS = 4096
FD_MAX_VOLUME_DIM = 4096
FD_MAX_VOLUME_VOXELS = 1 << 30


class FdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fusedir error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("map_dtype", ctypes.c_int32), ("patch", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
        ("refine_step0", ctypes.c_float), ("top_k", ctypes.c_int32),
        ("z_near", ctypes.c_float), ("mode", ctypes.c_int32),
        ("mlp", ctypes.c_void_p), ("learned_iters", ctypes.c_int32),
        ("learned_step0", ctypes.c_float), ("fallback_cost", ctypes.c_float),
        ("proposal", ctypes.c_int32), ("proposal_dirs", ctypes.c_void_p),
        ("head_centre", ctypes.c_float * 3), ("vis_tau", ctypes.c_float),
        ("depth_maps", ctypes.c_void_p), ("fpmvo_lambda", ctypes.c_float),
        ("fpmvo_samples", ctypes.c_int32), ("fpmvo_delta", ctypes.c_float),
        ("stream", ctypes.c_void_p), ("ctx", ctypes.c_void_p),
    ]


class Scene(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_void_p), ("n_points", ctypes.c_int64),
        ("cams", ctypes.c_void_p), ("n_views", ctypes.c_int32),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("orient_maps", ctypes.c_void_p), ("conf_maps", ctypes.c_void_p),
        ("depth_maps", ctypes.c_void_p),
        ("dirs", ctypes.c_void_p), ("costs", ctypes.c_void_p),
        ("head_centre", ctypes.c_float * 3),
        ("proposal_dirs", ctypes.c_void_p),
    ]


class GaborParams(ctypes.Structure):
    _fields_ = [
        ("n_orient", ctypes.c_int32), ("radius", ctypes.c_int32),
        ("sigma_along", ctypes.c_float), ("sigma_across", ctypes.c_float),
        ("wavelength", ctypes.c_float), ("out_dtype", ctypes.c_int32),
        ("stream", ctypes.c_void_p), ("ctx", ctypes.c_void_p),
    ]


class VolumeGrid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("voxel", ctypes.c_float),
                ("dims", ctypes.c_int32 * 3)]


class GrowParams(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_float), ("max_steps", ctypes.c_int32),
        ("min_coherence", ctypes.c_float), ("max_bend_cos", ctypes.c_float),
        ("voxel_cap", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("seed_mode", ctypes.c_int32), ("centre", ctypes.c_float * 3),
        ("stream", ctypes.c_void_p), ("ctx", ctypes.c_void_p),
    ]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_lib = None


def lib():
    """Load libfusedir.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2604_05794_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, f32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                             ctypes.c_float)
    pp = ctypes.POINTER(Params)
    sig = {
        "fd_params_init": (None, [pp]),
        "fd_context_create": (ctypes.c_int, [ctypes.POINTER(P)]),
        "fd_context_reserve": (ctypes.c_int, [P, i64, i32, i32]),
        "fd_context_destroy": (None, [P]),
        "fd_fuse_directions": (ctypes.c_int, [P, i64, P, i32, P, P, pp, P, P]),
        "fd_fuse_directions_noalloc": (ctypes.c_int, [P, i64, P, i32, P, P, pp, P, P]),
        "fd_last_fallback_count": (ctypes.c_int, [P, P, ctypes.POINTER(i64)]),
        "fd_last_fallback_split": (ctypes.c_int, [P, P, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "fd_fuse_directions_batched": (ctypes.c_int, [ctypes.POINTER(Scene), i32, pp, P]),
        "fd_mlp_create": (ctypes.c_int, [ctypes.POINTER(P), u64]),
        "fd_mlp_set_params": (ctypes.c_int, [P, P]),
        "fd_mlp_get_params": (ctypes.c_int, [P, P]),
        "fd_mlp_set_calibration": (ctypes.c_int, [P, f32, f32]),
        "fd_mlp_get_calibration": (ctypes.c_int, [P, ctypes.POINTER(f32), ctypes.POINTER(f32)]),
        "fd_mlp_save": (ctypes.c_int, [P, ctypes.c_char_p]),
        "fd_mlp_load": (ctypes.c_int, [P, ctypes.c_char_p]),
        "fd_mlp_forward": (ctypes.c_int, [P, P, i64, P, P]),
        "fd_mlp_loss_grad": (ctypes.c_int, [P, P, P, i32, P, P, P]),
        "fd_mlp_train_step": (ctypes.c_int, [P, P, P, i32, ctypes.POINTER(Adam), P, P]),
        "fd_mlp_destroy": (None, [P]),
        "fd_features": (ctypes.c_int, [P, i64, P, i32, P, P, pp, P]),
        "fd_autotune": (ctypes.c_int, [P, ctypes.POINTER(Scene), i32, pp, ctypes.c_char_p]),
        "fd_tuned_shape": (ctypes.c_int, [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "fd_set_tuned_shape": (ctypes.c_int, [P, i32, i32]),
        "fd_profile_enable": (ctypes.c_int, [P, ctypes.c_int]),
        "fd_profile_read": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(i64)]),
        "fd_gabor_params_init": (None, [ctypes.POINTER(GaborParams)]),
        "fd_orientation_maps": (ctypes.c_int, [P, i32, i32, i32, ctypes.POINTER(GaborParams),
                                               P, P]),
        "fd_fuse_volume": (ctypes.c_int, [P, P, P, i64, ctypes.POINTER(VolumeGrid), P, P, P,
                                          P, P, P]),
        "fd_grow_params_init": (None, [ctypes.POINTER(GrowParams)]),
        "fd_grow_strands": (ctypes.c_int, [ctypes.POINTER(VolumeGrid), P, P, P, P, P, i32,
                                           ctypes.POINTER(GrowParams), P, P, P, P]),
        "fd_link_segments": (ctypes.c_int, [P, P, P, P, P, i32, f32, f32, P, P, P]),
        "fd_strand_offsets": (ctypes.c_int, [P, i32, P, P, i32, P, P, P, P, P]),
        "fd_assemble_strands": (ctypes.c_int, [P, P, i32, i32, P, P, i32, P, P, i32, i32, P, P,
                                               i64, P, P, P]),
        "fd_probe_read": (ctypes.c_int, [P, i64, i32, i32, P, P]),
        "fd_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc != FD_OK:
        raise FdError(rc, lib().fd_last_error().decode(errors="replace"))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_tensor(t, name, dtype=None, shape_tail=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} must have trailing shape {shape_tail}, got {tuple(t.shape)}")
    return t


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Library-owned workspace (fd_context)."""

    def __init__(self, max_points=0, max_views=0, max_scenes=0):
        h = ctypes.c_void_p()
        _check(lib().fd_context_create(ctypes.byref(h)))
        self.handle = h
        if max_points or max_scenes:
            self.reserve(max_points, max_views, max_scenes)

    def reserve(self, max_points, max_views=0, max_scenes=0):
        _check(lib().fd_context_reserve(self.handle, int(max_points), int(max_views),
                                        int(max_scenes)))

    def fallback_count(self, stream=None) -> int:
        out = ctypes.c_int64()
        _check(lib().fd_last_fallback_count(self.handle, _stream_handle(stream),
                                            ctypes.byref(out)))
        return int(out.value)

    def fallback_split(self, stream=None):
        """(listed, in place) full searches of the last learned call."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fd_last_fallback_split(self.handle, _stream_handle(stream),
                                            ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def tuned(self):
        """(chunk, grid) of the batched search (fd_tuned_shape)."""
        c, g = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fd_tuned_shape(self.handle, ctypes.byref(c), ctypes.byref(g)))
        return c.value, g.value

    def set_tuned(self, chunk, grid):
        """fd_set_tuned_shape."""
        _check(lib().fd_set_tuned_shape(self.handle, int(chunk), int(grid)))

    def profile(self, on=True):
        _check(lib().fd_profile_enable(self.handle, int(bool(on))))

    def stage_time(self, stage):
        """(total ms, launches) recorded for one FD_STAGE_* since profile()."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().fd_profile_read(self.handle, int(stage), ctypes.byref(ms),
                                     ctypes.byref(cnt)))
        return float(ms.value), int(cnt.value)

    def close(self):
        if self.handle:
            lib().fd_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(width, height, map_dtype, *, patch=5, n_candidates=128, refine_iters=8,
                refine_step0=0.0, top_k=5, z_near=1e-3, mode=FD_MODE_PLAIN, mlp=None,
                learned_iters=2, learned_step0=0.0, fallback_cost=math.inf,
                proposal=FD_PROPOSAL_MLP, proposal_dirs=None, head_centre=(0.0, 0.0, 0.0),
                depth_maps=None, vis_tau=5e-3, fpmvo_lambda=3.0, fpmvo_samples=5,
                fpmvo_delta=5e-3, stream=None, ctx: Optional[Context] = None) -> Params:
    p = Params()
    lib().fd_params_init(ctypes.byref(p))
    p.width, p.height = int(width), int(height)
    p.map_dtype = int(map_dtype)
    p.patch = int(patch)
    p.n_candidates = int(n_candidates)
    p.refine_iters = int(refine_iters)
    p.refine_step0 = float(refine_step0)
    p.top_k = int(top_k)
    p.z_near = float(z_near)
    p.mode = int(mode)
    p.mlp = mlp.handle if mlp is not None else None
    p.learned_iters = int(learned_iters)
    p.learned_step0 = float(learned_step0)
    p.fallback_cost = float(fallback_cost)
    p.proposal = int(proposal)
    p.proposal_dirs = proposal_dirs.data_ptr() if proposal_dirs is not None else None
    for k in range(3):
        p.head_centre[k] = float(head_centre[k])
    p.vis_tau = float(vis_tau)
    p.depth_maps = depth_maps.data_ptr() if depth_maps is not None else None
    p.fpmvo_lambda = float(fpmvo_lambda)
    p.fpmvo_samples = int(fpmvo_samples)
    p.fpmvo_delta = float(fpmvo_delta)
    p.stream = _stream_handle(stream).value
    p.ctx = ctx.handle.value if ctx is not None else None
    return p


def map_dtype_of(t: torch.Tensor) -> int:
    if t.dtype == torch.float16:
        return FD_F16
    if t.dtype == torch.float32:
        return FD_F32
    raise TypeError(f"maps must be float16 or float32, got {t.dtype}")


def _check_depth(depth, orient_maps):
    if depth is None:
        return
    _dev_tensor(depth, "depth_maps", orient_maps.dtype)
    if depth.shape != orient_maps.shape:
        raise ValueError("depth_maps must have the shape of orient_maps")


def fuse_directions(points, cams, orient_maps, conf_maps, *, dirs=None, costs=None,
                    noalloc=False, **kw):
    """fd_fuse_directions on torch tensors.

    points (N, 3) float32, cams (V, 16) float32, maps (V, H, W) float16 or
    float32 (same dtype), all on the current HIP device.  Keyword arguments
    are the fields of fd_params (see make_params).  Returns (dirs (N, 3),
    costs (N,)) float32, enqueued on `stream` (default: torch's current
    stream).  noalloc=True calls fd_fuse_directions_noalloc instead (plain
    mode, at most FD_NOALLOC_MAX_POINTS points; pass dirs and costs to
    allocate nothing here either).
    """
    _dev_tensor(points, "points", torch.float32, (3,))
    _dev_tensor(cams, "cams", torch.float32, (16,))
    _dev_tensor(orient_maps, "orient_maps")
    _dev_tensor(conf_maps, "conf_maps", orient_maps.dtype)
    if orient_maps.dim() != 3 or conf_maps.shape != orient_maps.shape:
        raise ValueError("orient_maps and conf_maps must both be (V, H, W)")
    V, H, W = orient_maps.shape
    if cams.shape[0] != V:
        raise ValueError(f"{cams.shape[0]} cameras for {V} maps")
    n = points.shape[0]
    if dirs is None:
        dirs = torch.empty((n, 3), dtype=torch.float32, device=points.device)
    if costs is None:
        costs = torch.empty((n,), dtype=torch.float32, device=points.device)
    _dev_tensor(dirs, "dirs", torch.float32, (3,))
    _dev_tensor(costs, "costs", torch.float32)
    _check_depth(kw.get("depth_maps"), orient_maps)
    p = make_params(W, H, map_dtype_of(orient_maps), **kw)
    fn = lib().fd_fuse_directions_noalloc if noalloc else lib().fd_fuse_directions
    _check(fn(_ptr(points), n, _ptr(cams), V, _ptr(orient_maps), _ptr(conf_maps),
              ctypes.byref(p), _ptr(dirs), _ptr(costs)))
    return dirs, costs


def _np_f32(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float32)


class MLP:
    """Direction-proposal network (fd_mlp): 112 -> 256 -> 256 -> 256 -> 3."""

    def __init__(self, seed=0, path=None):
        h = ctypes.c_void_p()
        _check(lib().fd_mlp_create(ctypes.byref(h), int(seed)))
        self.handle = h
        if path is not None:
            self.load(path)

    def set_params(self, params):
        import numpy as np
        p = _np_f32(params)
        assert p.size == FD_MLP_N_PARAMS
        _check(lib().fd_mlp_set_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        import numpy as np
        p = np.empty(FD_MLP_N_PARAMS, np.float32)
        _check(lib().fd_mlp_get_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def set_calibration(self, learned_step0, fallback_cost):
        _check(lib().fd_mlp_set_calibration(self.handle, float(learned_step0),
                                            float(fallback_cost)))

    def calibration(self):
        s0 = ctypes.c_float()
        tau = ctypes.c_float()
        _check(lib().fd_mlp_get_calibration(self.handle, ctypes.byref(s0), ctypes.byref(tau)))
        return float(s0.value), float(tau.value)

    def save(self, path):
        _check(lib().fd_mlp_save(self.handle, os.fsencode(path)))

    def load(self, path):
        _check(lib().fd_mlp_load(self.handle, os.fsencode(path)))

    def forward(self, feats, out=None, stream=None):
        """feats: (B, 112) bfloat16 CUDA tensor -> (B, 3) float32 unit directions."""
        _dev_tensor(feats, "feats", torch.bfloat16, (FD_FEATURE_DIM,))
        B = feats.shape[0]
        if out is None:
            out = torch.empty((B, 3), dtype=torch.float32, device=feats.device)
        _dev_tensor(out, "out", torch.float32, (3,))
        _check(lib().fd_mlp_forward(self.handle, _ptr(feats), B, _ptr(out),
                                    _stream_handle(stream)))
        return out

    def loss_grad(self, feats, targets, stream=None):
        _dev_tensor(feats, "feats", torch.bfloat16, (FD_FEATURE_DIM,))
        _dev_tensor(targets, "targets", torch.float32, (3,))
        grad = torch.empty(FD_MLP_N_PARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        _check(lib().fd_mlp_loss_grad(self.handle, _ptr(feats), _ptr(targets), feats.shape[0],
                                      _ptr(grad), _ptr(loss), _stream_handle(stream)))
        return loss, grad

    def train_step(self, feats, targets, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   loss=None, stream=None):
        _dev_tensor(feats, "feats", torch.bfloat16, (FD_FEATURE_DIM,))
        _dev_tensor(targets, "targets", torch.float32, (3,))
        opt = Adam(float(lr), float(beta1), float(beta2), float(eps))
        _check(lib().fd_mlp_train_step(self.handle, _ptr(feats), _ptr(targets), feats.shape[0],
                                       ctypes.byref(opt), _ptr(loss), _stream_handle(stream)))
        return loss

    def close(self):
        if self.handle:
            lib().fd_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(points, cams, orient_maps, conf_maps, head_centre=(0.0, 0.0, 0.0), out=None,
             stream=None, z_near=1e-3, depth_maps=None, vis_tau=5e-3):
    """fd_features: (N, 112) bfloat16 proposal-network inputs, point order."""
    _dev_tensor(points, "points", torch.float32, (3,))
    _dev_tensor(cams, "cams", torch.float32, (16,))
    _dev_tensor(orient_maps, "orient_maps")
    _dev_tensor(conf_maps, "conf_maps", orient_maps.dtype)
    V, H, W = orient_maps.shape
    n = points.shape[0]
    if out is None:
        out = torch.empty((n, FD_FEATURE_DIM), dtype=torch.bfloat16, device=points.device)
    _check_depth(depth_maps, orient_maps)
    p = make_params(W, H, map_dtype_of(orient_maps), head_centre=head_centre, stream=stream,
                    z_near=z_near, depth_maps=depth_maps, vis_tau=vis_tau)
    _check(lib().fd_features(_ptr(points), n, _ptr(cams), V, _ptr(orient_maps), _ptr(conf_maps),
                             ctypes.byref(p), _ptr(out)))
    return out


def orientation_maps(frames, *, n_orient=32, radius=8, sigma_along=2.4, sigma_across=1.8,
                     wavelength=4.0, out_dtype=torch.float16, theta=None, conf=None,
                     stream=None, ctx: Optional["Context"] = None):
    """fd_orientation_maps: (V, H, W) float32 grey frames -> (theta, conf)
    maps of out_dtype, the inputs of fuse_directions."""
    _dev_tensor(frames, "frames", torch.float32)
    if frames.dim() != 3:
        raise ValueError("frames must be (n_frames, height, width)")
    V, H, W = frames.shape
    dt = {torch.float16: FD_F16, torch.float32: FD_F32}.get(out_dtype)
    if dt is None:
        raise TypeError("out_dtype must be torch.float16 or torch.float32")
    if theta is None:
        theta = torch.empty((V, H, W), dtype=out_dtype, device=frames.device)
    if conf is None:
        conf = torch.empty((V, H, W), dtype=out_dtype, device=frames.device)
    _dev_tensor(theta, "theta", out_dtype)
    _dev_tensor(conf, "conf", out_dtype)
    if theta.shape != frames.shape or conf.shape != frames.shape:
        raise ValueError("theta and conf must have the frames' shape")
    p = GaborParams()
    lib().fd_gabor_params_init(ctypes.byref(p))
    p.n_orient, p.radius = n_orient, radius
    p.sigma_along, p.sigma_across, p.wavelength = sigma_along, sigma_across, wavelength
    p.out_dtype = dt
    p.stream = _stream_handle(stream).value
    p.ctx = ctx.handle.value if ctx is not None else None
    _check(lib().fd_orientation_maps(_ptr(frames), V, W, H, ctypes.byref(p), _ptr(theta),
                                     _ptr(conf)))
    return theta, conf


def fuse_volume(points, dirs, origin, voxel, dims, *, weights=None, occ=None, dir_out=None,
                coherence=None, tensor=False, stream=None, ctx: Optional["Context"] = None):
    """fd_fuse_volume: occupancy (nz, ny, nx) uint32 (as int32 storage),
    orientation (nz, ny, nx, 3) float32, coherence (nz, ny, nx) float32 and,
    with tensor=True, the sums (nz, ny, nx, 6) float64."""
    _dev_tensor(points, "points", torch.float32, (3,))
    _dev_tensor(dirs, "dirs", torch.float32, (3,))
    n = points.shape[0]
    if dirs.shape[0] != n:
        raise ValueError("points and dirs must have the same length")
    if weights is not None:
        _dev_tensor(weights, "weights", torch.float32)
        if weights.shape != (n,):
            raise ValueError("weights must be (n_points,)")
    nx, ny, nz = (int(x) for x in dims)
    dev = points.device
    shape = (nz, ny, nx)
    g = VolumeGrid()
    for a in range(3):
        g.origin[a] = float(origin[a])
    g.voxel = float(voxel)
    g.dims[0], g.dims[1], g.dims[2] = nx, ny, nz
    if not all(1 <= x <= FD_MAX_VOLUME_DIM for x in (nx, ny, nz)) or \
            nx * ny * nz > FD_MAX_VOLUME_VOXELS:
        # the library rejects the grid before it looks at any output
        _check(lib().fd_fuse_volume(_ptr(points), _ptr(dirs), _ptr(weights), n, ctypes.byref(g),
                                    _stream_handle(stream), None, None, None, None, None))
    if occ is None:
        occ = torch.empty(shape, dtype=torch.int32, device=dev)
    if dir_out is None:
        dir_out = torch.empty(shape + (3,), dtype=torch.float32, device=dev)
    if coherence is None:
        coherence = torch.empty(shape, dtype=torch.float32, device=dev)
    _dev_tensor(occ, "occ", torch.int32)
    _dev_tensor(dir_out, "dir_out", torch.float32)
    _dev_tensor(coherence, "coherence", torch.float32)
    if occ.numel() != nx * ny * nz or dir_out.numel() != 3 * nx * ny * nz or \
            coherence.numel() != nx * ny * nz:
        raise ValueError("output sizes do not match the grid")
    T = torch.empty(shape + (6,), dtype=torch.float64, device=dev) if tensor else None
    _check(lib().fd_fuse_volume(_ptr(points), _ptr(dirs), _ptr(weights), n, ctypes.byref(g),
                                _stream_handle(stream), ctx.handle if ctx is not None else None,
                                _ptr(occ), _ptr(dir_out), _ptr(coherence), _ptr(T)))
    return (occ, dir_out, coherence, T) if tensor else (occ, dir_out, coherence)


def _grid_struct(origin, voxel, dims):
    g = VolumeGrid()
    for a in range(3):
        g.origin[a] = float(origin[a])
    g.voxel = float(voxel)
    g.dims[0], g.dims[1], g.dims[2] = (int(x) for x in dims)
    return g


def grow_strands(occ, dir_vol, coherence, origin, voxel, dims, seeds, seed_dirs=None, *,
                 crossings, seed_mode=FD_SEED_GIVEN, centre=(0.0, 0.0, 0.0), step=1e-3,
                 max_steps=200, min_coherence=0.2, max_bend_cos=math.cos(math.radians(30.0)),
                 voxel_cap=8, batch=4096, stream=None, ctx: Optional["Context"] = None):
    """fd_grow_strands: traces from seeds through a volume (occ int32/uint32
    storage, dir (.., 3) float32, coherence float32, as fuse_volume returns
    them); crossings (nv,) int32 storage is read and updated.  Returns verts
    (n, max_steps + 1, 3), n_verts (n,), last_dir (n, 3)."""
    _dev_tensor(occ, "occ", torch.int32)
    _dev_tensor(dir_vol, "dir", torch.float32)
    _dev_tensor(coherence, "coherence", torch.float32)
    _dev_tensor(crossings, "crossings", torch.int32)
    nv = int(dims[0]) * int(dims[1]) * int(dims[2])
    if occ.numel() != nv or dir_vol.numel() != 3 * nv or coherence.numel() != nv or \
            crossings.numel() != nv:
        raise ValueError("volume arrays do not match the grid")
    _dev_tensor(seeds, "seeds", torch.float32, (3,))
    n = seeds.shape[0]
    if seed_dirs is not None:
        _dev_tensor(seed_dirs, "seed_dirs", torch.float32, (3,))
        if seed_dirs.shape[0] != n:
            raise ValueError("seed_dirs must match seeds")
    if not 1 <= int(max_steps) <= FD_MAX_GROW_STEPS:
        raise FdError(FD_E_INVAL, f"max_steps must be in [1, {FD_MAX_GROW_STEPS}]")
    dev = seeds.device
    verts = torch.empty((n, int(max_steps) + 1, 3), dtype=torch.float32, device=dev)
    n_verts = torch.empty((n,), dtype=torch.int32, device=dev)
    last = torch.empty((n, 3), dtype=torch.float32, device=dev)
    p = GrowParams()
    lib().fd_grow_params_init(ctypes.byref(p))
    p.step, p.max_steps, p.min_coherence = float(step), int(max_steps), float(min_coherence)
    p.max_bend_cos, p.voxel_cap, p.batch = float(max_bend_cos), int(voxel_cap), int(batch)
    p.seed_mode = int(seed_mode)
    for a in range(3):
        p.centre[a] = float(centre[a])
    p.stream = _stream_handle(stream).value
    p.ctx = ctx.handle.value if ctx is not None else None
    g = _grid_struct(origin, voxel, dims)
    _check(lib().fd_grow_strands(ctypes.byref(g), _ptr(occ), _ptr(dir_vol), _ptr(coherence),
                                 _ptr(seeds), _ptr(seed_dirs), n, ctypes.byref(p),
                                 _ptr(crossings), _ptr(verts), _ptr(n_verts), _ptr(last)))
    return verts, n_verts, last


def link_segments(starts, start_dirs, ends, end_dirs, flags, max_dist, min_cos, *, succ=None,
                  stream=None, ctx: Optional["Context"] = None):
    """fd_link_segments (Eq. 13): succ (n,) int32, the accepted successor of
    each piece or -1."""
    for t_, nm in ((starts, "starts"), (start_dirs, "start_dirs"), (ends, "ends"),
                   (end_dirs, "end_dirs")):
        _dev_tensor(t_, nm, torch.float32, (3,))
    _dev_tensor(flags, "flags", torch.uint8)
    n = starts.shape[0]
    if any(x.shape[0] != n for x in (start_dirs, ends, end_dirs, flags)):
        raise ValueError("piece arrays must have the same length")
    if succ is None:
        succ = torch.empty((n,), dtype=torch.int32, device=starts.device)
    _dev_tensor(succ, "succ", torch.int32)
    _check(lib().fd_link_segments(_ptr(starts), _ptr(start_dirs), _ptr(ends), _ptr(end_dirs),
                                  _ptr(flags), n, float(max_dist), float(min_cos),
                                  _stream_handle(stream), ctx.handle if ctx is not None else None,
                                  _ptr(succ)))
    return succ


def assemble_strands(guide, fwd, bwd, succ, *, out=None, stream=None,
                     ctx: Optional["Context"] = None):
    """Strands from linked pieces (fd_strand_offsets, then
    fd_assemble_strands): guide, fwd, bwd are (verts, n_verts, last_dir)
    as grow_strands returns them; succ over the guide pieces then the
    segments.  Returns (offsets (n_guide + 1,) int64, verts, pieces
    (n_guide,) int32).  Without `out` the total is read back to size the
    output and verts is (total, 3); with `out` ((capacity, 3) float32)
    nothing is read back, rows past the capacity are not written and verts
    is `out` itself."""
    gv, gn = guide[0], guide[1]
    fv, fn = fwd[0], fwd[1]
    bv, bn = bwd[0], bwd[1]
    for t_, nm in ((gv, "guide verts"), (fv, "forward verts"), (bv, "backward verts")):
        _dev_tensor(t_, nm, torch.float32)
    for t_, nm in ((gn, "guide n_verts"), (fn, "forward n_verts"), (bn, "backward n_verts"),
                   (succ, "succ")):
        _dev_tensor(t_, nm, torch.int32)
    ng, ns = gn.shape[0], fn.shape[0]
    if bn.shape[0] != ns or succ.shape[0] != ng + ns:
        raise ValueError("segment halves and links must match the piece counts")
    dev = gv.device
    off = torch.empty(ng + 1, dtype=torch.int64, device=dev)
    pieces = torch.empty(max(ng, 1), dtype=torch.int32, device=dev)
    sh = _stream_handle(stream)
    ch = ctx.handle if ctx is not None else None
    _check(lib().fd_strand_offsets(_ptr(gn), ng, _ptr(fn), _ptr(bn), ns, _ptr(succ), sh, ch,
                                   _ptr(off), _ptr(pieces)))
    if out is None:
        total = int(off[-1].item())
        buf = torch.empty((max(total, 1), 3), dtype=torch.float32, device=dev)
    else:
        _dev_tensor(out, "out", torch.float32, (3,))
        buf, total = out, out.shape[0]
    _check(lib().fd_assemble_strands(_ptr(gv), _ptr(gn), ng, gv.shape[1], _ptr(fv), _ptr(fn),
                                     fv.shape[1], _ptr(bv), _ptr(bn), bv.shape[1], ns, _ptr(succ),
                                     _ptr(off), total, sh, ch, _ptr(buf)))
    return off, (buf[:total] if out is None else buf), pieces[:ng]


def _scene_struct(sc):
    """sc: dict with points, cams, orient_maps, conf_maps, dirs, costs and
    optional head_centre and depth_maps (CUDA tensors)."""
    s = Scene()
    pts, cams, th, cf = sc["points"], sc["cams"], sc["orient_maps"], sc["conf_maps"]
    _dev_tensor(pts, "points", torch.float32, (3,))
    _dev_tensor(cams, "cams", torch.float32, (16,))
    _dev_tensor(th, "orient_maps")
    _dev_tensor(cf, "conf_maps", th.dtype)
    _dev_tensor(sc["dirs"], "dirs", torch.float32, (3,))
    _dev_tensor(sc["costs"], "costs", torch.float32)
    V, H, W = th.shape
    s.points = pts.data_ptr()
    s.n_points = pts.shape[0]
    s.cams = cams.data_ptr()
    s.n_views = V
    s.width, s.height = W, H
    s.orient_maps = th.data_ptr()
    s.conf_maps = cf.data_ptr()
    dep = sc.get("depth_maps")
    _check_depth(dep, th)
    s.depth_maps = dep.data_ptr() if dep is not None else None
    s.dirs = sc["dirs"].data_ptr()
    s.costs = sc["costs"].data_ptr()
    hc = sc.get("head_centre", (0.0, 0.0, 0.0))
    for k in range(3):
        s.head_centre[k] = float(hc[k])
    prop = sc.get("proposal_dirs")
    if prop is not None:
        _dev_tensor(prop, "proposal_dirs", torch.float32, (3,))
        if prop.shape[0] != pts.shape[0]:
            raise ValueError("proposal_dirs must have one row per point")
    s.proposal_dirs = prop.data_ptr() if prop is not None else None
    return s, map_dtype_of(th)


def _scene_array(scenes):
    arr = (Scene * max(1, len(scenes)))()
    dt = None
    for k, sc in enumerate(scenes):
        arr[k], d = _scene_struct(sc)
        if dt is not None and d != dt:
            raise TypeError("all scenes of a batch need the same map dtype")
        dt = d
    return arr, (FD_F16 if dt is None else dt)


def fuse_batched(scenes, ctx: Context, **kw):
    """fd_fuse_directions_batched: scenes is a list of dicts (points, cams,
    orient_maps, conf_maps, dirs, costs[, head_centre]); outputs are written
    into each scene's dirs / costs."""
    arr, dt = _scene_array(scenes)
    p = make_params(1, 1, dt, ctx=ctx, **kw)
    _check(lib().fd_fuse_directions_batched(arr, len(scenes), ctypes.byref(p), ctx.handle))


def autotune(scenes, ctx: Context, cache_path=None, **kw):
    """fd_autotune on sample scenes (same form as fuse_batched)."""
    arr, dt = _scene_array(scenes)
    p = make_params(1, 1, dt, ctx=ctx, **kw)
    _check(lib().fd_autotune(ctx.handle, arr, len(scenes), ctypes.byref(p),
                             os.fsencode(cache_path) if cache_path else None))


def probe_read(buf, reps, blocks, sink=None, stream=None):
    """fd_probe_read: every one of `blocks` workgroups reads the whole device
    buffer `buf` (a multiple of 16 bytes) `reps` times."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    nbytes = buf.numel() * buf.element_size()
    if sink is None:
        sink = torch.empty(int(blocks) * 256, dtype=torch.int32, device=buf.device)
    _check(lib().fd_probe_read(_ptr(buf), nbytes, int(reps), int(blocks), _ptr(sink),
                               _stream_handle(stream)))
    return sink
