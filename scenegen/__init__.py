"""Seeded synthetic hair scenes: strands, points, cameras, orientation maps.

Input generation only.  This module holds none of the direction-fusion
arithmetic: it grows strand polylines on a spherical scalp, samples points on
them, places pinhole cameras on an orbit and renders each view's orientation
(angle of the strand's image, in [0, pi)) and confidence maps with a z-buffer
(``raster.c``), then adds von Mises orientation noise and outlier pixels.  The
oracle and the GPU library both read what it writes; neither is imported
here.

Units: metres, world z up, scalp sphere of radius 0.10 m at the origin.
Camera record (16 float32): fx, fy, cx, cy, R[9] (row-major, world->camera),
t[3]; OpenCV axes (x right, y down, z forward); texel (i, j) centred on pixel
coordinate (i, j); principal point ((W-1)/2, (H-1)/2).

The recipes are the workloads the paper's method is exercised on here; the
paper's own evaluation data (rendered USC-HairSalon/Hair20K hairstyles and
captured videos) is not available, so these scenes stand in for it.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libscenegen.so")

SCALP_RADIUS = 0.10
ORBIT_RADIUS = 0.6
ELEVATION_DEG = 15.0
HFOV_DEG = 50.0
POLY_STEP = 0.5e-3


def build() -> str:
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
                    "-o", tmp, os.path.join(_HERE, "raster.c"), "-lm"], check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _raster_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.scenegen_raster.restype = ctypes.c_int
        L.scenegen_raster.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_double, P, P, P, P,
                                      ctypes.c_int32]
        L.scenegen_visible_views.restype = ctypes.c_int
        L.scenegen_visible_views.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, P, ctypes.c_double, P,
                                             ctypes.c_int32]
        _lib = L
    return _lib


@dataclasses.dataclass
class Scene:
    points: np.ndarray          # (N, 3) float32
    gt: np.ndarray              # (N, 3) float32 unit tangents of the source segment
    cams: np.ndarray            # (V, 16) float32
    theta: np.ndarray           # (V, H, W) float32 or float16, radians in [0, pi]
    conf: np.ndarray            # (V, H, W) same dtype, [0, 1]
    depth: Optional[np.ndarray]  # (V, H, W) camera-space Z (map dtype), +inf background
    head_centre: np.ndarray     # (3,) float32
    meta: dict

    @property
    def n_points(self):
        return len(self.points)

    @property
    def n_views(self):
        return self.cams.shape[0]

    @property
    def height(self):
        return self.theta.shape[1]

    @property
    def width(self):
        return self.theta.shape[2]

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.points, self.cams, self.theta, self.conf):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


# ---- cameras ------------------------------------------------------------------

def look_at_camera(centre, target, width, height, hfov_deg=HFOV_DEG, up=(0.0, 0.0, 1.0)):
    """16-float pinhole record looking from ``centre`` at ``target``."""
    centre = np.asarray(centre, np.float64)
    fwd = np.asarray(target, np.float64) - centre
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(fwd, np.array([1.0, 0.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ centre
    f = width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))
    cam = np.concatenate([[f, f, (width - 1) / 2.0, (height - 1) / 2.0], R.ravel(), t])
    return cam.astype(np.float32)


def orbit_cameras(n_views, width, height, arc_deg=360.0, radius=ORBIT_RADIUS,
                  elevation_deg=ELEVATION_DEG, hfov_deg=HFOV_DEG):
    """Cameras on a horizontal orbit around the origin.  A 360 degree orbit
    spaces them evenly; a partial arc spans [-arc/2, +arc/2] inclusive."""
    if arc_deg >= 360.0:
        az = np.arange(n_views) * (360.0 / n_views)
    elif n_views == 1:
        az = np.zeros(1)
    else:
        az = np.linspace(-arc_deg / 2.0, arc_deg / 2.0, n_views)
    el = math.radians(elevation_deg)
    cams = []
    for a in np.radians(az):
        c = radius * np.array([math.cos(el) * math.cos(a), math.cos(el) * math.sin(a),
                               math.sin(el)])
        cams.append(look_at_camera(c, (0.0, 0.0, 0.0), width, height, hfov_deg))
    return np.stack(cams)


# ---- strands ------------------------------------------------------------------

def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def grow_strands(rng, n_strands, kind_mix, length_mm=(60.0, 150.0), helix_r_mm=(5.0, 20.0),
                 pitch_mm=(10.0, 40.0), wave_amp_mm=(5.0, 15.0), wave_len_mm=(20.0, 60.0),
                 max_polar_deg=100.0, scalp_radius=SCALP_RADIUS):
    """Polylines with ~0.5 mm vertex spacing.

    Roots are uniform by area on the scalp cap (polar angle <= max_polar_deg
    from +z).  The centreline leaves along the surface normal n and bends
    towards a fall direction g (down and slightly outward):
    a(s) = normalize((1 - s/L) n + (s/L) g).  A helix winds around it in a
    parallel-transported frame with a random phase; a wave oscillates along
    the frame's first axis; a straight strand is the centreline.  Strand
    length L is the length of the strand itself (helix or wave included).  ``kind_mix`` is
    a dict kind -> fraction over {"helix", "wavy", "straight"}.
    Returns (verts (M, 3) float64, offsets (S + 1,) int64).
    """
    kinds = list(kind_mix)
    probs = np.array([kind_mix[k] for k in kinds], np.float64)
    probs /= probs.sum()
    kind_idx = rng.choice(len(kinds), size=n_strands, p=probs)
    cos_max = math.cos(math.radians(max_polar_deg))
    cz = rng.uniform(cos_max, 1.0, n_strands)
    az = rng.uniform(0.0, 2 * math.pi, n_strands)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    n = np.stack([sz * np.cos(az), sz * np.sin(az), cz], 1)
    g = _unit(np.stack([0.4 * np.cos(az), 0.4 * np.sin(az), -np.ones_like(az)], 1))
    L = rng.uniform(*length_mm, n_strands) * 1e-3
    r = rng.uniform(*helix_r_mm, n_strands) * 1e-3
    pitch = rng.uniform(*pitch_mm, n_strands) * 1e-3
    amp = rng.uniform(*wave_amp_mm, n_strands) * 1e-3
    wlen = rng.uniform(*wave_len_mm, n_strands) * 1e-3
    phase = rng.uniform(0.0, 2 * math.pi, n_strands)
    # arc-length stretch of each shape relative to its centreline
    stretch = np.ones(n_strands)
    kname = np.array(kinds)[kind_idx]
    hel = kname == "helix"
    stretch[hel] = np.sqrt(1.0 + (2 * math.pi * r[hel] / pitch[hel]) ** 2)
    wav = kname == "wavy"
    tt = np.linspace(0, 2 * math.pi, 64, endpoint=False)
    kk = (2 * math.pi * amp[wav] / wlen[wav])[:, None]
    stretch[wav] = np.mean(np.sqrt(1.0 + (kk * np.cos(tt)[None, :]) ** 2), axis=1)
    Lc = L / stretch
    nv = np.maximum(2, np.ceil(L / POLY_STEP).astype(np.int64) + 1)
    J = int(nv.max())
    j = np.arange(J)[None, :]
    ds = Lc / (nv - 1)
    s = np.minimum(j, (nv - 1)[:, None]) * ds[:, None]          # (S, J), clamped past the end
    w = (s / Lc[:, None])[..., None]
    a = _unit((1 - w) * n[:, None, :] + w * g[:, None, :])       # (S, J, 3)
    # the centreline lies in the plane of n and g, so a parallel-transported
    # normal frame is the plane normal b and a x b
    c = scalp_radius * n[:, None, :] + np.concatenate(
        [np.zeros((n_strands, 1, 3)), np.cumsum(0.5 * (a[:, 1:] + a[:, :-1]) * ds[:, None, None],
                                                 axis=1)], axis=1)
    b = _unit(np.cross(n, g))[:, None, :]
    e2 = np.cross(a, b)
    om = 2 * math.pi / pitch
    ang = om[:, None] * s + phase[:, None]
    off_h = r[:, None, None] * (np.cos(ang)[..., None] * b + np.sin(ang)[..., None] * e2)
    off_w = amp[:, None, None] * np.sin(2 * math.pi * s / wlen[:, None] + phase[:, None])[..., None] * b
    off = np.where(hel[:, None, None], off_h, np.where(wav[:, None, None], off_w, 0.0))
    off = off - off[:, :1, :]
    x = c + off
    valid = j < nv[:, None]
    verts = [x[valid]]
    offs = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
    return verts[0], offs


def sample_points(rng, verts, offs, n_points, jitter_sigma):
    """Points uniform by arc length over all strand segments, with isotropic
    Gaussian jitter; the tangent of the source segment is the ground truth."""
    seg_start = np.ones(len(verts), bool)
    seg_start[offs[1:] - 1] = False          # last vertex of a strand starts no segment
    idx = np.nonzero(seg_start)[0]
    d = verts[idx + 1] - verts[idx]
    ln = np.linalg.norm(d, axis=1)
    cum = np.cumsum(ln)
    u = rng.uniform(0.0, cum[-1], n_points)
    k = np.searchsorted(cum, u, side="right")
    k = np.minimum(k, len(idx) - 1)
    before = np.where(k > 0, cum[np.maximum(k - 1, 0)], 0.0)
    frac = ((u - before) / ln[k])[:, None]
    p = verts[idx[k]] + frac * d[k]
    p = p + rng.normal(0.0, jitter_sigma, p.shape) if jitter_sigma > 0 else p
    gt = d[k] / ln[k][:, None]
    gt = np.where(gt[:, 2:3] < 0, -gt, gt)
    return p.astype(np.float32), gt.astype(np.float32)


# ---- maps ---------------------------------------------------------------------

def render_maps(rng_views, verts, offs, cams, width, height, kappa, outlier_frac,
                dtype, head_radius=SCALP_RADIUS, n_threads=0):
    """Orientation, confidence and depth maps of every view.

    Covered texels get the strand image angle, then (if kappa is not None)
    von Mises noise of concentration kappa on the angle and confidence
    ~ U(0.6, 1); a fraction ``outlier_frac`` of covered texels is replaced by
    angle ~ U[0, pi) and confidence ~ U(0, 1).  kappa None means noise-free:
    confidence 1 and the exact angle.  Background: angle 0, confidence 0.
    Depth: camera-space Z of the nearest strand or head surface, +inf where
    the ray meets neither (float32; the caller casts it with the maps).
    """
    V = len(cams)
    v32 = np.ascontiguousarray(verts, np.float32)
    theta = np.empty((V, height, width), np.float32)
    depth = np.empty((V, height, width), np.float32)
    cov = np.empty((V, height, width), np.uint8)
    cams = np.ascontiguousarray(cams, np.float32)
    offs = np.ascontiguousarray(offs, np.int64)
    _raster_lib().scenegen_raster(v32.ctypes.data, offs.ctypes.data, len(offs) - 1,
                                  cams.ctypes.data, V, width, height, float(head_radius),
                                  theta.ctypes.data, depth.ctypes.data, cov.ctypes.data, None,
                                  int(n_threads))
    conf = np.zeros((V, height, width), np.float32)
    for v in range(V):
        rng = rng_views[v]
        m = cov[v].astype(bool)
        nc = int(m.sum())
        th = theta[v][m].astype(np.float64)
        if kappa is None:
            c = np.ones(nc)
        else:
            th = np.mod(th + rng.vonmises(0.0, kappa, nc), math.pi)
            c = rng.uniform(0.6, 1.0, nc)
        if outlier_frac > 0:
            o = rng.uniform(0.0, 1.0, nc) < outlier_frac
            no = int(o.sum())
            th[o] = rng.uniform(0.0, math.pi, no)
            c[o] = rng.uniform(0.0, 1.0, no)
        theta[v][m] = th
        conf[v][m] = c
    if dtype == np.float16:
        theta16 = theta.astype(np.float16)
        conf16 = conf.astype(np.float16)
        return theta16, conf16, depth
    return theta, conf, depth


VIS_TAU = 5e-3   # visibility tolerance: half the paper's 2 Delta = 10 mm depth range


def visible_views(points, cams, depth, tau=VIS_TAU, n_threads=0):
    """Number of views in which each point is visible (in front, inside the
    image, within tau of the nearest-texel depth)."""
    pts = np.ascontiguousarray(points, np.float32)
    cams = np.ascontiguousarray(cams, np.float32)
    dep = np.ascontiguousarray(depth, np.float32)
    V, H, W = dep.shape
    out = np.empty(len(pts), np.int32)
    _raster_lib().scenegen_visible_views(pts.ctypes.data, len(pts), cams.ctypes.data, V, W, H,
                                         dep.ctypes.data, float(tau), out.ctypes.data,
                                         int(n_threads))
    return out


def render_images(rng, verts, offs, cams, width, height, noise=0.02,
                  head_radius=SCALP_RADIUS, n_threads=0):
    """Grey-level frames of the strands (the input of orientation extraction):
    each strand has its own albedo U(0.35, 1), the scalp 0.15, the background
    0, plus Gaussian noise of std `noise`; z-buffered like the maps, so the
    frames and the maps of a scene agree texel for texel."""
    V = len(cams)
    v32 = np.ascontiguousarray(verts, np.float32)
    theta = np.empty((V, height, width), np.float32)
    depth = np.empty((V, height, width), np.float32)
    cov = np.empty((V, height, width), np.uint8)
    sid = np.empty((V, height, width), np.int32)
    cams = np.ascontiguousarray(cams, np.float32)
    offs = np.ascontiguousarray(offs, np.int64)
    _raster_lib().scenegen_raster(v32.ctypes.data, offs.ctypes.data, len(offs) - 1,
                                  cams.ctypes.data, V, width, height, float(head_radius),
                                  theta.ctypes.data, depth.ctypes.data, cov.ctypes.data,
                                  sid.ctypes.data, int(n_threads))
    albedo = rng.uniform(0.35, 1.0, len(offs) - 1).astype(np.float32)
    img = np.where(sid >= 0, albedo[np.maximum(sid, 0)], 0.0).astype(np.float32)
    img[(sid < 0) & np.isfinite(depth)] = 0.15
    if noise > 0:
        img += rng.normal(0.0, noise, img.shape).astype(np.float32)
    return img


def make_frames(recipe, seed, n_threads=0):
    """The strands and cameras of `make_scene(recipe, seed)` as grey-level
    frames (V, H, W) float32, with the noise-free strand angle of every
    texel (V, H, W, radians in [0, pi)) and the strand coverage (V, H, W
    bool) for reference, and the cameras."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    r = dict(recipe)
    ss = np.random.SeedSequence(int(seed))
    s_strands, _, _ = ss.spawn(3)
    rng_s = np.random.Generator(np.random.PCG64(s_strands))
    verts, offs = grow_strands(
        rng_s, r["n_strands"], r["kinds"],
        helix_r_mm=r.get("helix_r_mm", (5.0, 20.0)), pitch_mm=r.get("pitch_mm", (10.0, 40.0)),
        wave_amp_mm=r.get("wave_amp_mm", (5.0, 15.0)),
        wave_len_mm=r.get("wave_len_mm", (20.0, 60.0)),
        length_mm=r.get("length_mm", (60.0, 150.0)))
    res = r["res"]
    cams = orbit_cameras(r["n_views"], res, res, r["arc_deg"])
    rng_f = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 7])))
    hr = r.get("head_radius", SCALP_RADIUS)
    frames = render_images(rng_f, verts, offs, cams, res, res, noise=r.get("frame_noise", 0.02),
                           head_radius=hr, n_threads=n_threads)
    theta, conf, _ = render_maps([None] * len(cams), verts, offs, cams, res, res, None, 0.0,
                                 np.float32, head_radius=hr, n_threads=n_threads)
    return frames, theta, conf > 0, cams


# ---- recipes ------------------------------------------------------------------

RECIPES = {
    # 10k points on 200 helical strands, 12 cameras on a 120 degree arc,
    # 256^2 float32 maps, kappa 50, no outliers; 3x3 patch, 48 candidates.
    "tiny": dict(n_points=10_000, n_strands=200, kinds={"helix": 1.0},
                 helix_r_mm=(5.0, 20.0), pitch_mm=(10.0, 40.0), n_views=12, arc_deg=120.0,
                 res=256, dtype="f32", kappa=50.0, outliers=0.0, jitter=2e-3,
                 patch=3, n_candidates=48, refine_iters=8),
    # 500k points on 20k strands (half straight, half wavy), 64 cameras on a
    # 360 degree orbit, 1024^2 float16 maps, kappa 50, 10% outlier texels;
    # 5x5 patch, 128 candidates, 8 refinement iterations.
    "realistic": dict(n_points=500_000, n_strands=20_000, kinds={"straight": 0.5, "wavy": 0.5},
                      wave_amp_mm=(5.0, 15.0), wave_len_mm=(20.0, 60.0), n_views=64,
                      arc_deg=360.0, res=1024, dtype="f16", kappa=50.0, outliers=0.10,
                      jitter=2e-3, patch=5, n_candidates=128, refine_iters=8),
    # one head of the hard set: tight curls, 128 cameras, kappa 10, 30% outliers
    "curls": dict(n_points=250_000, n_strands=8_000, kinds={"helix": 1.0},
                  helix_r_mm=(2.0, 6.0), pitch_mm=(4.0, 10.0), n_views=128, arc_deg=360.0,
                  res=1024, dtype="f16", kappa=10.0, outliers=0.30, jitter=2e-3,
                  patch=5, n_candidates=128, refine_iters=8),
}


def batched_recipes(n_scenes=16):
    """Uneven hairstyles for one batched launch: scene i has
    N_i = round(50k * 16^(i/15)), V_i = 32 + 32 * (5i mod 4) views and
    resolution [512, 768, 1024][7i mod 3], otherwise the realistic recipe."""
    out = []
    for i in range(n_scenes):
        r = dict(RECIPES["realistic"])
        r["n_points"] = int(round(50_000 * 16 ** (i / 15)))
        r["n_strands"] = max(1000, r["n_points"] // 25)
        r["n_views"] = 32 + 32 * ((5 * i) % 4)
        r["res"] = [512, 768, 1024][(7 * i) % 3]
        out.append(r)
    return out


def make_scene(recipe, seed, scale_points=1.0, n_threads=0) -> Scene:
    """Build one scene from a recipe dict (or a RECIPES key).  Points lie on
    the visible outer layer of the hair (seen in at least two views) unless
    the recipe sets outer=False, which samples the whole hair volume."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    r = dict(recipe)
    ss = np.random.SeedSequence(int(seed))
    s_strands, s_points, s_views = ss.spawn(3)
    rng_s = np.random.Generator(np.random.PCG64(s_strands))
    rng_p = np.random.Generator(np.random.PCG64(s_points))
    rng_v = [np.random.Generator(np.random.PCG64(x)) for x in s_views.spawn(r["n_views"])]
    verts, offs = grow_strands(
        rng_s, r["n_strands"], r["kinds"],
        helix_r_mm=r.get("helix_r_mm", (5.0, 20.0)), pitch_mm=r.get("pitch_mm", (10.0, 40.0)),
        wave_amp_mm=r.get("wave_amp_mm", (5.0, 15.0)),
        wave_len_mm=r.get("wave_len_mm", (20.0, 60.0)),
        length_mm=r.get("length_mm", (60.0, 150.0)))
    n_points = max(1, int(round(r["n_points"] * scale_points)))
    res = r["res"]
    cams = orbit_cameras(r["n_views"], res, res, r["arc_deg"])
    dtype = np.float16 if r["dtype"] == "f16" else np.float32
    theta, conf, depth = render_maps(rng_v, verts, offs, cams, res, res, r.get("kappa"),
                                     r.get("outliers", 0.0), dtype,
                                     head_radius=r.get("head_radius", SCALP_RADIUS),
                                     n_threads=n_threads)
    if r.get("outer", True):
        # the visible outer layer of the hair, as a reconstructed outer point
        # cloud would hold it: points (jitter included) visible in at least
        # two views; drawn in rounds until n_points are kept
        keep_p, keep_g, have = [], [], 0
        for _ in range(64):
            cand, cgt = sample_points(rng_p, verts, offs, max(4 * (n_points - have), 1024),
                                      r.get("jitter", 2e-3))
            ok = visible_views(cand, cams, depth, n_threads=n_threads) >= 2
            keep_p.append(cand[ok])
            keep_g.append(cgt[ok])
            have += int(ok.sum())
            if have >= n_points:
                break
        pts = np.concatenate(keep_p)[:n_points]
        gt = np.concatenate(keep_g)[:n_points]
    else:
        pts, gt = sample_points(rng_p, verts, offs, n_points, r.get("jitter", 2e-3))
    depth_out = depth.astype(dtype) if dtype == np.float16 else depth
    meta = dict(recipe=r, seed=int(seed), n_vertices=len(verts), n_strands=len(offs) - 1)
    return Scene(pts, gt, cams, theta, conf, depth_out, np.zeros(3, np.float32), meta)


def make_oriented_points(recipe, seed, n_points, noise_deg=10.0, outliers=0.1):
    """Oriented points over the whole hair volume of a recipe's strands (the
    strands of make_scene with the same seed): the stand-in for the fused
    outer and inferred inner point sets.  Directions are the ground-truth
    tangents turned by |N(0, noise_deg)| about a random perpendicular axis,
    with weight U(0.5, 1); an outlier fraction gets a uniform random direction
    and weight U(0, 0.5).  Returns (points, dirs, weights, gt), float32."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    r = dict(recipe)
    ss = np.random.SeedSequence(int(seed))
    s_strands, _, _, s_dirs = ss.spawn(4)
    rng_s = np.random.Generator(np.random.PCG64(s_strands))
    verts, offs = grow_strands(
        rng_s, r["n_strands"], r["kinds"],
        helix_r_mm=r.get("helix_r_mm", (5.0, 20.0)), pitch_mm=r.get("pitch_mm", (10.0, 40.0)),
        wave_amp_mm=r.get("wave_amp_mm", (5.0, 15.0)),
        wave_len_mm=r.get("wave_len_mm", (20.0, 60.0)),
        length_mm=r.get("length_mm", (60.0, 150.0)))
    rng = np.random.Generator(np.random.PCG64(s_dirs))
    pts, gt = sample_points(rng, verts, offs, int(n_points), r.get("jitter", 2e-3))
    g = gt.astype(np.float64)
    a = rng.normal(size=g.shape)
    a -= np.sum(a * g, axis=1, keepdims=True) * g
    a /= np.maximum(np.linalg.norm(a, axis=1, keepdims=True), 1e-300)
    ang = np.abs(rng.normal(0.0, math.radians(noise_deg), len(g)))[:, None]
    d = np.cos(ang) * g + np.sin(ang) * a
    w = rng.uniform(0.5, 1.0, len(g))
    out = rng.uniform(size=len(g)) < outliers
    d[out] = _unit(rng.normal(size=(int(out.sum()), 3)))
    w[out] = rng.uniform(0.0, 0.5, int(out.sum()))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return (pts.astype(np.float32), d.astype(np.float32), w.astype(np.float32),
            gt.astype(np.float32))


def scalp_seeds(recipe, seed):
    """Roots of a recipe's strands (those of make_scene / make_oriented_points
    with the same seed) and the outward scalp normals there: the seeds of
    the guide strands.  float32 (n_strands, 3) each."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    r = dict(recipe)
    ss = np.random.SeedSequence(int(seed))
    s_strands = ss.spawn(1)[0]
    rng_s = np.random.Generator(np.random.PCG64(s_strands))
    verts, offs = grow_strands(
        rng_s, r["n_strands"], r["kinds"],
        helix_r_mm=r.get("helix_r_mm", (5.0, 20.0)), pitch_mm=r.get("pitch_mm", (10.0, 40.0)),
        wave_amp_mm=r.get("wave_amp_mm", (5.0, 15.0)),
        wave_len_mm=r.get("wave_len_mm", (20.0, 60.0)),
        length_mm=r.get("length_mm", (60.0, 150.0)))
    roots = verts[offs[:-1]]
    normals = _unit(roots)
    return roots.astype(np.float32), normals.astype(np.float32)


def lattice_seeds(origin, voxel, dims, stride):
    """Centres of every stride-th voxel along each axis, x fastest: the
    seeds of the interior segments.  float32 (n, 3)."""
    nx, ny, nz = (int(d) for d in dims)
    ix = np.arange(0, nx, stride)
    iy = np.arange(0, ny, stride)
    iz = np.arange(0, nz, stride)
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    idx = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float64)
    pts = np.asarray(origin, np.float64) + (idx + 0.5) * float(voxel)
    return pts.astype(np.float32)


def head_grid(points, voxel):
    """A voxel grid covering the points with one empty voxel of margin:
    (origin float32[3], voxel float32, dims int32[3] as nx, ny, nz)."""
    h = np.float32(voxel)
    lo = np.floor(points.min(axis=0) / h) * h - h
    hi = points.max(axis=0)
    dims = (np.ceil((hi - lo) / h) + 1).astype(np.int32)
    return lo.astype(np.float32), h, dims


def method_params(recipe):
    """Search parameters a recipe is run with (patch, candidates, iterations)."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    return dict(patch=recipe["patch"], n_candidates=recipe["n_candidates"],
                refine_iters=recipe["refine_iters"])


# ---- small analytic scenes for tests -----------------------------------------

def straight_strand_scene(seed=0, n_points=50, n_views=8, res=256, arc_deg=120.0,
                          jitter=0.0, dtype=np.float32):
    """One straight strand in front of the scalp, noise-free maps, points
    exactly on the strand (ground truth = the strand direction)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = _unit(rng.normal(size=3))
    start = np.array([0.12, -0.02, 0.05]) + rng.uniform(-0.01, 0.01, 3)
    L = 0.06
    nv = int(math.ceil(L / POLY_STEP)) + 1
    verts = start[None, :] + np.linspace(0, L, nv)[:, None] * d[None, :]
    offs = np.array([0, nv], np.int64)
    pts, gt = sample_points(rng, verts, offs, n_points, jitter)
    cams = orbit_cameras(n_views, res, res, arc_deg)
    th, c, dep = render_maps([None] * n_views, verts, offs, cams, res, res, None, 0.0, dtype,
                             head_radius=0.0)
    dep = dep.astype(dtype)
    return Scene(pts, gt, cams, th, c, dep, np.zeros(3, np.float32),
                 dict(kind="straight_strand", seed=seed, direction=d.tolist()))


def random_direction_field_scene(seed, n_points=64, n_views=6, res=64, arc_deg=180.0,
                                 dtype=np.float32, smooth=False):
    """Points in a small ball, random (or smooth) orientation/confidence maps:
    a generic input for invariance and brute-force tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cams = orbit_cameras(n_views, res, res, arc_deg)
    pts = rng.normal(0.0, 0.03, (n_points, 3)).astype(np.float32)
    if smooth:
        yy, xx = np.mgrid[0:res, 0:res].astype(np.float64)
        theta = np.empty((n_views, res, res))
        conf = np.empty((n_views, res, res))
        for v in range(n_views):
            a, b, c, ph = rng.uniform(-1, 1, 4)
            theta[v] = np.mod(ph * 3 + 0.02 * (a * xx + b * yy) + 0.3 * np.sin(0.05 * c * xx),
                              math.pi)
            conf[v] = 0.55 + 0.4 * np.sin(0.03 * xx * a + 0.04 * yy * b + ph)
    else:
        theta = rng.uniform(0, math.pi, (n_views, res, res))
        conf = rng.uniform(0, 1, (n_views, res, res))
        conf[rng.uniform(0, 1, conf.shape) < 0.2] = 0.0
    return Scene(pts, np.zeros_like(pts), cams, theta.astype(dtype), conf.astype(dtype), None,
                 np.zeros(3, np.float32), dict(kind="random_field", seed=seed))
