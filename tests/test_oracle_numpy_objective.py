"""An independent NumPy statement of the objective, and closed forms of the
patch placement.  EfficientMonoHair Sec. 3.1: Eq. (4) (top-K confident
views), Eq. (8) (the candidate's image offset), Eqs. (9)-(11) (bidirectional,
confidence-weighted consistency, maximum over the fusion patch) and the mean
over the selected views.

The NumPy objective below is written from those equations without using any
part of the C oracle: the image direction of a candidate comes from the
projection Jacobian written as a 2 x 3 matrix (the oracle expands it
component-wise), the consistency is |r_hat . o| between unit vectors (the
oracle uses an angle difference), the top-K is a stable sort.  The two must
agree to 1e-12 on non-uniform maps, including patches that cross the image
border and background texels.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen


def _texels(m, xs, ys):
    """m[y, x] with zero outside the image (the patch border reading)."""
    H, W = m.shape
    inside = (xs >= 0) & (xs < W) & (ys >= 0) & (ys < H)
    out = np.zeros(np.broadcast(xs, ys).shape, np.float64)
    out[inside] = m[ys[inside], xs[inside]].astype(np.float64)
    return out


def _bilinear_doubled(theta, conf, x, y):
    """Confidence and unit doubled-angle mean at continuous (x, y) arrays:
    C = sum w_i C_i; m = sum w_i C_i (cos 2t_i, sin 2t_i)."""
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx, fy = x - x0, y - y0
    ix, iy = x0.astype(np.int64), y0.astype(np.int64)
    C = np.zeros_like(x)
    mx = np.zeros_like(x)
    my = np.zeros_like(x)
    for dx, dy, w in ((0, 0, (1 - fx) * (1 - fy)), (1, 0, fx * (1 - fy)),
                      (0, 1, (1 - fx) * fy), (1, 1, fx * fy)):
        c = _texels(conf, ix + dx, iy + dy)
        t = _texels(theta, ix + dx, iy + dy)
        C += w * c
        mx += w * c * np.cos(2 * t)
        my += w * c * np.sin(2 * t)
    return C, mx, my


def numpy_objective(cams, theta, conf, p, dirs, patch, top_k, z_near=1e-3):
    """J for one point and many directions (M x 3); +inf without a view."""
    cams = np.asarray(cams, np.float64)
    p = np.asarray(p, np.float64)
    V, H, W = theta.shape
    rows = []
    for v in range(V):
        f = cams[v, 0:2]
        c = cams[v, 2:4]
        R = cams[v, 4:13].reshape(3, 3)
        Xc = R @ p + cams[v, 13:16]
        if not Xc[2] > z_near:
            continue
        u = f * Xc[:2] / Xc[2] + c
        if not (0 <= u[0] <= W - 1 and 0 <= u[1] <= H - 1):
            continue
        Cc, _, _ = _bilinear_doubled(theta[v], conf[v], np.array([u[0]]), np.array([u[1]]))
        if not Cc[0] > 0:
            continue
        rows.append((-Cc[0], v, u, Xc, R, f))
    rows.sort(key=lambda r: (r[0], r[1]))          # stable: confidence, then index
    rows = rows[:top_k]
    dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
    if not rows:
        return np.full(len(dirs), math.inf)
    h = (patch - 1) // 2
    offs = np.arange(-h, h + 1, dtype=np.float64)
    total = np.zeros(len(dirs))
    for _, v, u, Xc, R, f in rows:
        X, Y, Z = Xc
        # d(pi)/d(X_c) of the pinhole, times R: the image offset of a small
        # step along d, up to the positive factor of the step
        Jpi = np.array([[f[0] / Z, 0.0, -f[0] * X / Z ** 2],
                        [0.0, f[1] / Z, -f[1] * Y / Z ** 2]]) @ R
        r = dirs @ Jpi.T                                   # M x 2
        rn = np.linalg.norm(r, axis=1)
        bx, by = np.meshgrid(offs, offs)                   # patch offsets (a, b)
        Cs, mx, my = _bilinear_doubled(theta[v], conf[v], (u[0] + bx).ravel(),
                                       (u[1] + by).ravel())
        mn = np.hypot(mx, my)
        ok = mn > 0
        half = 0.5 * np.arctan2(my[ok], mx[ok])
        o = np.stack([np.cos(half), np.sin(half)], axis=1)   # unit orientation
        with np.errstate(invalid="ignore", divide="ignore"):
            rh = r / rn[:, None]
        sim = np.abs(rh @ o.T) * Cs[ok][None, :]           # M x samples
        best = sim.max(axis=1) if ok.any() else np.zeros(len(dirs))
        best = np.where(rn > 0, best, 0.0)
        total += best
    return 1.0 - total / len(rows)


def _wide_points(n, seed, spread=0.3):
    """Points whose projections cover the whole image, the border included."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-spread, spread, (n, 3)).astype(np.float32)


@pytest.mark.parametrize("seed,patch,dtype", [(0, 3, np.float32), (1, 5, np.float16),
                                              (2, 7, np.float32)])
def test_numpy_objective_agrees_with_the_oracle(seed, patch, dtype):
    """10^4 random (point, direction) pairs per case on random maps with 20%
    background texels, points spread so that many patches cross the image
    border: |J_oracle - J_numpy| <= 1e-12."""
    sc = scenegen.random_direction_field_scene(40 + seed, n_points=4, n_views=7, res=40,
                                               dtype=dtype)
    pts = _wide_points(500, seed)
    rng = np.random.default_rng(seed)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=patch, top_k=5)
    n_fin = n_border = 0
    worst = 0.0
    for p in pts:
        ids, u = o.select_views(p)
        dirs = rng.normal(size=(20, 3))
        Jo = o.objective_many(p, dirs)
        Jn = numpy_objective(sc.cams, sc.theta, sc.conf, p, dirs, patch, 5)
        assert np.array_equal(np.isinf(Jo), np.isinf(Jn))
        fin = np.isfinite(Jo)
        if fin.any():
            worst = max(worst, float(np.max(np.abs(Jo[fin] - Jn[fin]))))
            n_fin += int(fin.sum())
            h = (patch - 1) // 2
            n_border += int(np.any((u < h) | (u > 39 - h)))
    assert worst <= 1e-12, worst
    assert n_fin >= 4000          # most pairs have a view
    assert n_border >= 30         # patches that reach past the image border


def test_numpy_objective_sees_a_planted_mistake():
    """The comparison is sharp: one texel next to the projection of the best
    view, its confidence scaled by 1.25 in the NumPy copy of the maps, moves J
    past the tolerance for most points."""
    sc = scenegen.random_direction_field_scene(44, n_points=4, n_views=5, res=32)
    pts = _wide_points(60, 4, spread=0.05)
    conf2 = sc.conf.copy()
    rng = np.random.default_rng(4)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, patch=3, top_k=5)
    moved = 0
    for p in pts:
        ids, u = o.select_views(p)
        if len(ids) == 0:
            continue
        v = ids[0]
        x, y = int(round(u[0][0])), int(round(u[0][1]))
        c2 = conf2.copy()
        c2[v, y, x] = np.float32(c2[v, y, x] * 1.25)
        dirs = rng.normal(size=(20, 3))
        Jo = o.objective_many(p, dirs)
        Jn = numpy_objective(sc.cams, sc.theta, c2, p, dirs, 3, 5)
        fin = np.isfinite(Jo) & np.isfinite(Jn)
        moved += np.any(np.abs(Jo[fin] - Jn[fin]) > 1e-12)
    assert moved >= 10


# ---- patch placement (Sec. 3.1.3) -------------------------------------------

def _backproject(cam, u, Z):
    cam = np.asarray(cam, np.float64)
    R = cam[4:13].reshape(3, 3)
    Xc = np.array([(u[0] - cam[2]) / cam[0] * Z, (u[1] - cam[3]) / cam[1] * Z, Z])
    return R.T @ (Xc - cam[13:16])


def _weight_1d(u, x_star, h):
    """Largest bilinear weight a patch sample u + a, a in {-h..h}, gives the
    texel at x_star."""
    return max(max(0.0, 1.0 - abs(u + a - x_star)) for a in range(-h, h + 1))


@pytest.mark.parametrize("patch", [1, 3, 5, 7])
def test_single_bright_texel_closed_form(patch):
    """One texel of confidence 1 on a faint uniform background of confidence
    c0, every texel at the same orientation theta*.  Each patch sample then
    has orientation theta* and confidence c0 + (1 - c0) w, w the bilinear
    weight the bright texel gets at that sample, so
        J(d) = 1 - (c0 + (1 - c0) max_(a,b) w_a w_b) |cos(phi(d) - theta*)|
    with w_a = max(0, 1 - |u_x + a - x*|).  This fixes where the patch sits
    (offsets (a, b) in whole pixels around the sub-pixel projection u)."""
    W = H = 32
    h = (patch - 1) // 2
    cams = scenegen.orbit_cameras(1, W, H, 0.0)
    cam = cams[0]
    th_star, c0 = 0.7, 0.01
    rng = np.random.default_rng(patch)
    checked = 0
    for trial in range(60):
        ut = rng.uniform(10, 21, 2)
        p = _backproject(cam, ut, 0.6).astype(np.float32)
        # the bright texel anywhere from inside the patch to just outside it
        xs, ys = (int(np.floor(ut[0])) + rng.integers(-h - 2, h + 3),
                  int(np.floor(ut[1])) + rng.integers(-h - 2, h + 3))
        theta = np.full((1, H, W), th_star, np.float32)
        conf = np.full((1, H, W), c0, np.float32)
        conf[0, ys, xs] = 1.0
        o = oracle.Oracle(cams, theta, conf, patch=patch, top_k=1)
        ids, u = o.select_views(p)
        assert list(ids) == [0]
        u = u[0]
        wmax = _weight_1d(u[0], xs, h) * _weight_1d(u[1], ys, h)
        cmax = float(np.float32(c0)) + (1.0 - float(np.float32(c0))) * wmax
        dirs = rng.normal(size=(8, 3))
        R = cam[4:13].reshape(3, 3).astype(np.float64)
        Xc = R @ p.astype(np.float64) + cam[13:16]
        for d in dirs:
            dc = R @ d
            rx = cam[0] * (dc[0] * Xc[2] - Xc[0] * dc[2])
            ry = cam[1] * (dc[1] * Xc[2] - Xc[1] * dc[2])
            phi = math.atan2(ry, rx)
            want = 1.0 - cmax * abs(math.cos(phi - float(np.float32(th_star))))
            assert o.objective(p, d) == pytest.approx(want, abs=1e-12)
            checked += 1
    assert checked == 480


def test_patch_placement_misplacements_are_visible():
    """Guards the closed form above: a patch centred on the rounded pixel, or
    spaced two pixels apart, gives a different maximum weight for most
    sub-pixel positions, so either slip would fail it."""
    rng = np.random.default_rng(9)
    diff_round = diff_space = 0
    for _ in range(200):
        u = rng.uniform(10, 21)
        xs = int(np.floor(u)) + int(rng.integers(-2, 3))
        w = _weight_1d(u, xs, 1)
        w_round = max(max(0.0, 1.0 - abs(round(u) + a - xs)) for a in (-1, 0, 1))
        w_space = max(max(0.0, 1.0 - abs(u + 2 * a - xs)) for a in (-1, 0, 1))
        diff_round += abs(w - w_round) > 1e-6
        diff_space += abs(w - w_space) > 1e-6
    assert diff_round > 100 and diff_space > 50
