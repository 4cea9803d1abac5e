"""GPU parity of the orientation and confidence maps (fd_orientation_maps: the
Gabor-filter extraction of Sec. 3.1) against the CPU oracle.

The kernel accumulates each response in binary32 from a binary32 bank; the
oracle does both in binary64.  So the orientation bins must agree except
where the oracle's best response and the one the GPU picked lie within the
binary32 accumulation bound of each other, and the confidences agree within
that bound carried through the confidence formula (derived below).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
# binary32 rounding of 289 products and partial sums, with margin: every
# response is within this many times sum_t |g(t)| |I(p + t)| of its exact value
REL = 4e-6


def _native():
    from paper_2604_05794_amd import native
    native.lib()
    return native


def _gpu(frames, out_dtype=torch.float32, **kw):
    nat = _native()
    fr = torch.from_numpy(np.ascontiguousarray(frames, np.float32)).to(DEV)
    th, cf = nat.orientation_maps(fr, out_dtype=out_dtype, **kw)
    torch.cuda.synchronize()
    return th.float().cpu().numpy(), cf.float().cpu().numpy()


def _bank_kw(kw):
    return dict(n_orient=kw.get("n_orient", 32), radius=kw.get("radius", 8),
                sigma_along=kw.get("sigma_along", 2.4), sigma_across=kw.get("sigma_across", 1.8),
                wavelength=kw.get("wavelength", 4.0))


def _check_frame(img, th_g, cf_g, bank, conf_abs=0.0, max_tie_frac=2e-3):
    """One frame against the oracle; returns the number of tie pixels."""
    N = bank.shape[0]
    th_o, cf_o, wmax, F = oracle.gabor(img, bank, responses=True)
    # sum_t |g_i(t)| |I(p + t)|, the scale of the binary32 error of F_i
    _, _, _, L1 = oracle.gabor(np.abs(img), np.abs(bank), responses=True)
    scale = L1.max(axis=-1)
    b_o = np.rint(th_o * N / math.pi).astype(int)
    b_g = np.rint(th_g * N / math.pi).astype(int)
    assert b_g.min() >= 0 and b_g.max() < N
    assert np.allclose(th_g, b_g * (math.pi / N), atol=1e-3)
    diff = b_g != b_o
    # a different bin only where the two responses are within rounding
    Fo = np.take_along_axis(F, b_o[..., None], -1)[..., 0]
    Fg = np.take_along_axis(F, b_g[..., None], -1)[..., 0]
    tie = Fo - Fg <= 2 * REL * scale
    assert np.all(tie[diff]), f"{np.sum(diff & ~tie)} pixels with a clear orientation mismatch"
    assert diff.mean() <= max_tie_frac
    # confidence: each |F_i - F_max| moves by at most 2 REL scale, so w by at
    # most 2 REL scale sqrt(sum_i d_i^2); C = w / wmax moves by that over wmax
    # plus C times the relative change of wmax
    k = np.arange(N)
    dk = np.minimum(k, N - k) * (math.pi / N)
    dw = 2 * REL * scale * math.sqrt(np.sum(dk * dk))
    bound = (dw / wmax + cf_o * (dw.max() / wmax) if wmax > 0 else 0 * dw) + conf_abs
    err = np.abs(cf_g - cf_o)
    ok = ~diff
    assert np.all(err[ok] <= bound[ok] + 1e-7), f"conf err {err[ok].max():.3e}"
    assert cf_g.min() >= 0.0 and cf_g.max() <= 1.0
    if wmax > 0:
        assert cf_g.max() == 1.0   # the frame's own maximum divides to exactly 1
    return int(diff.sum()), float(err[ok].max())


def test_tiny_frames_match_the_oracle():
    frames, _, _, _ = scenegen.make_frames("tiny", 0)
    th, cf = _gpu(frames)
    bank = oracle.gabor_bank()
    ties = 0
    for v in range(frames.shape[0]):
        t, e = _check_frame(frames[v], th[v], cf[v], bank)
        ties += t
    print("gabor tiny: tie pixels", ties, "of", frames.size, flush=True)


def test_full_resolution_frames_match_the_oracle():
    """Frames at the realistic workload's 1024 x 1024, four views."""
    r = dict(scenegen.RECIPES["realistic"])
    r["n_views"] = 4
    frames, _, _, _ = scenegen.make_frames(r, 3)
    assert frames.shape == (4, 1024, 1024)
    th, cf = _gpu(frames)
    bank = oracle.gabor_bank()
    for v in (0, 3):
        t, e = _check_frame(frames[v], th[v], cf[v], bank)
        print("gabor 1024^2 frame", v, "ties", t, "max conf err", e, flush=True)


@pytest.mark.parametrize("shape,kw", [
    ((1, 1, 1), dict()),
    ((2, 37, 53), dict(n_orient=8, radius=3)),
    ((3, 17, 16), dict(n_orient=16, radius=1)),
    ((1, 70, 45), dict(n_orient=32, radius=12, sigma_along=4.0, sigma_across=2.5,
                       wavelength=6.0)),
    ((2, 16, 33), dict(n_orient=16, radius=8, wavelength=3.0)),
])
def test_ragged_sizes_and_parameters(shape, kw):
    rng = np.random.default_rng(hash(shape) % 2**32)
    frames = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    th, cf = _gpu(frames, **kw)
    bank = oracle.gabor_bank(**_bank_kw(kw))
    for v in range(shape[0]):
        _check_frame(frames[v], th[v], cf[v], bank, max_tie_frac=0.01)


def test_half_maps_are_the_rounded_float_maps():
    frames, _, _, _ = scenegen.make_frames("tiny", 1)
    th32, cf32 = _gpu(frames[:3], torch.float32)
    th16, cf16 = _gpu(frames[:3], torch.float16)
    assert np.array_equal(th16, th32.astype(np.float16).astype(np.float32))
    assert np.array_equal(cf16, cf32.astype(np.float16).astype(np.float32))


@pytest.mark.parametrize("dt", [torch.float16, torch.float32])
def test_unaligned_confidence_buffer(dt):
    """A confidence buffer that is not 16-byte aligned takes the element-wise
    normalisation and holds the same maps as an aligned one."""
    nat = _native()
    frames, _, _, _ = scenegen.make_frames("tiny", 4)
    fr = torch.from_numpy(np.ascontiguousarray(frames[:3], np.float32)).to(DEV)
    V, H, W = fr.shape
    assert (H * W) % 8 == 0  # the aligned call takes the 8-pixel path
    th0, cf0 = nat.orientation_maps(fr, out_dtype=dt)
    buf = torch.full((V * H * W + 1,), 7.0, dtype=dt, device=DEV)
    cf1 = buf[1:].view(V, H, W)
    assert cf1.data_ptr() % 16 != 0
    th1, _ = nat.orientation_maps(fr, out_dtype=dt, conf=cf1)
    torch.cuda.synchronize()
    assert torch.equal(th0, th1) and torch.equal(cf0, cf1)
    assert buf[0].item() == 7.0  # nothing written before the buffer


def test_frames_are_independent():
    frames, _, _, _ = scenegen.make_frames("tiny", 2)
    th, cf = _gpu(frames[:5])
    for v in (0, 4):
        th1, cf1 = _gpu(frames[v:v + 1])
        assert np.array_equal(th1[0], th[v]) and np.array_equal(cf1[0], cf[v])


@pytest.mark.parametrize("i", [0, 5, 16, 27])
def test_grating_on_a_bin(i):
    N = 32
    t0 = math.pi * i / N
    yy, xx = np.mgrid[0:64, 0:80].astype(np.float64)
    img = np.cos(2 * math.pi * (-xx * math.sin(t0) + yy * math.cos(t0)) / 4.0)
    th, cf = _gpu(img[None].astype(np.float32))
    inner = (slice(10, -10), slice(10, -10))
    ridge = np.abs(img[inner]) >= 0.5
    assert np.all(np.rint(th[0][inner][ridge] * N / math.pi) == i)
    assert cf[0][inner][ridge].min() > 0.3


def test_zero_and_empty_inputs():
    nat = _native()
    th, cf = _gpu(np.zeros((2, 20, 24), np.float32))
    assert not th.any() and not cf.any()
    fr = torch.empty((0, 8, 8), dtype=torch.float32, device=DEV)
    t, c = nat.orientation_maps(fr)
    assert t.shape == (0, 8, 8) and c.shape == (0, 8, 8)


def test_invalid_arguments():
    nat = _native()
    fr = torch.zeros((1, 16, 16), dtype=torch.float32, device=DEV)
    for bad in (dict(n_orient=12), dict(n_orient=64), dict(radius=0), dict(radius=13),
                dict(sigma_along=0.0), dict(sigma_across=-1.0), dict(wavelength=float("nan")),
                dict(wavelength=float("inf"))):
        with pytest.raises(nat.FdError) as e:
            nat.orientation_maps(fr, **bad)
        assert e.value.code == nat.FD_E_INVAL
    with pytest.raises(TypeError):
        nat.orientation_maps(fr.double())


def test_maps_feed_the_direction_search():
    """Frames -> maps on the GPU -> direction search on the GPU, against the
    oracle's maps and the oracle's search on the same points."""
    from parity import assert_parity, compare
    nat = _native()
    sc = scenegen.make_scene("tiny", 0)
    frames, _, _, cams = scenegen.make_frames("tiny", 0)
    assert np.array_equal(cams, sc.cams)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    th_g, cf_g = nat.orientation_maps(t(frames), out_dtype=torch.float16)
    d, c = nat.fuse_directions(t(sc.points), t(sc.cams), th_g, cf_g,
                               depth_maps=t(sc.depth.astype(np.float16)), patch=3, top_k=5)
    torch.cuda.synchronize()
    bank = oracle.gabor_bank()
    th_o = np.empty(frames.shape, np.float16)
    cf_o = np.empty(frames.shape, np.float16)
    for v in range(frames.shape[0]):
        a, b, _ = oracle.gabor(frames[v], bank)
        th_o[v], cf_o[v] = a, b
    # the maps: GPU and oracle agree texel by texel up to the binary16
    # rounding of values on a rounding boundary (the Gabor tests above hold
    # the exact bar); the search on the GPU's maps is held to the full
    # parity protocol against the oracle's search on those same maps
    th_gn, cf_gn = th_g.cpu().numpy(), cf_g.cpu().numpy()
    assert np.mean(np.abs(cf_gn.astype(np.float32) - cf_o.astype(np.float32)) > 1e-3) < 1e-3
    idx = np.arange(0, sc.n_points, 7)
    orc = oracle.Oracle(sc.cams, th_gn, cf_gn, depth=sc.depth.astype(np.float16), patch=3,
                        top_k=5)
    do, co = orc.fuse(sc.points[idx])
    res = compare(orc, sc.points[idx], d.cpu().numpy()[idx], c.cpu().numpy()[idx], do, co)
    print("frames->maps->search", {k: v for k, v in res.items() if not k.endswith("_idx")},
          flush=True)
    assert_parity(res)
