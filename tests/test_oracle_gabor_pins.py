"""Pins of the oracle's orientation and confidence extraction (the Gabor-filter
maps the direction search consumes; the paper names the filters without
parameters, the readings are in oracle/gabor.c).

Checked against what the definition and geometry fix: an impulse image
answers with the kernels themselves (correlation indexing), a grating is
assigned its own orientation bin, mirror and transpose of the image permute
the bins exactly, scaling the image changes neither map, the bank has zero
mean, and a constant image carries no orientation.
"""
import math

import numpy as np
import pytest

import oracle

N = 32


@pytest.fixture(scope="module")
def bank():
    return oracle.gabor_bank(n_orient=N)


def _grating(t0, H=64, W=64, period=4.0):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    b = -xx * math.sin(t0) + yy * math.cos(t0)   # across the direction t0
    return np.cos(2 * math.pi * b / period).astype(np.float32)


def test_bank_is_zero_mean_and_symmetric(bank):
    assert np.abs(bank.sum(axis=(1, 2))).max() < 1e-12
    # an even kernel: g(-dx, -dy) = g(dx, dy)
    assert np.allclose(bank, bank[:, ::-1, ::-1], atol=1e-14)
    # orientation 0 is the x axis: the carrier varies along y only at dx = 0
    g0 = bank[0]
    r = (g0.shape[0] - 1) // 2
    assert g0[r, r] > 0 and g0[r, r] > g0[r + 1, r]


def test_impulse_answers_with_the_kernels(bank):
    H = W = 40
    img = np.zeros((H, W), np.float32)
    x0, y0 = 17, 21
    img[y0, x0] = 1.0
    _, _, _, F = oracle.gabor(img, bank, responses=True)
    r = (bank.shape[1] - 1) // 2
    for y in range(y0 - r, y0 + r + 1):
        for x in range(x0 - r, x0 + r + 1):
            # F_i(x, y) = |sum g_i(dx, dy) I(x + dx, y + dy)| = |g_i(x0 - x, y0 - y)|
            want = np.abs(bank[:, y0 - y + r, x0 - x + r])
            assert np.allclose(F[y, x], want, atol=1e-13)
    assert np.all(F[0, 0] == 0.0)


@pytest.mark.parametrize("i", [0, 3, 8, 13, 16, 21, 31])
def test_grating_on_a_bin_is_assigned_that_bin(bank, i):
    t0 = math.pi * i / N
    img = _grating(t0)
    th, cf, _ = oracle.gabor(img, bank)
    inner = (slice(10, -10), slice(10, -10))
    # the even kernels answer 0 on the grating's nodes (quarter period off a
    # ridge), so look at the pixels on or near a ridge
    ridge = np.abs(img[inner]) >= 0.5
    assert ridge.mean() > 0.3
    assert np.all(th[inner][ridge] == t0)
    assert cf[inner][ridge].min() > 0.3


@pytest.mark.parametrize("t0", [0.05, 0.6, 1.3, 2.0, 2.9])
def test_grating_off_bin_goes_to_the_nearest_bin(bank, t0):
    img = _grating(t0)
    th, _, _ = oracle.gabor(img, bank)
    inner = (slice(10, -10), slice(10, -10))
    ridge = np.abs(img[inner]) >= 0.5
    want = (round(t0 * N / math.pi) % N) * math.pi / N
    assert np.all(np.abs(th[inner][ridge] - want) < 1e-12)


def test_mirror_and_transpose_permute_the_bins_exactly(bank):
    rng = np.random.default_rng(5)
    img = rng.normal(size=(48, 56)).astype(np.float32)
    th, cf, m = oracle.gabor(img, bank)
    b = np.rint(th * N / math.pi).astype(int)
    # x mirror: direction (cos t, sin t) -> (-cos t, sin t), bin i -> (N - i) mod N
    thm, cfm, mm = oracle.gabor(img[:, ::-1].copy(), bank)
    bm = np.rint(thm * N / math.pi).astype(int)[:, ::-1]
    assert np.mean(bm == (N - b) % N) > 0.999
    assert abs(mm - m) < 1e-9 * m
    # transpose: (x, y) -> (y, x), direction angle t -> pi/2 - t, bin i -> (N/2 - i) mod N
    tht, cft, mt = oracle.gabor(img.T.copy(), bank)
    bt = np.rint(tht * N / math.pi).astype(int).T
    assert np.mean(bt == (N // 2 - b) % N) > 0.999
    assert np.allclose(cft.T, cf, atol=1e-9)


def test_scaling_the_image_changes_neither_map(bank):
    rng = np.random.default_rng(6)
    img = rng.uniform(0, 1, (40, 40)).astype(np.float32)
    th, cf, m = oracle.gabor(img, bank)
    th2, cf2, m2 = oracle.gabor((img * 4.0).astype(np.float32), bank)
    assert np.array_equal(th, th2)
    assert np.allclose(cf, cf2, atol=1e-12) and abs(m2 - 4 * m) < 1e-9 * m


def test_constant_image_has_no_orientation(bank):
    img = np.full((32, 32), 0.7, np.float32)
    th, cf, m, F = oracle.gabor(img, bank, responses=True)
    inner = (slice(8, -8), slice(8, -8))   # windows that do not reach the zero border
    # zero-mean kernels: only rounding is left inside (the border answers)
    assert np.abs(F[inner]).max() < 1e-12 * np.abs(F).max()
    assert np.abs(cf[inner]).max() < 1e-9
    th0, cf0, m0 = oracle.gabor(np.zeros((16, 16), np.float32), bank)
    assert m0 == 0.0 and not th0.any() and not cf0.any()


def test_clean_grating_is_more_confident_than_noise(bank):
    rng = np.random.default_rng(7)
    noise = rng.normal(size=(64, 64)).astype(np.float32)
    g = _grating(1.1)
    both = np.concatenate([g, noise], axis=1)
    _, cf, _ = oracle.gabor(both, bank)
    assert cf[10:-10, 10:54].mean() > 2 * cf[10:-10, 74:-10].mean()
