"""Pins of the oracle's image-quality metrics (Sec. 3.1, Eqs. (snr), (mse),
(psnr), (ssim)) against closed forms: identical images, a constant offset, a
scaled image, the SNR/PSNR identity, a single SSIM window computed from its
moments by hand, and crops against explicitly cut-out images."""
import math

import numpy as np

from oracle import oracle as O


def test_identical_images():
    N = 16
    ref = np.random.default_rng(1).uniform(0, 1, N * N)
    assert O.mse(ref, ref, N) == 0.0
    assert O.snr(ref, ref, N) == float("inf") and O.psnr(ref, ref, N) == float("inf")
    assert O.ssim(ref, ref, N) == 1.0


def test_constant_offset_and_scale_closed_forms():
    N = 12
    ref = np.random.default_rng(2).uniform(0.2, 1.0, N * N)
    e = 0.03
    img = ref + e
    assert math.isclose(O.mse(ref, img, N), e * e, rel_tol=1e-12)
    assert math.isclose(O.snr(ref, img, N), 10 * math.log10(np.sum(ref ** 2) / (N * N * e * e)), rel_tol=1e-12)
    assert math.isclose(O.psnr(ref, img, N), 10 * math.log10(np.max(ref) ** 2 / (e * e)), rel_tol=1e-12)
    a = 0.9
    assert math.isclose(O.snr(ref, a * ref, N), -20 * math.log10(1 - a), rel_tol=1e-12)
    # PSNR - SNR = 10 log10(MAX^2 N^2 / sum I0^2) for any image
    img2 = ref + np.random.default_rng(3).normal(0, 0.01, N * N)
    assert math.isclose(O.psnr(ref, img2, N) - O.snr(ref, img2, N),
                        10 * math.log10(np.max(ref) ** 2 * N * N / np.sum(ref ** 2)), rel_tol=1e-10)


def test_single_window_by_hand():
    """A 7 x 7 image is one window: SSIM from its two means, variances and
    covariance (sample estimates), c1 = (0.01 L)^2, c2 = (0.03 L)^2."""
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 2, 49)
    y = 0.7 * x + 0.3 + rng.normal(0, 0.05, 49)
    mx, my = x.mean(), y.mean()
    vx, vy = x.var(ddof=1), y.var(ddof=1)
    cxy = np.cov(x, y, ddof=1)[0, 1]
    L = x.max() - x.min()
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    expect = (2 * mx * my + c1) * (2 * cxy + c2) / ((mx ** 2 + my ** 2 + c1) * (vx + vy + c2))
    assert math.isclose(O.ssim(x, y, 7), expect, rel_tol=1e-12)
    # a constant shift keeps the structure term at 1: only the luminance term remains
    s = 0.25
    lum = (2 * mx * (mx + s) + c1) / (mx ** 2 + (mx + s) ** 2 + c1)
    assert math.isclose(O.ssim(x, x + s, 7), lum, rel_tol=1e-12)


def test_crop_equals_cut_out_image():
    N = 20
    rng = np.random.default_rng(5)
    ref = rng.uniform(0, 1, N * N)
    img = ref + rng.normal(0, 0.02, N * N)
    crop = (3, 2, 4, 1)                              # bottom, top, left, right
    r2 = ref.reshape(N, N)[3:N - 2, 4:N - 1]
    i2 = img.reshape(N, N)[3:N - 2, 4:N - 1]
    assert math.isclose(O.mse(ref, img, N, crop), float(np.mean((r2 - i2) ** 2)), rel_tol=1e-12)
    assert math.isclose(O.snr(ref, img, N, crop), 10 * math.log10(np.sum(r2 ** 2) / np.sum((r2 - i2) ** 2)),
                        rel_tol=1e-12)
    # SSIM of a square crop equals SSIM of the cut-out square image
    crop_sq = (3, 2, 4, 1 + 0)
    h, w = N - 3 - 2, N - 4 - 1
    assert h == w
    assert math.isclose(O.ssim(ref, img, N, crop_sq), O.ssim(r2.ravel(), i2.ravel(), h), rel_tol=1e-12)
