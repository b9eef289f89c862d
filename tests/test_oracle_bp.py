"""Pins of the oracle's back-projection (Eq. Err_img and the update after it)
and its approximate cross bilateral filter (Section 4.3) against library
filters, fixed points and convergence."""
import math

import numpy as np
import pytest
from scipy import ndimage

import synthdata
from oracle import backproject as bp
from oracle import imaging


def test_normalised_gaussian_matches_scipy_constant_mode_ratio():
    rng = np.random.default_rng(0)
    E = rng.standard_normal((37, 29))
    s = 1.5
    num = ndimage.gaussian_filter(E, s, truncate=5 / s, mode="constant")
    den = ndimage.gaussian_filter(np.ones_like(E), s, truncate=5 / s, mode="constant")
    assert np.abs(bp.gauss_filter_normalised(E, s) - num / den).max() < 1e-13


def test_box_mean_matches_in_image_window_mean():
    rng = np.random.default_rng(1)
    I = rng.random((23, 31))
    mu = bp.box_mean(I, 5)
    for (y, x) in [(0, 0), (11, 17), (22, 30), (5, 0), (3, 29)]:
        win = I[max(0, y - 5):y + 6, max(0, x - 5):x + 6]
        assert abs(mu[y, x] - win.mean()) < 1e-13
    num = ndimage.uniform_filter(I, 11, mode="constant")
    den = ndimage.uniform_filter(np.ones_like(I), 11, mode="constant")
    assert np.abs(mu - num / den).max() < 1e-12


def test_consistent_estimate_is_a_fixed_point():
    I0 = synthdata.fractal_voronoi_image(2, 40, 44).astype(np.float64)
    lr = imaging.degrade(I0, 2, to_f32=False)
    I1 = bp.bp_step(I0, lr, 2, 1.0, 1.5, 0.1)
    assert np.array_equal(I1, I0)


def test_range_weight_and_textbook_limit():
    rng = np.random.default_rng(2)
    I = rng.random((30, 30))
    S = bp.range_weight(I, 1.5, 0.1)
    assert S.max() <= 1.0 and S.min() > 0.0
    assert np.allclose(bp.range_weight(np.full((9, 9), 0.4), 1.5, 0.1), 1.0)
    # sigma_r = inf: Irani's back-projection with a Gaussian back-projection filter
    lr = rng.random((15, 15))
    up = bp.bp_step(I, lr, 2, 1.0, 1.5, math.inf)
    e = lr - ndimage.gaussian_filter(I, 1.0, truncate=3.0, mode="nearest")[::2, ::2]
    E = imaging.bicubic_up(e, 2)
    ref = I + ndimage.gaussian_filter(E, 1.5, truncate=5 / 1.5, mode="constant") / \
        ndimage.gaussian_filter(np.ones_like(E), 1.5, truncate=5 / 1.5, mode="constant")
    assert np.abs(up - ref).max() < 1e-12
    # with sigma_r -> inf the exact cross bilateral filter is the normalised Gaussian
    ex = bp.exact_cross_bilateral(E, I, 1.5, 1e9)
    assert np.abs(ex - bp.gauss_filter_normalised(E, 1.5)).max() < 1e-12


def _residual(I, lr, s):
    return np.abs(imaging.degrade(I, s, to_f32=False) - lr).max()


def test_back_projection_reduces_lr_residual():
    hr = synthdata.fractal_voronoi_image(3, 64, 64).astype(np.float64)
    lr = imaging.degrade(hr, 2, to_f32=False)
    I = imaging.bicubic_up(lr, 2)
    r = [_residual(I, lr, 2)]
    for _ in range(4):
        I = bp.bp_step(I, lr, 2, 1.0, 1.5, 0.1)
        r.append(_residual(I, lr, 2))
    assert all(b < a for a, b in zip(r, r[1:]))


def test_band_limited_input_converges():
    """On a band-limited LR target the textbook iteration contracts every
    frequency, so the LR residual goes to zero."""
    h = 24
    yy, xx = np.meshgrid(np.arange(h), np.arange(h), indexing="ij")
    lr = 0.5 + 0.2 * np.cos(2 * np.pi * yy / h) * np.cos(2 * np.pi * 2 * xx / h)
    I = np.full((2 * h, 2 * h), 0.5)
    r = []
    for _ in range(100):
        I = bp.bp_step(I, lr, 2, 1.0, 1.5, math.inf)
        r.append(_residual(I, lr, 2))
    assert all(b < a for a, b in zip(r, r[1:]))
    assert r[-1] < 3e-5 and r[-1] < 0.1 * r[19]


def _S(d, sigma_r):
    return math.exp(-(d * d) / (2.0 * sigma_r * sigma_r))


@pytest.mark.parametrize("sigma_s,sigma_r", [(1.5, 0.1), (1.0, 0.05)])
def test_range_weight_closed_form_single_bright_pixel(sigma_s, sigma_r):
    """Eq. sx2 on a zero image with one bright pixel v: the window of side
    2R + 1 (R = ceil(3 sigma_s)) around x has mean v / (its in-image pixel
    count) when it holds the bright pixel and 0 otherwise, so every S(x) has
    a closed form. Fails for a swap of sigma_s and sigma_r, a dropped factor
    2, another window radius, a missing window mean or a border count over
    out-of-image pixels."""
    R = int(math.ceil(3.0 * sigma_s))
    v = 0.1
    H = W = 4 * R + 6
    yc, xc = 2 * R + 2, 2 * R + 3
    I = np.zeros((H, W))
    I[yc, xc] = v
    S = bp.range_weight(I, sigma_s, sigma_r)
    n = (2 * R + 1) ** 2
    assert abs(S[yc, xc] - _S(v - v / n, sigma_r)) < 1e-15
    # inside the bright pixel's window: I = 0, mean v / n
    for dy, dx in [(0, R), (R, -R), (-2, 3)]:
        assert abs(S[yc + dy, xc + dx] - _S(v / n, sigma_r)) < 1e-15
    # just outside it: mean 0
    for dy, dx in [(0, R + 1), (R + 1, 0), (-R - 1, R)]:
        assert S[yc + dy, xc + dx] == 1.0
    # at the border the window holds only its in-image pixels
    J = np.zeros((H, W))
    J[1, 2] = v
    SJ = bp.range_weight(J, sigma_s, sigma_r)
    assert abs(SJ[0, 0] - _S(v / ((R + 1) * (R + 1)), sigma_r)) < 1e-15
    assert abs(SJ[1, 2] - _S(v - v / ((R + 2) * (R + 3)), sigma_r)) < 1e-15


def test_update_range_weight_is_taken_on_the_current_estimate():
    """One iteration I + S * F with F the normalised Gaussian of the bicubic
    upsampled LR error (built here from scipy's filters) and S of Eq. sx2
    evaluated on the current HR estimate I: checked pixel by pixel against
    the closed form of S for a single bright pixel, so a range weight taken on
    the error image or on the LR image instead fails."""
    sigma_s, sigma_r, v = 1.5, 0.1, 0.1
    H = 40
    I = np.zeros((H, H))
    I[20, 21] = v
    lr = np.zeros((H // 2, H // 2))
    e = lr - ndimage.gaussian_filter(I, 1.0, truncate=3.0, mode="nearest")[::2, ::2]
    E = imaging.bicubic_up(e, 2)
    F = ndimage.gaussian_filter(E, sigma_s, truncate=5 / sigma_s, mode="constant") / \
        ndimage.gaussian_filter(np.ones_like(E), sigma_s, truncate=5 / sigma_s, mode="constant")
    I1 = bp.bp_step(I, lr, 2, 1.0, sigma_s, sigma_r)
    expect = {(20, 21): _S(v - v / 121, sigma_r), (20, 24): _S(v / 121, sigma_r), (17, 18): _S(v / 121, sigma_r),
              (20, 27): 1.0, (13, 21): 1.0}
    for (y, x), s in expect.items():
        assert abs(F[y, x]) > 1e-6
        assert abs((I1[y, x] - I[y, x]) - s * F[y, x]) < 1e-14 * max(1.0, abs(F[y, x]))


def test_approximate_vs_exact_cross_bilateral_error():
    """Section 4.3 replaces the per-pair range kernel of the cross bilateral
    filter (Eq. bl_filter, Eq. normalization, guide I, filtered E) by one
    range factor per pixel (Eq. sx2, Eq. bl_filter_3). Reported here on a
    bicubic start of a 64^2 LR image: the relative RMS difference of the two
    filters, which falls to 0 as sigma_r grows (both become the normalised
    Gaussian). Measured: 0.94, 0.78, 0.49 for sigma_r = 0.05, 0.1, 0.2."""
    hr = synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 51, 128, 128).astype(np.float64)
    lr = imaging.degrade(hr, 2, to_f32=False)
    I = imaging.bicubic_up(lr, 2)
    E = imaging.bicubic_up(lr - imaging.degrade(I, 2, to_f32=False), 2)
    F = bp.gauss_filter_normalised(E, 1.5)
    rel = []
    for sr in (0.05, 0.1, 0.2, 1.0, 1e6):
        approx = bp.range_weight(I, 1.5, sr) * F
        exact = bp.exact_cross_bilateral(E, I, 1.5, sr)
        rel.append(float(np.sqrt(((approx - exact) ** 2).mean() / (exact ** 2).mean())))
    assert all(b < a for a, b in zip(rel, rel[1:])), rel
    assert 0.6 < rel[1] < 0.95 and rel[-1] < 1e-6, rel


def test_exact_filter_back_projection_limits():
    """The back-projection with the exact cross bilateral filter equals the
    approximate one when the range kernel is flat (sigma_r -> inf: both add
    the normalised Gaussian of the upsampled error), and both reduce the RMS
    LR residual of a bicubic start at the workloads' sigma_r (measured: 0.027
    to 0.022 approximate, 0.015 exact, in 3 iterations)."""
    hr = synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 52, 64, 72).astype(np.float64)
    lr = imaging.degrade(hr, 2, to_f32=False)
    I0 = imaging.bicubic_up(lr, 2)
    a = bp.backproject(I0, lr, 2, 2, 1.0, 1.5, math.inf)
    e = bp.backproject_exact(I0, lr, 2, 2, 1.0, 1.5, 1e12)
    assert np.abs(a - e).max() < 1e-10
    def rms(I):
        return float(np.sqrt(((imaging.degrade(I, 2, to_f32=False) - lr) ** 2).mean()))

    for f in (bp.backproject, bp.backproject_exact):
        out = f(I0, lr, 2, 3, 1.0, 1.5, 0.1)
        assert rms(out) < 0.9 * rms(I0)
