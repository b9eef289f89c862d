"""Pins of the oracle's back-projection (Eq. Err_img and the update after it)
and its approximate cross bilateral filter (Section 4.3) against library
filters, fixed points and convergence."""
import math

import numpy as np
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
