"""Pins of the oracle's degradation (Section 2.1), features (Section 4.1) and
bicubic interpolation against independent library routines and closed forms."""
import numpy as np
import pytest
from scipy import ndimage

import synthdata
from oracle import imaging


def test_gauss_weights_match_scipy_kernel():
    g = imaging.gauss_weights(1.0)
    assert len(g) == 7
    delta = np.zeros(21)
    delta[10] = 1.0
    ref = ndimage.gaussian_filter1d(delta, 1.0, truncate=3.0, mode="constant")[7:14]
    assert np.allclose(g, ref, rtol=0, atol=1e-15)
    assert abs(g.sum() - 1.0) < 1e-15 and np.array_equal(g, g[::-1])


@pytest.mark.parametrize("scale", [1, 2, 3, 4])
def test_degrade_matches_scipy_blur_then_decimate(scale):
    hr = synthdata.fractal_voronoi_image(5, 60, 48).astype(np.float64)
    ref = ndimage.gaussian_filter(hr, 1.0, truncate=3.0, mode="nearest")[::scale, ::scale]
    got = imaging.degrade(hr, scale, 1.0, to_f32=False)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() < 1e-14
    assert np.array_equal(imaging.degrade(hr, scale), got.astype(np.float32))


def test_degrade_constant_is_constant():
    lr = imaging.degrade(np.full((20, 30), 0.625), 2, to_f32=False)
    assert np.abs(lr - 0.625).max() < 1e-15


def test_gradient_maps_match_scipy_correlation():
    img = synthdata.fractal_voronoi_image(6, 40, 37)
    I = img.astype(np.float64)
    maps = imaging.gradient_maps(img)
    k1 = [-1.0, 0.0, 1.0]
    k2 = [-1.0, 0.0, 2.0, 0.0, -1.0]
    ref = [ndimage.correlate1d(I, k1, axis=1, mode="nearest"),
           ndimage.correlate1d(I, k1, axis=0, mode="nearest"),
           ndimage.correlate1d(I, k2, axis=1, mode="nearest"),
           ndimage.correlate1d(I, k2, axis=0, mode="nearest")]
    for ch in range(4):
        assert np.abs(maps[ch].astype(np.float64) - ref[ch]).max() <= 1e-7


def test_features_layout_and_invariants():
    lr = synthdata.fractal_voronoi_image(7, 30, 30)
    ij = np.array([[0, 0], [3, 7], [25, 25], [12, 0]])
    f0 = imaging.features(lr, ij, 0)
    # mean-removed pixels: zero mean, and pixels = v + mean
    mu = imaging.patch_mean(lr, ij)
    assert np.abs(f0.astype(np.float64).sum(1)).max() < 25 * 2e-8
    for r, (i, j) in enumerate(ij):
        patch = lr[i:i + 5, j:j + 5].astype(np.float64).ravel()
        assert np.abs(f0[r] - (patch - mu[r])).max() < 1e-7
        assert abs(mu[r] - patch.mean()) < 1e-15
    f1 = imaging.features(lr, ij, 1)
    I = lr.astype(np.float64)
    dx = ndimage.correlate1d(I, [-1.0, 0.0, 1.0], axis=1, mode="nearest")
    dyy = ndimage.correlate1d(I, [-1.0, 0.0, 2.0, 0.0, -1.0], axis=0, mode="nearest")
    for r, (i, j) in enumerate(ij):
        assert np.abs(f1[r, 0:25] - dx[i:i + 5, j:j + 5].ravel()).max() <= 1e-7
        assert np.abs(f1[r, 75:100] - dyy[i:i + 5, j:j + 5].ravel()).max() <= 1e-7
    # gradient features ignore the DC level
    f1b = imaging.features(lr * 0 + lr, ij, 1)
    assert np.array_equal(f1, f1b)


def test_keys_kernel_closed_form():
    assert imaging.keys_cubic(0.0) == 1.0
    assert imaging.keys_cubic(1.0) == 0.0 and imaging.keys_cubic(2.0) == 0.0
    # partition of unity at any phase
    for t in np.linspace(0, 1, 7, endpoint=False):
        assert abs(sum(imaging.keys_cubic(t - (a - 1)) for a in range(4)) - 1.0) < 1e-15
    assert abs(imaging.keys_cubic(0.5) - 0.5625) < 1e-15
    assert abs(imaging.keys_cubic(1.5) + 0.0625) < 1e-15


@pytest.mark.parametrize("scale", [1, 2, 3, 4])
def test_bicubic_samples_and_reproduces_quadratics(scale):
    h, w = 12, 15
    lr = synthdata.fractal_voronoi_image(8, h, w).astype(np.float64)
    up = imaging.bicubic_up(lr, scale)
    assert np.array_equal(up[::scale, ::scale], lr)
    yy, xx = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    quad = 0.3 * yy * yy - 0.2 * xx * yy + 0.1 * xx + 1.0
    upq = imaging.bicubic_up(quad, scale)
    Y, X = np.meshgrid(np.arange(scale * h) / scale, np.arange(scale * w) / scale, indexing="ij")
    ref = 0.3 * Y * Y - 0.2 * X * Y + 0.1 * X + 1.0
    inner = (slice(2 * scale, (h - 3) * scale), slice(2 * scale, (w - 3) * scale))
    assert np.abs(upq[inner] - ref[inner]).max() < 1e-12


@pytest.mark.parametrize("scale", [1, 2, 4])
def test_dictionary_pairs_recover_hr_patches(scale):
    hr = synthdata.image_stack(30, 3, 40, 40)
    pos = synthdata.sample_positions(31, 3, 40 // scale, 40 // scale, 5, 100)
    d = imaging.build_dictionary(hr, pos, scale, 1)
    ps = 5 * scale
    assert d.feat.shape == (100, 100) and d.resid.shape == (100, ps * ps)
    for n in (0, 57, 99):
        im, i, j = pos[n]
        patch = hr[im][scale * i:scale * i + ps, scale * j:scale * j + ps].astype(np.float64).ravel()
        assert np.abs(d.resid[n] + d.lr_mean[n] - patch).max() < 1e-7
        lr = imaging.degrade(hr[im], scale)
        assert np.array_equal(d.feat[n], imaging.features(lr, np.array([[i, j]]), 1)[0])
    # IDs run over images in row-major order
    key = pos[:, 0] * 1_000_000 + pos[:, 1] * 1000 + pos[:, 2]
    assert np.all(np.diff(key) > 0)


def test_interpolated_pairs_at_zoom_one_are_the_plain_pairs():
    """At zoom factor 1 the interpolation is the identity (Keys' weights are
    0, 1, 0, 0 at phase 0), so interpolated pairs equal the plain pairs of a
    zoom-1 dictionary at the same positions."""
    hr = synthdata.image_stack(synthdata.SEED_BASE + 60, 2, 40, 36)
    pos = synthdata.sample_positions(synthdata.SEED_BASE + 61, 2, 40, 36, 5, 300)
    for mode in (0, 1):
        a = imaging.build_dictionary(hr, pos, 1, mode)
        b = imaging.build_dictionary_interp(hr, pos, 1, mode)
        assert np.array_equal(a.feat, b.feat) and np.array_equal(a.resid, b.resid)


def test_interpolated_lr_is_the_bicubic_and_reproduces_quadratics():
    """The interpolated LR image is the fp32 rounding of the bicubic
    interpolation; Keys' kernel reproduces quadratics exactly away from the
    border, so a quadratic LR image comes back as the same quadratic sampled
    at X / s (to the fp32 rounding)."""
    for s in (2, 3, 4):
        yy, xx = np.meshgrid(np.arange(12.0), np.arange(14.0), indexing="ij")
        lr = (0.01 * yy * yy - 0.02 * xx * yy + 0.3 * xx + 0.1).astype(np.float32)
        up = imaging.interpolated_lr(lr, s)
        assert up.dtype == np.float32 and up.shape == (12 * s, 14 * s)
        assert np.array_equal(up, imaging.bicubic_up(lr, s).astype(np.float32))
        Y, X = np.meshgrid(np.arange(12 * s) / s, np.arange(14 * s) / s, indexing="ij")
        q = 0.01 * Y * Y - 0.02 * X * Y + 0.3 * X + 0.1
        inner = (slice(2 * s, 9 * s), slice(2 * s, 11 * s))
        assert np.abs(up[inner] - q[inner]).max() < 2e-6


def test_interpolated_pairs_self_reproduction():
    """A dictionary of every interpolated pair of one image (all 5x5 patches
    of the interpolated LR image and of the HR image): each query patch of
    the interpolated image finds itself and K = 1 gives back the HR image
    (the blend of its own HR patches at zoom factor 1)."""
    from oracle import pipeline
    hr = synthdata.fractal_voronoi_image(41, 40, 44)
    lr = imaging.degrade(hr, 2)
    H, W = hr.shape
    pos = np.concatenate([np.zeros(((H - 4) * (W - 4), 1), np.int64), imaging.all_positions(H, W)], axis=1)
    pre = pipeline.prepare_interp(hr[None], pos, 2, 1, L=4, k=6, w=4.0, seed=9)
    qr, up, out, _ = pipeline.run_interp(pre, lr, 2, 1, 1e-3, 0)
    assert np.all(qr.d2[:, 0] == 0.0)
    assert np.abs(out - hr.astype(np.float64)).max() < 1e-6
