"""Pins of the training-crop sampler and the bucket-entropy diagnostic
(oracle/training.py) against closed forms, brute force and statistics."""
import math

import numpy as np
import pytest

import synthdata
from oracle import lsh, training


def test_gradient_weights_closed_form_on_a_ramp():
    a = 0.125
    img = np.tile(a * np.arange(9, dtype=np.float32), (6, 1))      # I(r, c) = a c
    q = training.gradient_weights(img)
    # interior: dx = 2a, dy = 0; first and last column: dx = a (replicate border)
    assert np.all(q[:, 1:-1] == int(2 * a * 2 ** 20))
    assert np.all(q[:, 0] == int(a * 2 ** 20)) and np.all(q[:, -1] == int(a * 2 ** 20))
    # the transposed ramp weighs the same way along rows
    assert np.array_equal(training.gradient_weights(img.T.copy()), q.T)


def test_gradient_weights_brute_force_and_saturation():
    img = synthdata.fractal_voronoi_image(11, 7, 10)
    q = training.gradient_weights(img)
    H, W = img.shape
    for r in range(H):
        for c in range(W):
            x = lambda rr, cc: float(img[min(max(rr, 0), H - 1), min(max(cc, 0), W - 1)])
            g = abs(x(r, c + 1) - x(r, c - 1)) + abs(x(r + 1, c) - x(r - 1, c))
            assert q[r, c] == math.floor(g * 2 ** 20)
    big = np.zeros((3, 3), np.float32)
    big[1, 1] = 1e30
    big[0, 0] = np.nan
    qb = training.gradient_weights(big)
    assert qb[1, 0] == training.QMAX and qb[0, 1] == training.QMAX   # 1e30 and NaN saturate
    assert qb[2, 2] == 0


def test_centres_brute_force_on_tiny_images():
    img = synthdata.fractal_voronoi_image(12, 5, 6)
    draws = synthdata.crop_draws(13, 1, 400)[0]
    got = training.sample_centres(img, draws)
    q = [int(v) for v in training.gradient_weights(img).ravel()]
    T = sum(q)
    for x, g in zip(draws, got):
        t = int(x) % T
        acc, idx = 0, None
        for i, v in enumerate(q):
            acc += v
            if acc > t:
                idx = i
                break
        assert g == idx
        assert q[g] > 0                       # a pixel without gradient is never drawn


def test_centres_of_a_flat_image_are_uniform_and_an_edge_is_found():
    flat = np.full((8, 9), 0.5, np.float32)
    draws = synthdata.crop_draws(14, 1, 1000)[0]
    got = training.sample_centres(flat, draws)
    assert np.array_equal(got, (draws % np.uint64(72)).astype(np.int64))
    edge = np.zeros((20, 30), np.float32)
    edge[:, 17:] = 1.0                        # one vertical step between columns 16 and 17
    cols = training.sample_centres(edge, draws) % 30
    assert set(np.unique(cols)) == {16, 17}


def test_centre_frequencies_follow_the_weights():
    img = synthdata.fractal_voronoi_image(15, 6, 7)
    draws = synthdata.crop_draws(16, 1, 200_000)[0]
    got = training.sample_centres(img, draws)
    q = training.gradient_weights(img).ravel().astype(np.float64)
    p = q / q.sum()
    f = np.bincount(got, minlength=q.size) / draws.size
    # binomial standard deviation per pixel; 5 sigma
    assert np.all(np.abs(f - p) <= 5 * np.sqrt(p * (1 - p) / draws.size) + 1e-12)


def test_crops_are_clamped_sub_images():
    stack = synthdata.image_stack(17, 2, 40, 50)
    draws = synthdata.crop_draws(18, 2, 30)
    corners, crops = training.sample_crops(stack, draws, 24)
    assert corners.min() >= 0 and corners[..., 0].max() <= 16 and corners[..., 1].max() <= 26
    for i in range(2):
        cen = training.sample_centres(stack[i], draws[i])
        for j in range(30):
            r, c = divmod(int(cen[j]), 50)
            assert corners[i, j, 0] == min(max(r - 12, 0), 16) and corners[i, j, 1] == min(max(c - 12, 0), 26)
            r0, c0 = corners[i, j]
            assert np.array_equal(crops[i, j], stack[i, r0:r0 + 24, c0:c0 + 24])
    # a crop as large as the image is the image
    full_c, full = training.sample_crops(stack[:1, :24, :24].copy(), draws[:1, :3], 24)
    assert not full_c.any() and np.array_equal(full[0, 2], stack[0, :24, :24])


def test_bucket_entropy_closed_forms():
    N = 4096
    keys = np.zeros((N, 4), np.uint64)
    keys[:, 1] = np.arange(N) % 16            # 16 equal buckets
    keys[:, 2] = np.arange(N)                 # every row alone
    keys[:, 3] = (np.arange(N) < 1024)        # p = 1/4, 3/4
    h = training.bucket_entropy(keys)
    assert h[0] == 0.0
    assert abs(h[1] - 4.0) < 1e-12
    assert abs(h[2] - training.entropy_bound(N)) < 1e-12
    assert abs(h[3] - (0.25 * 2 + 0.75 * math.log2(4 / 3))) < 1e-12


def test_bucket_entropy_of_real_tables_brute_force_and_bounds():
    wl = synthdata.scaled(synthdata.WORKLOADS["tiny"], n_dict=3000)
    from oracle import imaging
    d = imaging.build_dictionary(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode)
    alpha, beta = lsh.hash_params(wl.hash_seed, wl.L, wl.k, wl.D, wl.w)
    keys = lsh.bucket_keys(lsh.codes(d.feat, alpha, beta, wl.w), wl.L, wl.k)
    h = training.bucket_entropy(keys)
    for l in (0, wl.L - 1):
        counts = {}
        for key in keys[:, l]:
            counts[int(key)] = counts.get(int(key), 0) + 1
        ref = -sum(c / 3000 * math.log2(c / 3000) for c in counts.values())
        assert abs(h[l] - ref) < 1e-12
    assert np.all(h > 0) and np.all(h <= training.entropy_bound(3000) + 1e-12)
    # wider bins hold more rows each: the mean entropy falls as r grows
    a4, b4 = lsh.hash_params(wl.hash_seed, wl.L, wl.k, wl.D, 4 * wl.w)
    keys2 = lsh.bucket_keys(lsh.codes(d.feat, a4, b4, 4 * wl.w), wl.L, wl.k)
    assert training.bucket_entropy(keys2).mean() < h.mean()
