"""Pins of the oracle's gradients (oracle/backward.py).

- Each one-axis operator matrix, applied as A_y X A_x^T, reproduces the
  forward function it stands for (degradation, bicubic upsampling,
  normalised Gaussian, box mean), written independently in `imaging` and
  `backproject`; the adjoint of each is then its transpose, which the
  dot-product test <A x, y> = <x, A^T y> checks through the forward function.
- dw/dlambda of the LLE weights against central differences, and its sum is
  0 (the weights sum to 1 for every lambda).
- The whole gradient (back-projection, blend, synthesis, LLE through lambda)
  against central differences of the FP64 loss, step 1e-3, at 64 random
  coordinates of the residual patches that some patch uses, and at lambda.
"""
import math

import numpy as np
import pytest

import synthdata
from oracle import backproject, backward, imaging, lle, pipeline

RNG = np.random.default_rng(20240611)


@pytest.mark.parametrize("scale", [1, 2, 3, 4])
@pytest.mark.parametrize("n_hr", [23, 36])
def test_axis_matrices_reproduce_forward_operators(scale, n_hr):
    H, W = n_hr, n_hr + 5
    h, w = (H + scale - 1) // scale, (W + scale - 1) // scale
    X = RNG.random((H, W))
    ops = backward.bp_ops(H, W, h, w, scale, 1.0, 1.5)
    assert np.allclose(backward.sep(ops.Dy, X, ops.Dx), imaging.degrade(X, scale, to_f32=False),
                       rtol=0, atol=1e-13)
    e = RNG.random((h, w)) - 0.5
    assert np.allclose(backward.sep(ops.Uy, e, ops.Ux), imaging.bicubic_up(e, scale, H, W),
                       rtol=0, atol=1e-13)
    assert np.allclose(backward.sep(ops.Ny, X, ops.Nx), backproject.gauss_filter_normalised(X, 1.5),
                       rtol=0, atol=1e-13)
    R = int(math.ceil(3 * 1.5))
    assert np.allclose(backward.sep(ops.By, X, ops.Bx), backproject.box_mean(X, R), rtol=0, atol=1e-12)


def test_dot_product_adjoints():
    scale, H, W = 2, 30, 26
    h, w = H // scale, W // scale
    ops = backward.bp_ops(H, W, h, w, scale, 1.0, 1.5)
    R = int(math.ceil(3 * 1.5))
    x = RNG.random((H, W))
    y_lr = RNG.random((h, w))
    y = RNG.random((H, W))
    e = RNG.random((h, w))
    # degradation: HR -> LR
    lhs = np.sum(imaging.degrade(x, scale, to_f32=False) * y_lr)
    assert math.isclose(lhs, np.sum(x * backward.sep(ops.Dy.T, y_lr, ops.Dx.T)), rel_tol=1e-12)
    # bicubic: LR -> HR
    lhs = np.sum(imaging.bicubic_up(e, scale, H, W) * y)
    assert math.isclose(lhs, np.sum(e * backward.sep(ops.Uy.T, y, ops.Ux.T)), rel_tol=1e-12)
    # normalised Gaussian and box mean: HR -> HR
    lhs = np.sum(backproject.gauss_filter_normalised(x, 1.5) * y)
    assert math.isclose(lhs, np.sum(x * backward.sep(ops.Ny.T, y, ops.Nx.T)), rel_tol=1e-12)
    lhs = np.sum(backproject.box_mean(x, R) * y)
    assert math.isclose(lhs, np.sum(x * backward.sep(ops.By.T, y, ops.Bx.T)), rel_tol=1e-12)


def test_lle_dw_dlambda():
    D, M = 30, 6
    q = RNG.standard_normal(D)
    Y = q + 0.3 * RNG.standard_normal((M, D))
    lam, h = 1e-2, 1e-6
    w, dw = backward.lle_dw_dlambda(q, Y, lam)
    assert np.allclose(w, lle.lle_weights(q, Y, lam), rtol=0, atol=1e-13)
    fd = (lle.lle_weights(q, Y, lam + h) - lle.lle_weights(q, Y, lam - h)) / (2 * h)
    assert np.allclose(dw, fd, rtol=1e-6, atol=1e-9)
    assert abs(dw.sum()) < 1e-12
    # every neighbour equal to the query: uniform weights for every lambda
    w0, dw0 = backward.lle_dw_dlambda(q, np.repeat(q[None], M, 0), lam)
    assert np.allclose(w0, 1.0 / M) and not dw0.any()


def _small_case(bp_iters, sigma_r, scale=2):
    wl = synthdata.scaled(synthdata.WORKLOADS["diff"], test_h=20, test_w=22, dict_images=4,
                          dict_hr=64 if scale < 4 else 128, n_dict=3000, L=8, k=4, w=32.0, K=5,
                          bp_iters=bp_iters, sigma_r=sigma_r, scale=scale)
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k,
                           wl.w, wl.hash_seed)
    gt = wl.test_image().astype(np.float64)
    lr = imaging.degrade(gt, wl.scale)
    rec = backward.forward(pre, lr, wl.scale, wl.K, wl.lam, bp_iters, wl.sigma_s, sigma_r)
    return wl, pre, gt, rec


@pytest.mark.parametrize("bp_iters,sigma_r,scale", [(0, 0.1, 2), (3, 0.1, 2), (2, math.inf, 2), (2, 0.1, 1),
                                                   (2, 0.1, 4)])
def test_gradient_matches_central_differences(bp_iters, sigma_r, scale):
    wl, pre, gt, rec = _small_case(bp_iters, sigma_r, scale)
    n_pix = gt.size
    assert (rec.qr.m > 0).mean() > 0.5

    def loss(out):
        return float(np.sum((out - gt) ** 2) / n_pix)

    assert np.allclose(backward.output_given(rec, pre, pre.dictionary.resid, wl.lam), rec.out,
                       rtol=0, atol=1e-12)
    g_out = 2.0 * (rec.out - gt) / n_pix
    g_r, g_lam = backward.backward(rec, pre, g_out)
    used = np.unique(rec.qr.ids[rec.qr.ids >= 0])
    rows = RNG.choice(used, 64)
    cols = RNG.integers(0, g_r.shape[1], 64)
    h = 1e-3
    resid = pre.dictionary.resid.astype(np.float64)
    scale = np.abs(g_r[used]).max()
    for n, c in zip(rows, cols):
        rp, rm = resid.copy(), resid.copy()
        rp[n, c] += h
        rm[n, c] -= h
        fd = (loss(backward.output_given(rec, pre, rp, wl.lam)) -
              loss(backward.output_given(rec, pre, rm, wl.lam))) / (2 * h)
        assert abs(fd - g_r[n, c]) <= 1e-4 * scale, (n, c, fd, g_r[n, c])
    hl = 1e-3 * wl.lam
    fd = (loss(backward.output_given(rec, pre, resid, wl.lam + hl)) -
          loss(backward.output_given(rec, pre, resid, wl.lam - hl))) / (2 * hl)
    assert abs(fd - g_lam) <= 1e-4 * abs(g_lam) + 1e-12, (fd, g_lam)
    # rows no patch uses get no gradient
    unused = np.setdiff1d(np.arange(g_r.shape[0]), used)
    assert not g_r[unused].any()
