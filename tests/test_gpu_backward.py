"""zh_backward and the autograd wrapper against the oracle gradient (FP64).

The same upstream gradient field enters both sides; the library's forward
output is within the pixel bar of the oracle's, and its gradients with
respect to the HR residual patches and lambda are within 1e-4 relative of
the oracle's (Frobenius norm over the residual array, and at 64 random
coordinates against the largest entry). Rows that no patch uses get exactly
zero. Two backward calls give bitwise equal results.
"""
import math

import numpy as np
import pytest

import synthdata
from oracle import backward as obw
from oracle import imaging, pipeline

pytestmark = pytest.mark.gpu

REL = 1e-4
PIX_TOL = 1e-5
SMALL = dict(test_h=20, test_w=22, dict_images=4, dict_hr=64, n_dict=3000, L=8, k=4, w=32.0, K=5)
MID = dict(test_h=44, test_w=40, dict_images=8, dict_hr=128, n_dict=20000, L=8, k=8, w=32.0, K=5)
# zoom x1 (5 x 5 HR patches) and x4 (20 x 20, more values than a wave's four chunks)
SMALL1 = dict(SMALL, scale=1)
SMALL4 = dict(SMALL, scale=4, dict_hr=128)
# the parameters of the 1024^2 workload (L = 24, k = 20, K = 8, early stop 72)
HEADP = dict(test_h=40, test_w=36, dict_images=8, dict_hr=128, n_dict=20000, L=24, k=20, w=32.0, K=8)
_cache = {}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _setup(cfg, bp_iters, sigma_r, cap=0):
    key = (tuple(sorted(cfg.items())), bp_iters, sigma_r, cap)
    if key in _cache:
        return _cache[key]
    from paper_1004_3980_amd.pipeline import GpuWorkload
    wl = synthdata.scaled(synthdata.WORKLOADS["diff"], bp_iters=bp_iters, sigma_r=sigma_r, **cfg)
    g = GpuWorkload(wl)
    g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, wl.w,
                           wl.hash_seed)
    gt = wl.test_image().astype(np.float64)
    lr = imaging.degrade(gt, wl.scale)
    rec = obw.forward(pre, lr, wl.scale, wl.K, wl.lam, bp_iters, wl.sigma_s, sigma_r, cap=cap)
    _cache[key] = (wl, g, pre, gt, rec)
    return _cache[key]


def _compare(g_gpu, glam_gpu, g_ref, glam_ref, used):
    d = g_gpu.astype(np.float64) - g_ref
    assert np.linalg.norm(d) <= REL * np.linalg.norm(g_ref), (np.linalg.norm(d), np.linalg.norm(g_ref))
    rng = np.random.default_rng(5)
    rows, cols = rng.choice(used, 64), rng.integers(0, g_ref.shape[1], 64)
    assert np.all(np.abs(d[rows, cols]) <= REL * np.abs(g_ref).max())
    unused = np.setdiff1d(np.arange(g_ref.shape[0]), used)
    assert not g_gpu[unused].any()
    assert abs(glam_gpu - glam_ref) <= REL * abs(glam_ref) + 1e-12, (glam_gpu, glam_ref)


@pytest.mark.parametrize("cfg,bp_iters,sigma_r,cap", [(SMALL, 0, 0.1, 0), (SMALL, 3, 0.1, 0), (SMALL, 2, math.inf, 0),
                                                      (MID, 3, 0.1, 0), (SMALL, 3, 0.1, 20), (MID, 3, 0.1, 40),
                                                      (SMALL1, 2, 0.1, 0), (SMALL4, 2, 0.1, 0), (SMALL4, 2, 0.1, 20),
                                                      (HEADP, 3, 0.1, 72)])
def test_backward_matches_oracle_gradient(gpu_ok, cfg, bp_iters, sigma_r, cap):
    """cap > 0: the early-stop search, whose FP64 Gram matrices the lambda
    adjoint takes over; cap = 0: the union search, Gram matrices formed in the
    backward."""
    torch = _torch()
    wl, g, pre, gt, rec = _setup(cfg, bp_iters, sigma_r, cap)
    out = g.forward_record(g.lr, wl.lam)
    assert np.abs(out.cpu().numpy() - rec.out).max() <= PIX_TOL
    rng = np.random.default_rng(3)
    g_out = rng.standard_normal(rec.out.shape) * 1e-3
    g_r, g_lam = obw.backward(rec, pre, g_out)
    gt_t = torch.from_numpy(g_out.astype(np.float32)).cuda()
    g_resid = torch.empty_like(g.resid)
    g_lambda = torch.empty(1, dtype=torch.float32, device="cuda")
    g.ctx.backward(gt_t, g_resid, g_lambda)
    first = g_resid.clone(), g_lambda.clone()
    g.ctx.backward(gt_t, g_resid, g_lambda)
    assert torch.equal(first[0], g_resid) and torch.equal(first[1], g_lambda)
    used = np.unique(rec.qr.ids[rec.qr.ids >= 0])
    _compare(g_resid.cpu().numpy(), float(g_lambda.item()), g_r, g_lam, used)


def test_autograd_function_mse(gpu_ok):
    torch = _torch()
    from paper_1004_3980_amd.autograd import zoom
    wl, g, pre, gt, rec = _setup(SMALL, 3, 0.1)
    resid = g.resid.requires_grad_(True)
    lam = torch.tensor(wl.lam, dtype=torch.float64, requires_grad=True)
    gt_t = torch.from_numpy(gt.astype(np.float32)).cuda()
    out = zoom(g.lr, resid, lam, g)
    loss = ((out - gt_t) ** 2).mean()
    loss.backward()
    g_out = (2.0 * (out.detach() - gt_t) / gt.size).cpu().numpy().astype(np.float64)
    g_r, g_lam = obw.backward(rec, pre, g_out)
    used = np.unique(rec.qr.ids[rec.qr.ids >= 0])
    _compare(resid.grad.cpu().numpy(), float(lam.grad.item()), g_r, g_lam, used)
    resid.grad = None
    resid.requires_grad_(False)


def test_backward_state_errors(gpu_ok):
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    wl, g, pre, gt, rec = _setup(SMALL, 3, 0.1)
    ctx = g.ctx
    H, W = wl.scale * g.lr.shape[0], wl.scale * g.lr.shape[1]
    gr = torch.zeros((H, W), device="cuda")
    g_resid = torch.empty_like(g.resid)
    g_lambda = torch.empty(1, device="cuda")
    ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
    with pytest.raises(zb.ZHError):
        ctx.backward(gr, g_resid, g_lambda)          # before zh_reconstruct
    ctx.lle_weights(wl.lam)
    out = torch.empty((H, W), device="cuda")
    ctx.reconstruct(out)
    ctx.backproject(out, 1, wl.sigma_s, wl.sigma_r)
    ctx.backproject(out, 1, wl.sigma_s, wl.sigma_r)
    with pytest.raises(zb.ZHError):
        ctx.backward(gr, g_resid, g_lambda)          # two back-projection calls
    ctx.reconstruct(out)
    ctx.backward(gr, g_resid, g_lambda)              # the blend alone is differentiable
    assert not g_resid.any() and g_lambda.item() == 0.0


@pytest.fixture(scope="module")
def gpu_ok():
    _torch()
    return True
