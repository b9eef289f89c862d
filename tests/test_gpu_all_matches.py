"""LLE over all M matches (zh_lle_all; Section 4.2, Eq. LinSys and Eq. HR_Rec
with m over every match the early-stop search found) against the oracle's
all-matches mode: candidate lists bitwise (ascending, -1 past M); weights
|dw| <= 2^-23 |w| + 1e-9 max|w| (FP64 solves on both sides in different
orders, condition number <= 1 + 1/lambda, then rounded to fp32); pixels and
back-projected pixels within 1e-5."""
import numpy as np
import pytest

import synthdata
from oracle import backproject as obp
from oracle import pipeline

pytestmark = pytest.mark.gpu

CASES = [("tiny", (("w", 16.0),), 24),
         ("mid", (("w", 80.0), ("test_h", 64), ("test_w", 56), ("n_dict", 60_000), ("dict_images", 16)), 48),
         ("tiny", (("w", 16.0), ("scale", 3), ("n_dict", 10_000)), 24),
         ("precision", (("n_dict", 100_000), ("dict_images", 8)), 72)]
# the 1024^2 workload's parameters on the top-left 40 x 36 crop of its LR image
CROP = {"precision": (40, 36)}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


@pytest.mark.parametrize("name,kw,cap", CASES)
def test_all_matches_against_oracle(name, kw, cap):
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    wl = synthdata.scaled(synthdata.WORKLOADS[name], cap=cap, **dict(kw))
    g = GpuWorkload(wl)
    g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
    if name in CROP:
        ch, cw = CROP[name]
        g.lr = g.lr[:ch, :cw].contiguous()
        g.h, g.w = ch, cw
        g.hr_out = torch.empty((wl.scale * ch, wl.scale * cw), device="cuda")
    lr_np = g.lr.cpu().numpy()
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, wl.w,
                           wl.hash_seed)
    qr = pipeline.query(pre, lr_np, wl.K, wl.lam, cap=cap, all_matches=True)
    hr_ref, _ = pipeline.reconstruct(qr, lr_np, wl.scale)
    hb_ref = obp.backproject(hr_ref, lr_np, wl.scale, wl.bp_iters, wl.blur_sigma, wl.sigma_s, wl.sigma_r)
    Q = len(qr.pos)
    ids = torch.empty((Q, cap), dtype=torch.int32, device="cuda")
    w = torch.empty((Q, cap), dtype=torch.float32, device="cuda")
    g.ctx.query(g.lr, g.h, g.w, wl.scale, wl.K)
    g.ctx.lle_all(wl.lam, ids, w)
    out = torch.empty_like(g.hr_out)
    g.ctx.reconstruct(out)
    g.ctx.sync()
    ids_n, w_n = ids.cpu().numpy(), w.cpu().numpy().astype(np.float64)
    M = np.array([len(c) for c in qr.cand])
    assert (M > wl.K).sum() > 0.2 * Q, "few patches with more matches than K"
    for q in range(Q):
        mq = M[q]
        assert np.array_equal(ids_n[q, :mq], qr.cand[q]), q
        assert (ids_n[q, mq:] == -1).all() and (w_n[q, mq:] == 0.0).all(), q
        if mq == 0:
            continue
        ref = qr.all_weights[q]
        dw = np.abs(w_n[q, :mq] - ref)
        assert (dw <= 2.0 ** -23 * np.abs(ref) + 1e-9 * np.abs(ref).max()).all(), (q, dw.max())
    assert np.abs(out.cpu().numpy().astype(np.float64) - hr_ref).max() < 1e-5
    hb = g.backproject(out.clone())
    assert np.abs(hb.cpu().numpy().astype(np.float64) - hb_ref).max() < 1e-5
    # the adjoint covers the K nearest only; the weights of the K nearest are gone
    g_resid = torch.empty_like(g.resid)
    g_lam = torch.empty(1, device="cuda")
    with pytest.raises(zb.ZHError) as e:
        g.ctx.backward(torch.zeros_like(out), g_resid, g_lam)
    assert e.value.status == zb.ZH_EUNSUPPORTED
    with pytest.raises(zb.ZHError) as e:
        g.ctx.get_results(w=torch.empty((Q, wl.K), device="cuda"))
    assert e.value.status == zb.ZH_ESTATE
    # back to the K nearest
    g.ctx.lle_weights(wl.lam)
    g.ctx.reconstruct(out)
    hr_k, _ = pipeline.reconstruct(pipeline.query(pre, lr_np, wl.K, wl.lam, cap=cap), lr_np, wl.scale)
    assert np.abs(out.cpu().numpy().astype(np.float64) - hr_k).max() < 1e-5


def test_all_matches_needs_the_early_stop():
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    wl = synthdata.WORKLOADS["tiny"]
    g = GpuWorkload(wl)
    for cap in (0, 96):
        g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
        g.ctx.query(g.lr, g.h, g.w, wl.scale, wl.K)
        with pytest.raises(zb.ZHError) as e:
            g.ctx.lle_all(wl.lam)
        assert e.value.status == zb.ZH_EUNSUPPORTED
