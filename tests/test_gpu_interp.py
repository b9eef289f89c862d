"""The interpolated pairing of Section 2.1 (LR training images interpolated
back to the HR size, both cut at the same places into 5 x 5 patches) on the
GPU against the oracle: the interpolated LR images (zh_upsample) and the
dictionary (zh_make_dictionary_interp) bitwise; the zoom-1 query of the
interpolated test image with its neighbours bitwise, weights to the path's
bar and pixels within 1e-5; the back-projection against the LR image
(zh_backproject_lr) within 1e-5."""
import numpy as np
import pytest

import synthdata
from oracle import backproject as obp
from oracle import imaging, pipeline

pytestmark = pytest.mark.gpu

SEED = synthdata.SEED_BASE + 7400
_state = {}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


@pytest.mark.parametrize("s,h,w", [(1, 17, 23), (2, 31, 40), (3, 20, 13), (4, 9, 11)])
def test_upsample_bit_exact(s, h, w):
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    ctx = zb.Context(0)
    lr = synthdata.fractal_voronoi_image(SEED + s, h, w)
    out = torch.empty((s * h, s * w), device="cuda")
    ctx.upsample(torch.from_numpy(lr).cuda(), h, w, s, out)
    ctx.sync()
    assert np.array_equal(out.cpu().numpy(), imaging.interpolated_lr(lr, s))
    ctx.close()


def _dictionary(s, mode, n=20000, n_img=8, H=128):
    torch = _torch()
    key = (s, mode, n, n_img, H)
    if key in _state:
        return _state[key]
    from paper_1004_3980_amd import zoomhash as zb
    ctx = zb.Context(0)
    hr = synthdata.image_stack(SEED + 10 * s, n_img, H, H)
    pos = synthdata.sample_positions(SEED + 10 * s + 1, n_img, H, H, 5, n)
    D = 25 if mode == 0 else 100
    feat = torch.empty((n, D), device="cuda")
    resid = torch.empty((n, 25), device="cuda")
    ctx.make_dictionary_interp(torch.from_numpy(hr).cuda(), n_img, H, H, torch.from_numpy(pos.astype(np.int32)).cuda(),
                               n, s, 1.0, mode, feat, resid)
    ctx.sync()
    ref = imaging.build_dictionary_interp(hr, pos, s, mode)
    _state[key] = (ctx, hr, pos, feat, resid, ref)
    return _state[key]


@pytest.mark.parametrize("s,mode", [(2, 0), (2, 1), (3, 1), (4, 0)])
def test_dictionary_bit_exact(s, mode):
    ctx, hr, pos, feat, resid, ref = _dictionary(s, mode, n=6000 if s > 2 else 20000, H=120 if s == 3 else 128)
    assert np.array_equal(feat.cpu().numpy(), ref.feat)
    assert np.array_equal(resid.cpu().numpy(), ref.resid)


@pytest.mark.parametrize("mode,L,k,w,cap", [(0, 8, 12, 8.0, 0), (0, 8, 12, 8.0, 24), (1, 16, 16, 32.0, 48)])
def test_zoom_through_interpolated_pairs(mode, L, k, w, cap):
    torch = _torch()
    ctx, hr, pos, feat, resid, ref = _dictionary(2, mode)
    K, lam, s = 5, 1e-3, 2
    ctx.set_query_opts(cap=cap, rerank=0, proj=1, lle_fp64=1)
    ctx.build_tables(feat, resid, feat.shape[0], feat.shape[1], 1, mode, L, k, w, 5)
    lr = synthdata.fractal_voronoi_image(SEED + 99, 48, 40)
    lr_t = torch.from_numpy(lr).cuda()
    up = torch.empty((96, 80), device="cuda")
    ctx.upsample(lr_t, 48, 40, s, up)
    ctx.query(up, 96, 80, 1, K)
    ctx.lle_weights(lam)
    out = torch.empty((96, 80), device="cuda")
    ctx.reconstruct(out)
    Q = 92 * 76
    ids = torch.empty((Q, K), dtype=torch.int32, device="cuda")
    m = torch.empty(Q, dtype=torch.int32, device="cuda")
    wt = torch.empty((Q, K), device="cuda")
    ctx.get_results(ids, None, m, wt, None)
    hb = out.clone()
    ctx.backproject_lr(hb, lr_t, 48, 40, s, 3, 1.5, 0.1)
    ctx.sync()
    pre = pipeline.prepare_interp(hr, pos, s, mode, L, k, w, 5)
    qr, up_ref, hr_ref, hb_ref = pipeline.run_interp(pre, lr, s, K, lam, 3, cap=cap)
    assert np.array_equal(up.cpu().numpy(), up_ref)
    assert (qr.m > 0).mean() > 0.4
    assert np.array_equal(m.cpu().numpy(), qr.m)
    assert np.array_equal(ids.cpu().numpy(), np.where(qr.ids >= 0, qr.ids, -1).astype(np.int32))
    dw = np.abs(wt.cpu().numpy().astype(np.float64) - qr.weights)
    assert (dw <= 2.0 ** -23 * np.abs(qr.weights) + 1e-10).all(), dw.max()
    assert np.abs(out.cpu().numpy() - hr_ref).max() < 1e-5
    assert np.abs(hb.cpu().numpy() - hb_ref).max() < 1e-5


def test_interpolated_dictionary_argument_errors():
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    ctx = zb.Context(0)
    hr = torch.zeros((1, 30, 30), device="cuda")
    feat = torch.zeros((1, 25), device="cuda")
    resid = torch.zeros((1, 25), device="cuda")
    for pos, H, s in (([0, 26, 0], 30, 2), ([0, 0, 26], 30, 2), ([1, 0, 0], 30, 2), ([0, 0, 0], 30, 4)):
        p = torch.tensor([pos], dtype=torch.int32, device="cuda")
        with pytest.raises(zb.ZHError) as e:
            ctx.make_dictionary_interp(hr, 1, H, H, p, 1, s, 1.0, 0, feat, resid)
        assert e.value.status == zb.ZH_EINVAL, (pos, s)
    ctx.close()
