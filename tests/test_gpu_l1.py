"""K nearest candidates under l1 (zh_knn_l1) against the oracle: neighbour
IDs, counts and l1 distances bit-exact (both sides sum |q_i - x_i| in index
order in FP64), LLE weights and pixels to the bars of the l2 path."""
import numpy as np
import pytest

import synthdata
from oracle import pipeline

pytestmark = pytest.mark.gpu

CASES = [("tiny", (), 12), ("tiny", (("scale", 4), ("n_dict", 6000), ("w", 8.0)), 12),
         ("mid", (("test_h", 96), ("test_w", 80)), 40)]
_state = {}


def _case(name, kw, cap):
    key = (name, kw, cap)
    if key not in _state:
        import torch
        assert torch.cuda.is_available(), "GPU test needs a GPU"
        from paper_1004_3980_amd.pipeline import GpuWorkload
        wl = synthdata.scaled(synthdata.WORKLOADS[name], **dict(kw))
        g = GpuWorkload(wl)
        pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, wl.w,
                               wl.hash_seed)
        lr = g.lr.cpu().numpy()
        qr = pipeline.query(pre, lr, wl.K, wl.lam, cap=cap, metric="l1")
        hr, _ = pipeline.reconstruct(qr, lr, wl.scale)
        _state[key] = (wl, g, qr, hr)
    return _state[key]


@pytest.mark.parametrize("rerank", [0, 32])
@pytest.mark.parametrize("name,kw,cap", CASES)
def test_l1_neighbours_weights_pixels(name, kw, cap, rerank):
    wl, g, qr, hr_ref = _case(name, kw, cap)
    g.set_mode(cap=cap, rerank=rerank, proj=1, lle_fp64=1)
    hr = g.zoom(metric="l1").cpu().numpy().astype(np.float64)
    r = g.results()
    assert np.array_equal(r["m"], qr.m)
    assert np.array_equal(r["ids"], np.where(qr.ids >= 0, qr.ids, -1).astype(np.int32))
    ok = qr.m > 0
    for q in np.nonzero(ok)[0][::7]:
        assert np.array_equal(r["d2"][q, :qr.m[q]], qr.d2[q, :qr.m[q]].astype(np.float32)), q
    dw = np.abs(r["w"].astype(np.float64) - qr.weights)
    assert (dw <= 2.0 ** -23 * np.abs(qr.weights) + 1e-10).all(), dw.max()
    assert np.abs(hr - hr_ref).max() < 1e-5


def test_l1_needs_the_early_stop():
    from paper_1004_3980_amd import zoomhash as zb
    wl, g, _, _ = _case(*CASES[0])
    g.set_mode(cap=0, rerank=0, proj=1, lle_fp64=1)
    g.ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
    with pytest.raises(zb.ZHError):
        g.ctx.knn_l1()
