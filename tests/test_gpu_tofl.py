"""The t-of-L candidate criterion (zh_candidates_t) against the oracle:
candidate sets and counts bit-exact for t = 1 (the union), 2, 3 and L."""
import numpy as np
import pytest

import synthdata
from oracle import lsh, pipeline

pytestmark = pytest.mark.gpu

_state = {}


def _case(name, kw):
    key = (name, kw)
    if key not in _state:
        import torch
        assert torch.cuda.is_available(), "GPU test needs a GPU"
        from paper_1004_3980_amd.pipeline import GpuWorkload
        wl = synthdata.scaled(synthdata.WORKLOADS[name], **dict(kw))
        g = GpuWorkload(wl)
        g.set_mode(cap=0, rerank=0, proj=1, lle_fp64=1)
        g.ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
        pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, wl.w,
                               wl.hash_seed)
        qr = pipeline.query(pre, g.lr.cpu().numpy(), wl.K, wl.lam, synthesize=False)
        _state[key] = (wl, g, pre, qr)
    return _state[key]


@pytest.mark.parametrize("name,kw", [("tiny", ()), ("tiny", (("test_h", 50), ("test_w", 77))),
                                     ("mid", (("test_h", 64), ("test_w", 72), ("n_dict", 60000),
                                              ("dict_images", 16)))])
def test_t_of_l_sets(name, kw):
    import torch
    wl, g, pre, qr = _case(name, kw)
    Q = qr.keys.shape[0]
    for t in sorted({1, 2, 3, wl.L}):
        ref = lsh.candidates_t(pre.tables, qr.keys, t)
        cap = max(1, max(len(r) for r in ref))
        counts = torch.full((Q,), -1, dtype=torch.int32, device="cuda")
        ids = torch.full((Q, cap), -1, dtype=torch.int32, device="cuda")
        g.ctx.candidates_t(t, cap, counts, ids)
        torch.cuda.synchronize()
        c, x = counts.cpu().numpy(), ids.cpu().numpy()
        for q in range(Q):
            assert c[q] == len(ref[q]), (t, q)
            assert np.array_equal(np.sort(x[q, :c[q]]), ref[q]), (t, q)
    # a short output row: counts stay whole, the first cap_per_query are written
    ref2 = lsh.candidates_t(pre.tables, qr.keys, 2)
    counts = torch.full((Q,), -1, dtype=torch.int32, device="cuda")
    ids = torch.full((Q, 3), -1, dtype=torch.int32, device="cuda")
    g.ctx.candidates_t(2, 3, counts, ids)
    c, x = counts.cpu().numpy(), ids.cpu().numpy()
    for q in range(Q):
        assert c[q] == len(ref2[q])
        assert np.all(np.isin(x[q, :min(3, c[q])], ref2[q])) and np.all(x[q, min(3, c[q]):] == -1)


def test_t_of_l_argument_errors():
    import torch
    from paper_1004_3980_amd import zoomhash as zb
    wl, g, _, _ = _case("tiny", ())
    counts = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(zb.ZHError):
        g.ctx.candidates_t(0, 4, counts, counts)
    with pytest.raises(zb.ZHError):
        g.ctx.candidates_t(wl.L + 1, 4, counts, counts)
