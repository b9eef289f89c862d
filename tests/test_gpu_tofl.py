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


MIDC = ("mid", (("test_h", 64), ("test_w", 72), ("n_dict", 60000), ("dict_images", 16)))


# t = 1 on the tiny workload: unions of up to 381 IDs; the mid crop at t = 1
# has sets of thousands
@pytest.mark.parametrize("name,kw,t", [("tiny", (), 1), ("tiny", (), 2), ("tiny", (), 3), (*MIDC, 1)])
def test_neighbours_from_t_of_l(name, kw, t):
    """K-NN (squared l2, sequential FP64 sums on both sides), LLE and the
    blend over the t-of-L candidates, every candidate ranked however many
    there are: IDs, counts, distances bitwise."""
    wl, g, pre, _ = _case(name, kw)
    lr = g.lr.cpu().numpy()
    qr = pipeline.query(pre, lr, wl.K, wl.lam, t=t)
    if name == "tiny" and t == 1:
        assert max(len(c) for c in qr.cand) > 256
    hr_ref, _ = pipeline.reconstruct(qr, lr, wl.scale)
    g.set_mode(cap=0, rerank=0, proj=1, lle_fp64=1)
    hr = g.zoom(metric=f"t={t}").cpu().numpy().astype(np.float64)
    r = g.results()
    assert np.array_equal(r["m"], qr.m)
    assert np.array_equal(r["ids"], np.where(qr.ids >= 0, qr.ids, -1).astype(np.int32))
    assert np.array_equal(r["ncand"], np.array([len(c) for c in qr.cand], dtype=np.int32))
    for q in np.nonzero(qr.m > 0)[0]:
        assert np.array_equal(r["d2"][q, :qr.m[q]], qr.d2[q, :qr.m[q]].astype(np.float32)), q
    dw = np.abs(r["w"].astype(np.float64) - qr.weights)
    assert (dw <= 2.0 ** -23 * np.abs(qr.weights) + 1e-10).all(), dw.max()
    assert np.abs(hr - hr_ref).max() < 1e-5
