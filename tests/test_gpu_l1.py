"""K nearest candidates under l1 (zh_knn_l1) against the oracle: neighbour
IDs, counts and l1 distances bit-exact (both sides sum |q_i - x_i| in index
order in FP64), LLE weights and pixels to the bars of the l2 path. At D = 100
the library prunes candidates with its l1 screen first; the last case (wide
bins) and the tie test run that path, the tiny ones (D = 25) the unscreened
one."""
import numpy as np
import pytest

import synthdata
from oracle import pipeline

pytestmark = pytest.mark.gpu

CASES = [("tiny", (), 12), ("tiny", (("scale", 4), ("n_dict", 6000), ("w", 8.0)), 12),
         ("mid", (("test_h", 96), ("test_w", 80)), 40),
         # bins wide enough at D = 100: 7,000 of the 7,728 patches have more
         # than K candidates, so the screen runs for them
         ("mid", (("w", 80.0), ("test_h", 96), ("test_w", 88), ("n_dict", 100_000), ("dict_images", 32)), 48)]
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
        _state[key] = (wl, g, qr, hr, pre)
    return _state[key]


@pytest.mark.parametrize("rerank", [0, 32])
@pytest.mark.parametrize("name,kw,cap", CASES)
def test_l1_neighbours_weights_pixels(name, kw, cap, rerank):
    wl, g, qr, hr_ref, _ = _case(name, kw, cap)
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
    wl, g, _, _, _ = _case(*CASES[0])
    g.set_mode(cap=0, rerank=0, proj=1, lle_fp64=1)
    g.ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
    with pytest.raises(zb.ZHError):
        g.ctx.knn_l1()


def test_l1_screen_ties_and_near_ties():
    """Dictionary rows copied over others (equal l1 distances, ties broken by
    ID), copies one ulp away in one coordinate, and rows scaled by 1000 (a
    coarse grid, loose bounds): the screen may prune only candidates farther
    than K others, so neighbours, counts and distances stay bitwise the
    oracle's over the same modified features."""
    import torch
    from oracle import imaging, lsh
    wl, g, qr, _, pre = _case(*CASES[3])
    cap = CASES[3][2]
    feat = pre.dictionary.feat.copy()
    rng = np.random.default_rng(11)
    two = qr.ids[qr.m >= 2][:, :2]
    pick = two[rng.choice(len(two), 300, replace=False)]
    for a, b in pick[:100]:
        feat[b] = feat[a]
    for a, b in pick[100:200]:
        feat[b] = feat[a]
        feat[b, 7] = np.nextafter(feat[a, 7], np.float32(np.inf))
    for _, b in pick[200:]:
        feat[b] = feat[b] * np.float32(1000.0)
    keys = lsh.bucket_keys(lsh.codes(feat, pre.alpha, pre.beta, pre.w), pre.L, pre.k)
    dic = imaging.Dictionary(feat, pre.dictionary.resid, pre.dictionary.scale, pre.dictionary.mode,
                             pre.dictionary.lr_mean)
    pre2 = pipeline.Prepared(dic, pre.alpha, pre.beta, lsh.Tables(keys), keys, pre.L, pre.k, pre.w)
    lr = g.lr.cpu().numpy()
    ref = pipeline.query(pre2, lr, wl.K, wl.lam, cap=cap, metric="l1", synthesize=False)
    ft = torch.from_numpy(feat).to(g.dev)
    ctx = g.ctx
    try:
        ctx.build_tables(ft, g.resid, g.n, g.D, wl.scale, wl.feat_mode, wl.L, wl.k, wl.w, wl.hash_seed)
        g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
        ctx.query(g.lr, g.h, g.w, wl.scale, wl.K)
        ctx.knn_l1()
        ctx.lle_weights(wl.lam)
        r = g.results()
    finally:
        ctx.build_tables(g.feat, g.resid, g.n, g.D, wl.scale, wl.feat_mode, wl.L, wl.k, wl.w, wl.hash_seed)
    assert np.array_equal(r["m"], ref.m)
    assert np.array_equal(r["ids"], np.where(ref.ids >= 0, ref.ids, -1).astype(np.int32))
    for q in np.nonzero(ref.m > 0)[0]:
        assert np.array_equal(r["d2"][q, :ref.m[q]], ref.d2[q, :ref.m[q]].astype(np.float32)), q
    # the copies do tie: some patch has two neighbours at the same l1 distance
    assert any(len(set(ref.d2[q, :ref.m[q]])) < ref.m[q] for q in range(len(ref.m)))


@pytest.mark.parametrize("case", [0, 3])
def test_query_metric_l1_equals_rerank(case):
    """zh_query under ZH_METRIC_L1 gives the neighbours, l1 distances, counts,
    weights and pixels of zh_query under l2 followed by zh_knn_l1, bitwise
    (the tiny case through the unscreened ranking, the wide-bin 256^2 case
    through the l1 screen), and the oracle's."""
    import torch
    wl, g, qr, hr_ref, _ = _case(*CASES[case])
    cap = CASES[case][2]
    g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
    a = g.zoom(metric="l1").clone()
    ra = g.results()
    b = g.zoom(metric="l1q").clone()
    rb = g.results()
    for k in ("ids", "d2", "m", "w", "ncand", "nsurv"):
        assert np.array_equal(ra[k], rb[k]), k
    assert torch.equal(a, b)
    # survivors of the l1 pass: at least the neighbours, at most the candidates;
    # all of them without the screen (D = 25), far fewer with it (D = 100)
    M = np.minimum(rb["ncand"], cap)
    assert (rb["m"] <= rb["nsurv"]).all() and (rb["nsurv"] <= M).all()
    if wl.D == 25:
        assert np.array_equal(rb["nsurv"], M)
    else:
        assert rb["nsurv"][M > wl.K].mean() < 0.5 * M[M > wl.K].mean()
    assert np.array_equal(rb["ids"], np.where(qr.ids >= 0, qr.ids, -1).astype(np.int32))
    assert np.abs(b.cpu().numpy().astype(np.float64) - hr_ref).max() < 1e-5


def test_query_metric_errors():
    import torch
    from paper_1004_3980_amd import zoomhash as zb
    wl, g, _, _, _ = _case(*CASES[0])
    ctx = g.ctx
    with pytest.raises(KeyError):
        ctx.set_query_metric("l3")
    assert ctx.lib.zh_set_query_metric(ctx.h, 2) == zb.ZH_EINVAL
    g.set_mode(cap=0, rerank=0, proj=1, lle_fp64=1)
    ctx.set_query_metric("l1")
    try:
        with pytest.raises(zb.ZHError):   # the l1 metric needs the early stop
            ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
        g.set_mode(cap=12, rerank=0, proj=1, lle_fp64=1)
        ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
        out = torch.empty((wl.scale * g.h, wl.scale * g.w), device=g.dev)
        with pytest.raises(zb.ZHError):   # the batched form ranks by squared l2
            ctx.run_batch([g.lr], [out], [wl.scale], wl.K, wl.lam, 1, 1.5, 0.1)
    finally:
        ctx.set_query_metric("l2")
    ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
