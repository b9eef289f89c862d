"""HIP path vs the FP64 oracle, stage by stage, through the C-ABI.

Bar: bit-exact for LR images, features, hash parameters, codes, keys,
candidate sets, neighbour IDs and counts; relative 1e-6 for fp32 distances;
LLE weights solved in FP64 on both sides and stored in fp32 by the library:
|dw| <= 2^-23 |w| + 1e-10 (rounding to fp32 plus a margin for the different
FP64 summation orders of a system with condition number <= 1 + 1/lambda);
1e-5 absolute
for pixels in [0, 1] (fp32 synthesis, blend and back-projection against FP64).
"""
import math

import numpy as np
import pytest

import synthdata
from oracle import backproject as obp
from oracle import imaging, lsh, pipeline

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-5
W_REL = 2.0 ** -23
W_ABS = 1e-10


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


@pytest.fixture(scope="module")
def gpu():
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    return zb.Context(0)


def _np(t):
    return t.detach().cpu().numpy()


class Case:
    """A workload on both sides: GPU (library) and CPU (oracle)."""

    def __init__(self, wl, cap=0, proj=1):
        from paper_1004_3980_amd.pipeline import GpuWorkload
        self.wl = wl
        self.g = GpuWorkload(wl, proj=proj)
        self.g.set_mode(cap=cap, proj=proj)
        hr = wl.dictionary_images()
        pos = wl.positions()
        self.pre = pipeline.prepare(hr, pos, wl.scale, wl.feat_mode, wl.L, wl.k, wl.w, wl.hash_seed)
        img = wl.test_image()
        self.lr = img if wl.test_lr_direct else imaging.degrade(img, wl.scale)
        self.qr = pipeline.query(self.pre, self.lr, wl.K, wl.lam, cap=cap)
        self.hr, self.cnt = pipeline.reconstruct(self.qr, self.lr, wl.scale)
        self.hr_bp = obp.backproject(self.hr, self.lr, wl.scale, wl.bp_iters, wl.blur_sigma,
                                     wl.sigma_s, wl.sigma_r)
        self.cap = cap


_cases = {}


def case(name, **kw):
    """Each case owns its context (tables are per scale and per context)."""
    key = (name, tuple(sorted(kw.items())))
    if key not in _cases:
        if isinstance(name, tuple):
            wl = synthdata.scaled(synthdata.WORKLOADS[name[0]], **dict(name[1]))
        else:
            wl = synthdata.WORKLOADS[name]
        _cases[key] = Case(wl, **kw)
    return _cases[key]


TINY = "tiny"
# ragged, non-square test image and a small early-stop limit
TINY_RAGGED = ("tiny", (("test_h", 50), ("test_w", 77)))
MID = "mid"
# zoom x3 (15 x 15 HR patches; the blend, synthesis and search at s = 3)
TINY3 = ("tiny", (("scale", 3), ("n_dict", 10000)))
# zoom x1 (de-blurring: 5 x 5 HR patches, the degradation is the blur alone)
# and x4 (20 x 20 HR patches, 400 values a row); bins of width 8 so that
# about two thirds of the patches find candidates (with the early stop: at x1
# some unions exceed the 8192 IDs the uncapped search takes)
TINY1 = ("tiny", (("scale", 1), ("w", 8.0)))
TINY4 = ("tiny", (("scale", 4), ("n_dict", 6000), ("w", 8.0)))
# piecewise-constant images (no noise): most gradient features are exactly
# zero, so the early-stop search meets bins of thousands of IDs and ties of
# distance 0 everywhere (the screen's bounds are all 0, every candidate is
# kept and ranked by ID)
FLAT = ("mid", (("amp", 0.0), ("test_h", 96), ("test_w", 96), ("n_dict", 60000), ("dict_images", 16)))


def test_dictionary_bit_exact(gpu):
    c = case(TINY)
    assert np.array_equal(_np(c.g.feat), c.pre.dictionary.feat)
    assert np.array_equal(_np(c.g.resid), c.pre.dictionary.resid)
    m = case(MID)
    assert np.array_equal(_np(m.g.feat), m.pre.dictionary.feat)
    assert np.array_equal(_np(m.g.resid), m.pre.dictionary.resid)


@pytest.mark.parametrize("scale", [1, 2, 3, 4])
def test_degrade_bit_exact(gpu, scale):
    torch = _torch()
    hr = synthdata.fractal_voronoi_image(77, 101, 66)
    t = torch.from_numpy(hr).cuda()
    h, w = (101 + scale - 1) // scale, (66 + scale - 1) // scale
    out = torch.empty((h, w), dtype=torch.float32, device="cuda")
    gpu.degrade(t, 1, 101, 66, scale, 1.0, out)
    assert np.array_equal(_np(out), imaging.degrade(hr, scale))


@pytest.mark.parametrize("mode", [0, 1])
def test_features_bit_exact(gpu, mode):
    torch = _torch()
    lr = synthdata.fractal_voronoi_image(78, 37, 52)
    D = 25 if mode == 0 else 100
    Q = 33 * 48
    feat = torch.empty((Q, D), dtype=torch.float32, device="cuda")
    mu = torch.empty(Q, dtype=torch.float64, device="cuda")
    gpu.features(torch.from_numpy(lr).cuda(), 37, 52, mode, feat, mu)
    pos = imaging.all_positions(37, 52)
    assert np.array_equal(_np(feat), imaging.features(lr, pos, mode))
    assert np.array_equal(_np(mu), imaging.patch_mean(lr, pos))


def test_hash_params_bitwise(gpu):
    c = case(TINY)
    wl = c.wl
    a, b = c.g.ctx.get_hash_params(wl.scale, wl.L, wl.k, wl.D)
    assert np.array_equal(a, c.pre.alpha) and np.array_equal(b, c.pre.beta)


@pytest.mark.parametrize("proj", [0, 1])
@pytest.mark.parametrize("name", [TINY, MID])
def test_codes_and_keys_bit_exact(gpu, name, proj):
    torch = _torch()
    c = case(name)
    wl = c.wl
    ctx = c.g.ctx
    ctx.set_query_opts(cap=c.cap, proj=proj)
    for feat in (c.qr.feat, c.pre.dictionary.feat[:50_000]):
        n = feat.shape[0]
        ft = torch.from_numpy(feat).cuda()
        codes = torch.empty((n, wl.L * wl.k), dtype=torch.int32, device="cuda")
        keys = torch.empty((n, wl.L), dtype=torch.int64, device="cuda")
        ctx.hash(wl.scale, ft, n, codes, keys)
        ctx.sync()
        ref = lsh.codes(feat, c.pre.alpha, c.pre.beta, wl.w)
        assert np.array_equal(_np(codes), ref)
        assert np.array_equal(_np(keys).view(np.uint64), lsh.bucket_keys(ref, wl.L, wl.k))
    ctx.set_query_opts(cap=c.cap, proj=1)


@pytest.mark.parametrize("fix_cap", ["0", "3"])
def test_codes_and_keys_when_fix_list_overflows(gpu, fix_cap, monkeypatch):
    """Tables whose uncertain codes do not fit the fix list (capacity forced
    to 0 or 3 entries) take the per-row recomputation path: same codes and
    keys."""
    torch = _torch()
    c = case(MID)
    wl = c.wl
    ctx = c.g.ctx
    monkeypatch.setenv("ZH_HASH_FIX_CAP", fix_cap)
    feat = c.pre.dictionary.feat[:50_000]
    n = feat.shape[0]
    ft = torch.from_numpy(feat).cuda()
    codes = torch.empty((n, wl.L * wl.k), dtype=torch.int32, device="cuda")
    keys = torch.empty((n, wl.L), dtype=torch.int64, device="cuda")
    ctx.hash(wl.scale, ft, n, codes, keys)
    ctx.sync()
    monkeypatch.delenv("ZH_HASH_FIX_CAP")
    ref = lsh.codes(feat, c.pre.alpha, c.pre.beta, wl.w)
    assert ctx.stats()["codes_fixed"] > 3
    assert np.array_equal(_np(codes), ref)
    assert np.array_equal(_np(keys).view(np.uint64), lsh.bucket_keys(ref, wl.L, wl.k))


@pytest.mark.parametrize("L,k,proj", [(7, 24, 1), (5, 28, 1), (3, 1, 1), (9, 13, 1), (7, 24, 0)])
def test_codes_and_keys_other_table_shapes(gpu, L, k, proj):
    """Tables of other shapes on the mid dictionary (D = 100): an odd table
    count (the last staged pair holds one table), k above 24 (one 16-row
    feature tile per wave instead of two), k = 1, and 1077 rows (a ragged
    last workgroup and a wave with one live tile). Codes and keys bitwise
    against the oracle's parameters; the original tables are restored."""
    torch = _torch()
    c = case(MID)
    wl, g = c.wl, c.g
    ctx = g.ctx
    alpha, beta = lsh.hash_params(wl.hash_seed, L, k, wl.D, wl.w)
    feat = c.pre.dictionary.feat[:1077]
    n = feat.shape[0]
    try:
        ctx.build_tables(g.feat, g.resid, g.n, g.D, wl.scale, wl.feat_mode, L, k, wl.w, wl.hash_seed)
        ctx.set_query_opts(cap=c.cap, proj=proj)
        a, b = ctx.get_hash_params(wl.scale, L, k, wl.D)
        assert np.array_equal(a, alpha) and np.array_equal(b, beta)
        ft = torch.from_numpy(feat).cuda()
        codes = torch.empty((n, L * k), dtype=torch.int32, device="cuda")
        keys = torch.empty((n, L), dtype=torch.int64, device="cuda")
        ctx.hash(wl.scale, ft, n, codes, keys)
        ctx.sync()
        ref = lsh.codes(feat, alpha, beta, wl.w)
        assert np.array_equal(_np(codes), ref)
        assert np.array_equal(_np(keys).view(np.uint64), lsh.bucket_keys(ref, L, k))
    finally:
        ctx.set_query_opts(cap=c.cap, proj=1)
        ctx.build_tables(g.feat, g.resid, g.n, g.D, wl.scale, wl.feat_mode, wl.L, wl.k, wl.w, wl.hash_seed)


def test_codes_boundary_cases_are_fixed(gpu):
    """Rows built so that alpha.v + beta sits within a few ulps of a bin
    edge: the fp32 and split-bf16 projections alone would misplace some of
    them; the certified decision must return the FP64 code for all."""
    torch = _torch()
    c = case(TINY)
    wl = c.wl
    rng = np.random.default_rng(9)
    A, beta = c.pre.alpha, c.pre.beta
    rows = []
    for t in range(400):
        j = int(rng.integers(0, A.shape[0]))
        v = rng.standard_normal(wl.D)
        s = float(A[j].astype(np.float64) @ v)
        target = (math.floor((s + beta[j]) / wl.w) + 1) * wl.w - beta[j]
        v = v * (target / s) if s != 0 else v
        rows.append(v.astype(np.float32))
    feat = np.stack(rows)
    ref = lsh.codes(feat, A, beta, wl.w)
    ctx = c.g.ctx
    for proj in (0, 1):
        ctx.set_query_opts(proj=proj)
        ft = torch.from_numpy(feat).cuda()
        codes = torch.empty((len(rows), wl.L * wl.k), dtype=torch.int32, device="cuda")
        ctx.hash(wl.scale, ft, len(rows), codes, None)
        ctx.sync()
        st = ctx.stats()
        assert np.array_equal(_np(codes), ref)
        assert st["codes_fixed"] > 0
    ctx.set_query_opts(proj=1)


def _gpu_candidates(c, cap_per_query):
    torch = _torch()
    g = c.g
    g.set_mode(cap=c.cap)
    g.ctx.query(g.lr, g.h, g.w, c.wl.scale, c.wl.K)
    counts = torch.zeros(g.Q, dtype=torch.int32, device="cuda")
    ids = torch.full((g.Q, cap_per_query), -1, dtype=torch.int32, device="cuda")
    g.ctx.candidates(cap_per_query, counts, ids)
    g.ctx.sync()
    return _np(counts), _np(ids)


@pytest.mark.parametrize("name,cap", [(TINY, 0), (TINY, 12), (TINY_RAGGED, 0), (TINY3, 12), (TINY1, 12), (TINY4, 12), (MID, 0), (MID, 40),
                                      (FLAT, 40)])
def test_candidate_sets_bit_exact(gpu, name, cap):
    c = case(name, cap=cap)
    maxc = max(len(x) for x in c.qr.cand)
    counts, ids = _gpu_candidates(c, max(1, maxc))
    for q in range(c.g.Q):
        ref = c.qr.cand[q]
        assert counts[q] == len(ref), q
        assert np.array_equal(ids[q, :len(ref)], ref), q


@pytest.mark.parametrize("name,cap", [(TINY, 0), (TINY, 12), (TINY_RAGGED, 0), (TINY3, 12), (TINY1, 12), (TINY4, 12), (MID, 0), (MID, 40),
                                      (FLAT, 40)])
def test_neighbours_weights_pixels(gpu, name, cap):
    torch = _torch()
    c = case(name, cap=cap)
    g, wl = c.g, c.wl
    g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
    hr = g.zoom()
    r = g.results()
    assert np.array_equal(r["m"], c.qr.m)
    assert np.array_equal(r["ids"], np.where(c.qr.ids >= 0, c.qr.ids, -1).astype(np.int32))
    ok = c.qr.m > 0
    d_ref = np.nan_to_num(c.qr.d2)
    assert np.allclose(r["d2"][ok], d_ref[ok].astype(np.float32), rtol=2e-6, atol=1e-30)
    dw = np.abs(r["w"].astype(np.float64) - c.qr.weights)
    assert (dw <= W_REL * np.abs(c.qr.weights) + W_ABS).all(), dw.max()
    out = _np(hr).astype(np.float64)
    assert np.abs(out - c.hr).max() < PIX_TOL
    hb = g.backproject(hr.clone())
    assert np.abs(_np(hb).astype(np.float64) - c.hr_bp).max() < PIX_TOL


@pytest.mark.parametrize("name,cap", [(TINY, 12), (TINY3, 12), (TINY1, 12), (TINY4, 12), (MID, 40), (FLAT, 40)])
def test_screened_form_neighbour_sets_and_pixels(gpu, name, cap):
    """Screened form (int8 screen, at most R = 32 exact fp32 rows, fp32 LLE
    with the FP64 redo): at most R survivors, the neighbour count of the
    oracle, and a neighbour set that is a K-nearest set of the FP64
    definition; where it differs from the oracle's, only by candidates tied
    with the K-th distance within fp32 rounding (2 gamma_{D+3}). Pixels
    within 1e-5."""
    R = 32
    c = case(name, cap=cap)
    g, wl = c.g, c.wl
    g.set_mode(cap=cap, rerank=R, proj=1, lle_fp64=0)
    hr = g.zoom()
    r = g.results()
    assert (r["nsurv"] <= R).all()
    assert np.array_equal(r["m"], c.qr.m)
    feat = c.pre.dictionary.feat.astype(np.float64)
    tie = 2.0 * (wl.D + 3) * 2.0 ** -24 * 1.01
    s, ps = wl.scale, 5 * wl.scale
    H, W = c.hr.shape
    covered = np.zeros((H, W), dtype=bool)   # HR pixels under a patch whose set differs
    nj = c.lr.shape[1] - 4
    for q in np.nonzero(c.qr.m > 0)[0]:
        mq = c.qr.m[q]
        mine, ref = np.sort(r["ids"][q, :mq]), np.sort(c.qr.ids[q, :mq])
        if np.array_equal(mine, ref):
            continue
        x = c.qr.feat[q].astype(np.float64)
        dk = np.nanmax(c.qr.d2[q, :mq])
        d_mine = ((feat[mine] - x) ** 2).sum(axis=1)
        assert (d_mine <= dk * (1.0 + tie) + 1e-30).all(), q
        i, j = divmod(int(q), nj)
        covered[s * i:s * i + ps, s * j:s * j + ps] = True
    g.set_mode(cap=cap)
    err = np.abs(_np(hr).astype(np.float64) - c.hr)
    assert err[~covered].max() < PIX_TOL


@pytest.mark.parametrize("rerank", [0, 32])
def test_early_stop_with_k_above_eight(gpu, rerank):
    """K = 12 with the early stop (the search's exact passes without the
    fused Gram, the LLE forming it): exact form bit-exact neighbours, the
    screened form a K-nearest set of the FP64 definition; pixels within 1e-5."""
    K, cap = 12, 40
    c = case(MID, cap=cap)
    g, wl = c.g, c.wl
    qr = pipeline.query(c.pre, c.lr, K, wl.lam, cap=cap)
    hr_ref, _ = pipeline.reconstruct(qr, c.lr, wl.scale)
    g.set_mode(cap=cap, rerank=rerank, proj=1, lle_fp64=1)
    hr = g.zoom(K=K)
    r = g.results(K=K)
    assert np.array_equal(r["m"], qr.m)
    if rerank == 0:
        assert np.array_equal(r["ids"], np.where(qr.ids >= 0, qr.ids, -1).astype(np.int32))
        assert np.abs(_np(hr).astype(np.float64) - hr_ref).max() < PIX_TOL
    else:
        assert (r["nsurv"] <= rerank).all()
        feat = c.pre.dictionary.feat.astype(np.float64)
        tie = 2.0 * (wl.D + 3) * 2.0 ** -24 * 1.01
        for q in np.nonzero(qr.m > 0)[0]:
            mq = qr.m[q]
            mine = np.sort(r["ids"][q, :mq])
            if np.array_equal(mine, np.sort(qr.ids[q, :mq])):
                continue
            d_mine = ((feat[mine] - qr.feat[q].astype(np.float64)) ** 2).sum(axis=1)
            assert (d_mine <= np.nanmax(qr.d2[q, :mq]) * (1.0 + tie) + 1e-30).all(), q
    g.set_mode(cap=cap)


def test_single_patch_image_and_k_edges(gpu):
    """Q = 1 (a 5x5 LR image), K = 1 and K = 16."""
    torch = _torch()
    c = case(TINY)
    g, wl = c.g, c.wl
    g.set_mode(cap=0)
    lr = c.lr[10:15, 20:25].copy()
    for K in (1, 16):
        qr = pipeline.query(c.pre, lr, K, wl.lam)
        out = torch.empty((10, 10), dtype=torch.float32, device="cuda")
        lt = torch.from_numpy(lr).cuda()
        g.ctx.query(lt, 5, 5, wl.scale, K)
        g.ctx.lle_weights(wl.lam)
        g.ctx.reconstruct(out)
        ids = torch.empty((1, K), dtype=torch.int32, device="cuda")
        m = torch.empty(1, dtype=torch.int32, device="cuda")
        g.ctx.get_results(ids, None, m, None, None)
        g.ctx.sync()
        assert _np(m)[0] == qr.m[0]
        assert np.array_equal(_np(ids)[0, :qr.m[0]], qr.ids[0, :qr.m[0]])
        hr_o, _ = pipeline.reconstruct(qr, lr, wl.scale)
        assert np.abs(_np(out) - hr_o).max() < PIX_TOL


def test_full_image_self_reproduction_on_gpu(gpu):
    """Dictionary of every pair of one image: K = 1 reconstructs the HR image."""
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    hr = synthdata.fractal_voronoi_image(40, 48, 48)
    ht = torch.from_numpy(hr).cuda()
    pos = np.concatenate([np.zeros((400, 1), np.int64), imaging.all_positions(24, 24)], axis=1)
    pt = torch.from_numpy(pos.astype(np.int32)).cuda()
    feat = torch.empty((400, 100), dtype=torch.float32, device="cuda")
    resid = torch.empty((400, 100), dtype=torch.float32, device="cuda")
    ctx = zb.Context(0)
    ctx.make_dictionary(ht, 1, 48, 48, pt, 400, 2, 1.0, 1, feat, resid)
    ctx.build_tables(feat, resid, 400, 100, 2, 1, 4, 6, 4.0, 7)
    lr = torch.empty((24, 24), dtype=torch.float32, device="cuda")
    ctx.degrade(ht, 1, 48, 48, 2, 1.0, lr)
    out = torch.empty((48, 48), dtype=torch.float32, device="cuda")
    ctx.query(lr, 24, 24, 2, 1)
    ctx.lle_weights(1e-3)
    ctx.reconstruct(out)
    ctx.sync()
    assert np.abs(_np(out) - hr).max() < 1e-6
    ctx.close()


def test_argument_and_state_errors(gpu):
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    ctx = zb.Context(0)
    lr = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(zb.ZHError) as e:
        ctx.query(lr, 8, 8, 2, 5)          # no tables
    assert e.value.status == zb.ZH_ESTATE
    with pytest.raises(zb.ZHError) as e:
        ctx.lle_weights(1e-3)              # before a query
    assert e.value.status == zb.ZH_ESTATE
    with pytest.raises(zb.ZHError) as e:
        ctx.set_query_opts(cap=1000)
    assert e.value.status == zb.ZH_EINVAL
    feat = torch.zeros((10, 25), dtype=torch.float32, device="cuda")
    resid = torch.zeros((10, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(zb.ZHError) as e:
        ctx.build_tables(feat, resid, 10, 25, 2, 0, 0, 4, 4.0, 1)   # L = 0
    assert e.value.status == zb.ZH_EINVAL
    with pytest.raises(zb.ZHError) as e:
        ctx.build_tables(feat, resid, 10, 25, 2, 0, 4, 4, -1.0, 1)  # w <= 0
    assert e.value.status == zb.ZH_EINVAL
    ctx.build_tables(feat, resid, 10, 25, 2, 0, 2, 3, 4.0, 1)
    with pytest.raises(zb.ZHError) as e:
        ctx.query(lr, 8, 8, 2, 17)         # K > 16
    assert e.value.status == zb.ZH_EINVAL
    with pytest.raises(zb.ZHError) as e:
        ctx.query(lr, 4, 8, 2, 5)          # image smaller than a patch
    assert e.value.status == zb.ZH_EINVAL
    ctx.close()
