"""Parity at the parameters of the 1024^2 workload, and on variants of the
64^2 and 256^2 workloads whose bins are wide enough for most patches to find
candidates.

Headline parameters: 4-gradient features (D = 100), L = 24 tables of k = 20
hashes (three bf16 MFMA tiles per pair of tables in the projection),
w = 32, K = 8 (the search's fused 8 x 8 Gram matrices with every row live),
early stop at 3L = 72, against a 200,000-pair dictionary cut from the
workload's training images, on the top-left 136 x 144 crop of its 1024^2 LR
image (97% of the crop's patches find candidates, 55% reach the early stop,
84% have 8 neighbours). Exact form: codes, keys, candidate sets, neighbour
IDs and counts bitwise; distances relative 2e-6; weights
|dw| <= 2^-23 |w| + 1e-10; pixels and back-projected pixels within 1e-5.
Screened form (int8 screen, at most R = 32 exact rows, fp32 LLE with the
FP64 redo): no patch over R (truncated = 0), K-nearest sets of the FP64
definition, pixels within 1e-5 away from patches whose set differs within
fp32 ties.

Variants: the 64^2 workload with w = 16 (97% of its patches find
candidates; 31% at w = 4) and the 256^2 workload with w = 80 and the early
stop at 3L = 48 (96%; 1% at w = 4).
"""
import numpy as np
import pytest

import synthdata
from oracle import backproject as obp
from oracle import imaging, pipeline

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-5
W_REL = 2.0 ** -23
W_ABS = 1e-10

HEAD = ("precision", (("n_dict", 200_000), ("dict_images", 16)))
HEAD_CROP = (136, 144)      # top-left LR crop of the workload's 1024^2 LR image
TINY_W16 = ("tiny", (("w", 16.0),))
MID_W80 = ("mid", (("w", 80.0), ("test_h", 96), ("test_w", 88), ("n_dict", 100_000), ("dict_images", 32)))
_cases = {}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


class Case:
    def __init__(self, spec, cap):
        from paper_1004_3980_amd.pipeline import GpuWorkload
        name, kw = spec
        wl = synthdata.scaled(synthdata.WORKLOADS[name], cap=cap, **dict(kw))
        self.wl = wl
        self.g = GpuWorkload(wl)
        self.g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
        if spec is HEAD:
            ch, cw = HEAD_CROP
            g = self.g
            g.lr = g.lr[:ch, :cw].contiguous()
            g.h, g.w = ch, cw
            g.Q = (ch - 4) * (cw - 4)
            g.hr_out = g.torch.empty((wl.scale * ch, wl.scale * cw), dtype=g.torch.float32, device=g.dev)
        self.pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k,
                                    wl.w, wl.hash_seed)
        self.lr = self.g.lr.cpu().numpy()
        if not wl.test_lr_direct:
            full = imaging.degrade(wl.test_image(), wl.scale)
            assert np.array_equal(self.lr, full[:self.lr.shape[0], :self.lr.shape[1]])
        self.qr = pipeline.query(self.pre, self.lr, wl.K, wl.lam, cap=cap)
        self.hr, _ = pipeline.reconstruct(self.qr, self.lr, wl.scale)
        self.hr_bp = obp.backproject(self.hr, self.lr, wl.scale, wl.bp_iters, wl.blur_sigma, wl.sigma_s,
                                     wl.sigma_r)
        self.cap = cap


def case(spec, cap):
    key = (spec, cap)
    if key not in _cases:
        _torch()
        _cases[key] = Case(spec, cap)
    return _cases[key]


CASES = [(HEAD, 72), (TINY_W16, 0), (TINY_W16, 24), (MID_W80, 48)]


@pytest.mark.parametrize("spec,cap", CASES)
def test_workload_is_not_degenerate(spec, cap):
    c = case(spec, cap)
    m = c.qr.m
    assert (m > 0).mean() >= 0.9, (m > 0).mean()
    if spec is HEAD:
        # the early stop and every row of the fused 8 x 8 Gram matrices are exercised
        ncand = np.array([len(x) for x in c.qr.cand])
        assert (ncand == 72).mean() > 0.3 and (m == 8).mean() > 0.8


@pytest.mark.parametrize("spec,cap", CASES)
def test_codes_keys_candidates(spec, cap):
    torch = _torch()
    c = case(spec, cap)
    wl, g = c.wl, c.g
    Q = len(c.qr.pos)
    feat = torch.from_numpy(c.qr.feat).cuda()
    codes = torch.empty((Q, wl.L * wl.k), dtype=torch.int32, device="cuda")
    keys = torch.empty((Q, wl.L), dtype=torch.int64, device="cuda")
    g.ctx.hash(wl.scale, feat, Q, codes, keys)
    assert np.array_equal(codes.cpu().numpy(), c.qr.codes)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), c.qr.keys)
    g.ctx.query(g.lr, g.lr.shape[0], g.lr.shape[1], wl.scale, wl.K)
    maxc = max(1, max(len(x) for x in c.qr.cand))
    counts = torch.empty(Q, dtype=torch.int32, device="cuda")
    ids = torch.full((Q, maxc), -1, dtype=torch.int32, device="cuda")
    g.ctx.candidates(maxc, counts, ids)
    cn, ci = counts.cpu().numpy(), ids.cpu().numpy()
    for q in range(Q):
        ref = c.qr.cand[q]
        assert cn[q] == len(ref), q
        assert np.array_equal(ci[q, :len(ref)], ref), q


@pytest.mark.parametrize("spec,cap", CASES)
def test_exact_form(spec, cap):
    c = case(spec, cap)
    g = c.g
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
    assert np.abs(hr.cpu().numpy().astype(np.float64) - c.hr).max() < PIX_TOL
    hb = g.backproject(hr.clone())
    assert np.abs(hb.cpu().numpy().astype(np.float64) - c.hr_bp).max() < PIX_TOL
    st = g.ctx.stats()
    assert st["truncated"] == 0


@pytest.mark.parametrize("spec,cap", [(HEAD, 72), (TINY_W16, 24), (MID_W80, 48)])
def test_screened_form(spec, cap):
    R = 32
    c = case(spec, cap)
    g, wl = c.g, c.wl
    g.set_mode(cap=cap, rerank=R, proj=1, lle_fp64=0)
    hr = g.zoom()
    r = g.results()
    assert g.ctx.stats()["truncated"] == 0
    assert (r["nsurv"] <= R).all()
    assert np.array_equal(r["m"], c.qr.m)
    feat = c.pre.dictionary.feat.astype(np.float64)
    tie = 2.0 * (wl.D + 3) * 2.0 ** -24 * 1.01
    s, ps = wl.scale, 5 * wl.scale
    covered = np.zeros(c.hr.shape, dtype=bool)
    nj = c.lr.shape[1] - 4
    for q in np.nonzero(c.qr.m > 0)[0]:
        mq = c.qr.m[q]
        mine, ref = np.sort(r["ids"][q, :mq]), np.sort(c.qr.ids[q, :mq])
        if np.array_equal(mine, ref):
            continue
        dk = np.nanmax(c.qr.d2[q, :mq])
        d_mine = ((feat[mine] - c.qr.feat[q].astype(np.float64)) ** 2).sum(axis=1)
        assert (d_mine <= dk * (1.0 + tie) + 1e-30).all(), q
        i, j = divmod(int(q), nj)
        covered[s * i:s * i + ps, s * j:s * j + ps] = True
    err = np.abs(hr.cpu().numpy().astype(np.float64) - c.hr)
    assert err[~covered].max() < PIX_TOL
    g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)


def test_batch_at_headline_parameters():
    """zh_run_batch with the headline parameters and the screened form
    (R = 32, fp32 LLE): bitwise equal to the images run one by one."""
    torch = _torch()
    c = case(HEAD, 72)
    g, wl = c.g, c.wl
    ctx = g.ctx
    ctx.set_query_opts(cap=72, rerank=32, proj=1, lle_fp64=0)
    sizes = [(40, 52), (23, 17), (5, 5), (61, 30)]
    lrs = [torch.from_numpy(synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 7300 + i, h, w)).cuda()
           for i, (h, w) in enumerate(sizes)]
    ref = []
    for lr, (h, w) in zip(lrs, sizes):
        out = torch.empty((2 * h, 2 * w), device="cuda")
        ctx.query(lr, h, w, 2, wl.K)
        ctx.lle_weights(wl.lam)
        ctx.reconstruct(out)
        ctx.backproject(out, wl.bp_iters, wl.sigma_s, wl.sigma_r)
        ref.append(out)
    outs = [torch.full((2 * h, 2 * w), -1.0, device="cuda") for h, w in sizes]
    for _ in range(2):
        ctx.run_batch(lrs, outs, [2] * len(sizes), wl.K, wl.lam, wl.bp_iters, wl.sigma_s, wl.sigma_r)
        ctx.sync()
        for a, b, sz in zip(ref, outs, sizes):
            assert torch.equal(a, b), sz
    g.set_mode(cap=72, rerank=0, proj=1, lle_fp64=1)
