"""Batched form (zh_run_batch): many LR images of uneven size at x2, x3 and x4
in one captured launch chain. Bar: bit-exact against the same images run one
by one through zh_query, zh_lle_weights, zh_reconstruct and
zh_backproject (odd and even iteration counts, a one-patch image, graph
replays, after autotuning, whose tile height both forms then use), and an
x3 and an x4 image within 1e-5 of the FP64 oracle.
"""
import numpy as np
import pytest

import synthdata
from oracle import pipeline

pytestmark = pytest.mark.gpu

SIZES = [(20, 24, 2), (31, 17, 2), (9, 40, 2), (5, 5, 2), (25, 25, 3), (14, 30, 3), (12, 12, 3), (5, 9, 3),
         (18, 21, 4), (5, 7, 4)]
WL2 = dict(dict_images=6, dict_hr=96, n_dict=8000, L=8, k=8, w=32.0, K=5, cap=40)
WL3 = dict(dict_images=10, dict_hr=96, n_dict=6000, L=8, k=8, w=32.0, K=5, cap=40, scale=3)
WL4 = dict(dict_images=10, dict_hr=128, n_dict=6000, L=8, k=8, w=32.0, K=5, cap=40, scale=4)
_state = {}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _setup():
    if _state:
        return _state
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    ctx = zb.Context(0)
    wl2 = synthdata.scaled(synthdata.WORKLOADS["mid"], **WL2)
    wl3 = synthdata.scaled(synthdata.WORKLOADS["mid"], **WL3)
    wl4 = synthdata.scaled(synthdata.WORKLOADS["mid"], **WL4)
    g2 = GpuWorkload(wl2, ctx=ctx)
    g3 = GpuWorkload(wl3, ctx=ctx)
    g4 = GpuWorkload(wl4, ctx=ctx)
    ctx.set_query_opts(cap=40, rerank=0, proj=1, lle_fp64=1)
    lrs = [torch.from_numpy(synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 7000 + i, h, w)).cuda()
           for i, (h, w, s) in enumerate(SIZES)]
    _state.update(ctx=ctx, g2=g2, g3=g3, g4=g4, wl2=wl2, wl3=wl3, wl4=wl4, lrs=lrs, torch=torch)
    return _state


def _one_by_one(st, iters, K, lam, ss, sr):
    torch, ctx = st["torch"], st["ctx"]
    outs = []
    for lr, (h, w, s) in zip(st["lrs"], SIZES):
        out = torch.empty((s * h, s * w), dtype=torch.float32, device="cuda")
        ctx.query(lr, h, w, s, K)
        ctx.lle_weights(lam)
        ctx.reconstruct(out)
        ctx.backproject(out, iters, ss, sr)
        outs.append(out)
    ctx.sync()
    return outs


def _batch(st, iters, K, lam, ss, sr, tune=False):
    torch, ctx = st["torch"], st["ctx"]
    outs = [torch.full((s * h, s * w), -1.0, dtype=torch.float32, device="cuda") for h, w, s in SIZES]
    args = (st["lrs"], outs, [s for _, _, s in SIZES], K, lam, iters, ss, sr)
    info = ctx.tune_batch(*args) if tune else None
    for o in outs:
        o.fill_(-1.0)
    ctx.run_batch(*args)
    ctx.sync()
    return outs, info


@pytest.mark.parametrize("iters", [0, 1, 2])
def test_batch_equals_image_by_image(iters):
    st = _setup()
    torch = st["torch"]
    ref = _one_by_one(st, iters, 5, 1e-3, 1.5, 0.1)
    got, _ = _batch(st, iters, 5, 1e-3, 1.5, 0.1)
    for r, g, sz in zip(ref, got, SIZES):
        assert torch.equal(r, g), sz
    # the captured graph replayed
    got2, _ = _batch(st, iters, 5, 1e-3, 1.5, 0.1)
    for r, g in zip(ref, got2):
        assert torch.equal(r, g)


def test_batch_after_autotuning():
    """The tuned tile height of the fused synthesis and blend is the
    context's: images run one by one after the tuning equal the batch."""
    st = _setup()
    torch = st["torch"]
    got, info = _batch(st, 3, 5, 1e-3, 1.5, 0.1, tune=True)
    ref = _one_by_one(st, 3, 5, 1e-3, 1.5, 0.1)
    assert info["bp_tile"] in (16, 32) and info["bp_grid_per_cu"] in (2, 4, 8)
    assert all(t > 0 for t in info["bp_ms"])
    assert info["synth_rows"] in (4, 8) and all(t > 0 for t in info["synth_ms"]) and info["from_cache"] == 0
    for r, g in zip(ref, got):
        assert torch.equal(r, g)


def test_tuning_cache(tmp_path, monkeypatch):
    """With ZH_TUNE_CACHE set, the first tuning of a batch times and appends
    its choice (one JSON object per line, keyed by device, HIP runtime and
    batch); the next tuning of the same batch takes it from the file without
    timing; another batch (other K) is timed again. Outputs stay equal to the
    images run one by one."""
    import json
    st = _setup()
    torch = st["torch"]
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("ZH_TUNE_CACHE", str(path))
    got, info = _batch(st, 2, 5, 1e-3, 1.5, 0.1, tune=True)
    ref = _one_by_one(st, 2, 5, 1e-3, 1.5, 0.1)
    assert info["from_cache"] == 0
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["bp_tile"] == info["bp_tile"] and rec["synth_rows"] == info["synth_rows"]
    assert rec["arch"].startswith("gfx9") and rec["hip_runtime"] > 0
    got2, info2 = _batch(st, 2, 5, 1e-3, 1.5, 0.1, tune=True)
    assert info2["from_cache"] == 1 and info2["bp_ms"] == [0.0] * 6
    assert (info2["bp_tile"], info2["bp_grid_per_cu"], info2["synth_rows"]) == \
        (info["bp_tile"], info["bp_grid_per_cu"], info["synth_rows"])
    assert len(path.read_text().splitlines()) == 1
    for r, a, b in zip(ref, got, got2):
        assert torch.equal(r, a) and torch.equal(r, b)
    _, info3 = _batch(st, 2, 6, 1e-3, 1.5, 0.1, tune=True)
    assert info3["from_cache"] == 0 and len(path.read_text().splitlines()) == 2


@pytest.mark.parametrize("size", [(14, 30, 3), (18, 21, 4)])
def test_batch_image_against_oracle(size):
    st = _setup()
    s = size[2]
    wl = st[f"wl{s}"]
    got, _ = _batch(st, 2, 5, 1e-3, 1.5, 0.1)
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), s, wl.feat_mode, wl.L, wl.k, wl.w,
                           wl.hash_seed)
    i = SIZES.index(size)
    lr = st["lrs"][i].cpu().numpy()
    _, _, hr_bp = pipeline.run(pre, lr, s, 5, 1e-3, 2, 1.5, 0.1, cap=40)
    assert np.abs(got[i].cpu().numpy() - hr_bp).max() <= 1e-5


def test_batch_argument_errors():
    st = _setup()
    torch = st["torch"]
    from paper_1004_3980_amd import zoomhash as zb
    lr = st["lrs"][0]
    out = torch.empty((2 * lr.shape[0], 2 * lr.shape[1]), device="cuda")
    with pytest.raises(zb.ZHError):
        st["ctx"].run_batch([lr], [out], [1], 5, 1e-3, 1, 1.5, 0.1)     # no tables at x1
    with pytest.raises(zb.ZHError):
        st["ctx"].run_batch([lr], [out], [2], 0, 1e-3, 1, 1.5, 0.1)     # K = 0
    with pytest.raises(ValueError):
        st["ctx"].run_batch([lr], [], [2], 5, 1e-3, 1, 1.5, 0.1)


def test_batch_graph_recaptured_after_buffers_or_tables_change():
    """A captured batch graph holds the addresses of the context's buffers and
    the parameters of its tables. A zh_query on a larger image with a larger
    K (the query buffers are reallocated) and a rebuild of the x2 tables with
    other parameters both happen between two zh_run_batch calls of the same
    batch: each later call must capture again and still equal the images run
    one by one."""
    st = _setup()
    torch, ctx = st["torch"], st["ctx"]
    ref = _one_by_one(st, 1, 5, 1e-3, 1.5, 0.1)
    got, _ = _batch(st, 1, 5, 1e-3, 1.5, 0.1)
    for r, g in zip(ref, got):
        assert torch.equal(r, g)
    big = torch.from_numpy(synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 7100, 120, 100)).cuda()
    ctx.query(big, 120, 100, 2, 16)
    ctx.lle_weights(1e-3)
    got2, _ = _batch(st, 1, 5, 1e-3, 1.5, 0.1)
    for r, g, sz in zip(ref, got2, SIZES):
        assert torch.equal(r, g), sz
    # other x2 tables (L = 6, k = 6), then the original ones again
    g2, wl2 = st["g2"], st["wl2"]
    try:
        ctx.build_tables(g2.feat, g2.resid, g2.n, g2.D, 2, wl2.feat_mode, 6, 6, wl2.w, wl2.hash_seed)
        ref3 = _one_by_one(st, 1, 5, 1e-3, 1.5, 0.1)
        got3, _ = _batch(st, 1, 5, 1e-3, 1.5, 0.1)
        for r, g, sz in zip(ref3, got3, SIZES):
            assert torch.equal(r, g), sz
        assert any(not torch.equal(a, b) for a, b, sz in zip(ref, ref3, SIZES) if sz[2] == 2)
    finally:
        ctx.build_tables(g2.feat, g2.resid, g2.n, g2.D, 2, wl2.feat_mode, wl2.L, wl2.k, wl2.w, wl2.hash_seed)
