#!/usr/bin/env python3
"""Throughput of the patch-hashing zoom path on one MI355X.

Metric: LR patches/s of hash + K-NN + LLE + blend (zh_query, zh_lle_weights,
zh_reconstruct) on a 1024x1024 LR image at x2 (1,040,400 patches) against a
2,000,000-pair dictionary (4-gradient features, D = 100), L = 24 tables of
k = 20 hashes, K = 8, with the dictionary, tables and LR image resident in
HBM. The default form ("screened") bounds every candidate's distance from
below with int8 coordinates in the dictionary's leading principal directions
and gives exact fp32 distances to at most 32 of them (those the bounds cannot
rule out; the number of patches where more were left is reported and is 0);
--form exact does the same with no limit and certifies the selection against
FP64.

One JSON line on stdout. Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# --metric: the form of GpuWorkload.zoom that measures it
ZOOM_METRIC = {"l2": "l2", "l1": "l1q", "l1-rerank": "l1"}
MFMA_BF16_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def psnr(x, ref):
    mse = float(np.mean((np.asarray(x, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def search_bytes(ncand, nsurv, wl, gram_bytes):
    """Algorithmic HBM bytes of one launch of the early-stop search kernel
    (each byte the kernel needs, read or written once).

    Per patch: its L bins (offset, count: 8 B each), its feature row (4D B),
    its coded rotated coordinates (two rows of 64 int8 codes and three
    floats: 140 B), the output (K ids, K distances,
    count, candidate count, survivor count) and the packed Gram matrix of the
    neighbours (36 entries of gram_bytes). Per distinct candidate: its ID
    (4 B) and its 64-byte screen row (int8 coordinates in the leading
    principal directions and the bounds). Per row given an exact distance:
    its fp32 feature row (4D B)."""
    M = ncand.astype(np.int64)
    S = nsurv.astype(np.int64)
    D, L, K = wl.D, wl.L, wl.K
    per_q = 8 * L + 4 * D + 140 + 8 * K + 12 + 36 * gram_bytes
    return int(len(M) * per_q + (M * (4 + 64)).sum() + (S * 4 * D).sum())


def l1_rank_bytes(ncand, nsurv, wl, cap):
    """Algorithmic HBM bytes of one launch of the l1 ranking with the screen
    (D = 100). Per patch: its feature row (4D B), the output (K ids, K
    distances, count, survivor count). Per candidate: its ID (4 B), and,
    where there are more than K candidates, its screen row (D codes, three
    floats). Per survivor: its fp32 feature row (4D B)."""
    M = np.minimum(ncand.astype(np.int64), cap)
    S = nsurv.astype(np.int64)
    D, K = wl.D, wl.K
    per_q = 4 * D + 8 * K + 8
    return int(len(M) * per_q + (4 * M).sum() + ((D + 12) * M * (M > K)).sum() + (S * 4 * D).sum())


def traffic_from_profile(form):
    """HBM bytes per search launch from the committed rocprofv3 counter summary,
    if it was taken with the current search kernel source."""
    path = os.path.join(ROOT, "profiles", f"search_{form}_traffic.json")
    src = os.path.join(ROOT, "paper_1004_3980_amd", "csrc", "k_search.hip")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("k_search_sha256") != sha:
        return None
    return float(rec["hbm_bytes_per_launch"])


# MI355X: 256 compute units of 4 SIMDs at 2.4 GHz; a wave64 VALU instruction
# takes 4 cycles of its SIMD.
SIMDS = 1024
CLOCK_HZ = 2.4e9


def issue_from_profile(name, src_name, launch_ms):
    """Issue fractions of a kernel from the committed rocprofv3 counter summary
    profiles/<name>_counters.json (SQ_WAVES, SQ_INSTS_VALU and
    SQ_VALU_MFMA_BUSY_CYCLES per launch), if it was taken with the current
    source: VALU instructions x 4 cycles, and matrix-core busy cycles, over the
    SIMD cycles of this run's launch time."""
    path = os.path.join(ROOT, "profiles", f"{name}_counters.json")
    src = os.path.join(ROOT, "paper_1004_3980_amd", "csrc", src_name)
    if not os.path.exists(path) or launch_ms <= 0:
        return {}
    with open(path) as f:
        rec = json.load(f)
    if rec.get("src_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return {}
    cyc = launch_ms * 1e-3 * CLOCK_HZ * SIMDS
    out = {"valu_issue_frac": round(rec["valu_insts"] * 4.0 / cyc, 4)}
    if rec.get("mfma_busy_cycles"):
        out["mfma_busy_frac"] = round(rec["mfma_busy_cycles"] / cyc, 4)
    return out


# ---- CPU baseline: the FP64 oracle on the host cores -----------------------------
#
# The oracle runs in a child process started before this process touches the
# GPU; it waits on its stdin until the GPU timings are done, so that it does
# not compete with them. For each sample it builds the tables (timed apart,
# the code projection on every core), then times the query, LLE, synthesis
# and blend on one thread, and across all cores with one worker process per
# core over chunks of the patches (forked after the build).

def _oracle_chunk(arg):
    q0, q1 = arg
    st = _ORC
    qr = st["opipe"].query(st["pre"], st["lr"], st["K"], st["lam"], pos=st["pos"][q0:q1], cap=st["cap"])
    return qr.ids, qr.m, qr.patches


_ORC = {}


def _oracle_sample(name, wl, lr, cores, log_fn):
    import multiprocessing as mp
    from oracle import _clib
    from oracle import imaging as oim
    from oracle import lle as olle
    from oracle import pipeline as opipe
    _clib.set_threads(cores)
    t0 = time.perf_counter()
    pre = opipe.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, wl.w,
                        wl.hash_seed)
    t_build = time.perf_counter() - t0
    pos = oim.all_positions(*lr.shape)
    Q = len(pos)
    _clib.set_threads(1)
    t0 = time.perf_counter()
    qr = opipe.query(pre, lr, wl.K, wl.lam, cap=wl.cap)
    hr1, _ = opipe.reconstruct(qr, lr, wl.scale)
    t_one = time.perf_counter() - t0
    _ORC.update(opipe=opipe, pre=pre, lr=lr, pos=pos, K=wl.K, lam=wl.lam, cap=wl.cap)
    nchunk = 4 * cores
    bounds = [(Q * i // nchunk, Q * (i + 1) // nchunk) for i in range(nchunk)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        parts = pool.map(_oracle_chunk, bounds)
    patches = [p for _, _, ps in parts for p in ps]
    m = np.concatenate([pm for _, pm, _ in parts])
    hrn, _ = olle.blend(patches, pos, m > 0, wl.scale, np.asarray(lr, np.float32))
    t_all = time.perf_counter() - t0
    ids = np.concatenate([pi for pi, _, _ in parts])
    assert np.array_equal(ids, qr.ids) and np.array_equal(hrn, hr1)
    rec = {"patches": int(Q), "table_build_s": round(t_build, 2), "one_thread_s": round(t_one, 2),
           "one_thread_patches_per_s": Q / t_one, "all_cores_s": round(t_all, 2),
           "all_cores_patches_per_s": Q / t_all, "dictionary_pairs": wl.n_dict,
           "mean_candidates": float(np.mean([len(c) for c in qr.cand]))}
    log_fn(f"[oracle] {name}: {Q} patches, build {t_build:.1f} s, one thread {Q / t_one:.4g}/s, "
           f"{cores} workers {Q / t_all:.4g}/s")
    return rec, qr, hr1


def oracle_child(args):
    """Child process: wait for "go" on stdin, then time the oracle and print
    one JSON record; the precision crop's oracle result goes to args.oracle_out."""
    import synthdata
    from oracle import imaging as oim
    if not sys.stdin.readline().strip():
        return
    cores = len(os.sched_getaffinity(0))
    out = {"cores": cores, "os_cpu_count": os.cpu_count(), "affinity": cores, "samples": {}}
    for name in ("tiny", "mid"):
        wl = synthdata.WORKLOADS[name]
        lr = wl.test_image() if wl.test_lr_direct else oim.degrade(wl.test_image(), wl.scale)
        out["samples"][name], _, _ = _oracle_sample(name, wl, np.ascontiguousarray(lr), cores, log)
    wl = synthdata.WORKLOADS[args.workload]
    if args.scale not in (0, wl.scale):
        wl = synthdata.at_scale(wl, args.scale)
    img = wl.test_image()
    lr = img if wl.test_lr_direct else oim.degrade(img, wl.scale)
    crop = args.crop
    lr_c = np.ascontiguousarray(lr[:crop, :crop])
    rec, qr, hr_c = _oracle_sample(f"{wl.name} crop", wl, lr_c, cores, log)
    out["samples"][f"{wl.name}_crop{crop}"] = rec
    # Section 4.3's approximation of the cross bilateral filter, on the
    # crop's oracle result: the back-projection with each filter
    from oracle import backproject as obp
    t0 = time.perf_counter()
    hr_a = obp.backproject(hr_c, lr_c, wl.scale, wl.bp_iters, wl.blur_sigma, wl.sigma_s, wl.sigma_r)
    hr_e = obp.backproject_exact(hr_c, lr_c, wl.scale, wl.bp_iters, wl.blur_sigma, wl.sigma_s, wl.sigma_r)
    bil = {"crop": crop, "iters": wl.bp_iters, "sigma_s": wl.sigma_s, "sigma_r": wl.sigma_r,
           "max_abs_approximate_vs_exact": float(np.abs(hr_a - hr_e).max()),
           "psnr_approximate_vs_exact_db": psnr(hr_a, hr_e), "seconds": round(time.perf_counter() - t0, 2)}
    if not wl.test_lr_direct:
        gt = np.asarray(img, np.float64)[: wl.scale * crop, : wl.scale * crop]
        bil["psnr_gt_db"] = {"before": psnr(hr_c, gt), "approximate": psnr(hr_a, gt), "exact": psnr(hr_e, gt)}
    out["bilateral_approximation"] = bil
    log(f"[oracle] cross bilateral approximation on the crop: {json.dumps(bil)}")
    np.savez(args.oracle_out, ids=qr.ids, m=qr.m, hr=hr_c)
    print(json.dumps(out), flush=True)


def start_oracle_child(args):
    """Start the oracle's timing process (before any GPU work); returns
    (process, path of its result file)."""
    import subprocess
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".npz")
    os.close(fd)
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", "--oracle-out", path,
           "--workload", args.workload, "--scale", str(args.scale), "--crop", str(args.crop)]
    env = dict(os.environ, OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    p = subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
    return p, path


def finish_oracle_child(proc, path, wl, crop):
    """Release the child, read its record; the cpu_baseline object, the
    oracle's neighbour IDs and counts and HR crop."""
    out, _ = proc.communicate("go\n", timeout=900)
    if proc.returncode != 0:
        raise RuntimeError(f"oracle timing process failed ({proc.returncode})")
    rec = json.loads(out.strip().splitlines()[-1])
    z = np.load(path)
    os.unlink(path)
    key = f"{wl.name}_crop{crop}"
    s = rec["samples"][key]
    cpu = {"value": s["all_cores_patches_per_s"], "unit": "LR patches/s", "cores": rec["cores"], "kind": "oracle",
           "sample": f"{crop}x{crop} LR crop ({s['patches']} patches) of the same image against the full "
                     f"{wl.n_dict}-pair dictionary: features, codes, candidates (early stop {wl.cap}), exact "
                     f"K-NN, FP64 LLE, synthesis, blend, on {rec['cores']} worker processes over chunks of the "
                     f"patches ({s['all_cores_s']} s); table build ({s['table_build_s']} s, the projection on "
                     f"{rec['cores']} threads) excluded",
           "one_thread_value": s["one_thread_patches_per_s"],
           "os_cpu_count": rec["os_cpu_count"], "affinity": rec["affinity"],
           "samples": rec["samples"]}
    cpu["bilateral_approximation"] = rec.get("bilateral_approximation")
    return cpu, z["ids"], z["m"], z["hr"]


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="precision")
    ap.add_argument("--form", choices=["screened", "exact", "batched", "diff", "tools", "tofl"], default="screened",
                    help="screened/exact: the 1024^2 workload (the headline line); batched: 64 images "
                         "at x2/x3 in one captured graph against per-image launches; diff: forward and "
                         "backward of the differentiation workload")
    ap.add_argument("--metric", choices=["l2", "l1", "l1-rerank"], default="l2",
                    help="screened/exact: neighbours by squared l2 (the path), by l1 (the query ranks under "
                         "l1) or re-ranked under l1 after the l2 query (zh_knn_l1)")
    ap.add_argument("--scale", type=int, default=0,
                    help="screened/exact: run the workload at this zoom factor (1..4) instead of its own")
    ap.add_argument("--crop", type=int, default=256, help="LR crop side for quality and the CPU leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="leave the batched form out of the default line")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times "
                         "(reference dispatch for scaling HBM counters)")
    ap.add_argument("--oracle-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--oracle-out", default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_child:
        return oracle_child(args)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this path is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    # the oracle's process starts before this one touches the GPU
    child = None
    if args.form in ("screened", "exact") and not (args.no_quality and args.no_cpu_baseline):
        child = start_oracle_child(args)

    import torch
    import synthdata
    from paper_1004_3980_amd.pipeline import GpuWorkload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.form == "batched":
        return bench_batched(args)
    if args.form == "diff":
        return bench_diff(args)
    if args.form == "tools":
        return bench_tools(args)
    if args.form == "tofl":
        return bench_tofl(args)
    wl = synthdata.WORKLOADS[args.workload]
    own_scale = args.scale in (0, wl.scale)
    if not own_scale:
        wl = synthdata.at_scale(wl, args.scale)
    log(f"[bench] building {wl.name}: {wl.n_dict} pairs, LR {wl.test_h}x{wl.test_w} x{wl.scale}")
    t0 = time.perf_counter()
    g = GpuWorkload(wl, device=0)
    torch.cuda.synchronize()
    log(f"[bench] inputs + dictionary + tables ready in {time.perf_counter() - t0:.1f} s")

    def set_form(form):
        if form == "screened":
            g.set_mode(cap=wl.cap, rerank=wl.rerank, proj=1, lle_fp64=0)
        else:
            g.set_mode(cap=wl.cap, rerank=0, proj=1, lle_fp64=1)

    def timed(form, steps, warmup, stages=None):
        set_form(form)
        for _ in range(warmup):
            g.zoom(metric=ZOOM_METRIC[args.metric])
        torch.cuda.synchronize()
        g.ctx.get_timing()
        g.ctx.set_timing(True, stages)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.zoom(metric=ZOOM_METRIC[args.metric])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.ctx.set_timing(False)
        st = g.ctx.get_timing()
        return dt, st

    # the timed steps bracket only the search kernel with HIP events (each
    # pair of events leaves a short gap on the stream); the other stages are
    # timed in a pass of their own
    dt, stages = timed(args.form, args.steps, args.warmup, stages=["search"])
    Q = g.Q
    value = Q * args.steps / dt
    res = g.results()
    search_ms = stages["search"][0] / max(1, stages["search"][1])
    _, stages_all = timed(args.form, max(2, args.steps // 2), 0)
    ms_stage = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages_all.items()}
    ms_stage["search"] = search_ms
    log(f"[bench] {args.form}: {value:.4g} patches/s, {1e3 * dt / args.steps:.3f} ms/step; "
        f"stages ms {json.dumps({k: round(v, 4) for k, v in ms_stage.items()})}")

    # dominant kernel: the candidate search
    dom = max(("hash", "probe", "search", "lle", "synth", "blend"), key=lambda k: ms_stage[k])
    if args.metric != "l2":
        # the l1 ranking: its algorithmic bytes, and the survivors of its screen
        M = np.minimum(res["ncand"], wl.cap)
        extra_l1 = {"mean_candidates": float(M.mean()), "mean_survivors": float(res["nsurv"].mean()),
                    "rank_bytes": l1_rank_bytes(res["ncand"], res["nsurv"], wl, wl.cap)}
        log(f"[bench] l1 ranking: {json.dumps(extra_l1)}")
    sb = search_bytes(res["ncand"], res["nsurv"], wl, 4 if args.form == "screened" else 8)
    ach = sb / (ms_stage["search"] * 1e-3) / 1e9
    traffic = traffic_from_profile(args.form) if own_scale and args.metric == "l2" else None
    roof = {"bound": "hbm", "kernel": "k_search", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": traffic, "algorithmic_bytes": sb, "launch_ms": round(ms_stage["search"], 4),
            "dominant_stage": dom}
    if own_scale and args.metric == "l2" and args.form == "screened":
        roof.update(issue_from_profile("search_screened", "k_search.hip", ms_stage["search"]))
    if args.metric != "l2":
        # the search stage holds the union and the l1 ranking together: no one
        # kernel's duration to divide by (the l2 line carries the roofline)
        roof = None
    # the projection of the hash (Eq. hash_fn) against the bf16 matrix-core peak:
    # useful flops 2 Q D L k over the hash stage (projection, codes, keys, FP64 fixes)
    hflop = 2.0 * Q * wl.D * wl.L * wl.k
    hach = hflop / (ms_stage["hash"] * 1e-3) / 1e12 if ms_stage["hash"] > 0 else 0.0
    hash_roof = {"bound": "mfma", "kernel": "k_hash", "achieved": round(hach, 2), "peak": MFMA_BF16_PEAK_TFLOPS,
                 "unit": "TFLOP/s", "frac": round(hach / MFMA_BF16_PEAK_TFLOPS, 4), "flops": hflop,
                 "launch_ms": round(ms_stage["hash"], 4)}
    if own_scale:
        hash_roof.update(issue_from_profile("hash", "k_hash.hip", ms_stage["hash"]))

    # other form on the same image, back-projection, whole path with back-projection
    other = "exact" if args.form == "screened" else "screened"
    dt2, st2 = timed(other, max(2, args.steps // 2), 1)
    other_rec = {"form": other, "value": Q * max(2, args.steps // 2) / dt2,
                 "ms_per_step": 1e3 * dt2 / max(2, args.steps // 2)}
    set_form(args.form)
    g.zoom()
    hr = g.hr_out.clone()
    torch.cuda.synchronize()
    g.ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.backproject(hr.clone())
    torch.cuda.synchronize()
    bp_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    g.ctx.set_timing(False)
    bst = g.ctx.get_timing()
    stats = g.ctx.stats()
    # the batched form (its own context, dictionaries and images), before the
    # oracle's process is released
    batched = None
    if args.form == "screened" and args.metric == "l2" and own_scale and not args.no_batched:
        log("[bench] batched form")
        b = run_batched(args)
        batched = {"value": b["value"], "unit": b["unit"], "ms_per_step": b["ms_per_step"], "steps": b["steps"],
                   "workload": b["config"]["workload"], "patches_per_step": b["config"]["patches_per_step"],
                   "per_image_launches": b["extra"]["per_image_launches"],
                   "speedup_vs_per_image": b["extra"]["speedup_vs_per_image"],
                   "outputs_equal_per_image": b["extra"]["outputs_equal_per_image"],
                   "tuning": b["extra"]["tuning"]}
        if not batched["outputs_equal_per_image"]:
            raise SystemExit("batched outputs differ from the images run one by one")

    extra = {"ms_per_stage": {k: round(v, 4) for k, v in ms_stage.items()},
             **({"l1_ranking": extra_l1} if args.metric != "l2" else {}),
             "hash_roofline": hash_roof,
             "backprojection_ms": round(bp_ms, 3), "bp_iters": wl.bp_iters,
             "value_with_backprojection": Q / (dt / args.steps + bp_ms * 1e-3),
             "other_form": other_rec,
             "mean_candidates": float(res["ncand"].mean()),
             "mean_survivors": float(res["nsurv"].mean()),
             "patches_without_neighbours": int((res["m"] == 0).sum()),
             "truncated_patches": stats["truncated"],
             "batched_form": batched,
             "similarity_checks_saved": float(wl.n_dict / max(1e-9, res["ncand"].mean())),
             "stats": stats}

    # quality on a crop against the FP64 oracle, and the oracle's CPU rates
    cpu = None
    if child is not None:
        crop = args.crop
        gt = g.hr_gt.cpu().numpy()[: wl.scale * crop, : wl.scale * crop] if g.hr_gt is not None else None
        log(f"[bench] oracle timings on the host (tiny, mid, the {crop}x{crop} crop)")
        cpu, ids_o, m_o, hr_o = finish_oracle_child(*child, wl, crop)
        child = None
        lr_c = g.lr[:crop, :crop].contiguous()
        out = torch.empty((wl.scale * crop, wl.scale * crop), dtype=torch.float32, device="cuda")
        quality = {}
        for form in ("screened", "exact"):
            set_form(form)
            g.zoom(lr=lr_c, out=out)
            r = g.results()
            st_q = g.ctx.stats()
            ok = m_o > 0
            inter = [len(np.intersect1d(r["ids"][q, :r["m"][q]], ids_o[q, :m_o[q]])) for q in np.nonzero(ok)[0]]
            rec_k = float(np.sum(inter) / max(1, m_o[ok].sum()))
            o = out.cpu().numpy()
            qrec = {"recall_at_k": rec_k, "ids_equal": bool(np.array_equal(
                r["ids"], np.where(ids_o >= 0, ids_o, -1).astype(np.int32))),
                "max_abs_vs_oracle": float(np.abs(o - hr_o).max()),
                "psnr_vs_oracle_db": psnr(o, hr_o), "truncated": st_q["truncated"]}
            if gt is not None:
                qrec["psnr_gt_db"] = psnr(o, gt)
            quality[form] = qrec
        if gt is not None:
            p_or = psnr(hr_o, gt)
            quality["oracle_psnr_gt_db"] = p_or
            for form in ("screened", "exact"):
                quality[form]["psnr_loss_db"] = p_or - quality[form]["psnr_gt_db"]
        extra["quality_crop"] = quality
        extra["bilateral_approximation"] = cpu.pop("bilateral_approximation", None)
        set_form(args.form)
        if quality["screened"]["truncated"] or quality["exact"]["truncated"]:
            raise SystemExit("screened form cut the exact rows of some patch of the crop (truncated > 0)")
        if args.no_cpu_baseline:
            cpu = None

    out = {
        "metric": f"LR patches/sec (hash+KNN+LLE+blend) at 1024² ×{wl.scale}; recall@K, PSNR vs FP64",
        "value": value,
        "unit": "LR patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16/fp32" if args.form == "screened" else "fp32/fp64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.test_h}x{wl.test_w} LR x{wl.scale}, "
                               f"{wl.n_dict}-pair dictionary (4-gradient features, D={wl.D}), "
                               f"L={wl.L} k={wl.k} w={wl.w:g} K={wl.K}, early stop {wl.cap}, "
                               f"form {args.form}" + (f" (int8 principal-coordinate screen, at most {wl.rerank} "
                                                      "exact fp32 rows)" if args.form == "screened" else "")
                               + {"l2": "", "l1": ", neighbours under l1 (query metric l1)",
                                  "l1-rerank": ", neighbours re-ranked under l1 (zh_knn_l1)"}[args.metric],
                   "patches_per_step": Q, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["extra"]["copy_probe_bytes"] = n * 4
    print(json.dumps(out), flush=True)


def bench_tofl(args):
    """The paper's run-time axis on the 256^2 workload of the differentiation
    form (256^2 LR, L = 16, k = 16, w = 32): the similarity checks per LR
    patch (distinct candidates) against the dictionary size N, with and
    without the early stop at 3L, and the t-of-L criterion (t = 1..4) at
    N = 200k."""
    import torch
    import synthdata
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    base = synthdata.WORKLOADS["diff"]
    ctx = zb.Context(0)
    curve, tofl = [], []
    for N in (25_000, 50_000, 100_000, 200_000):
        wl = synthdata.scaled(base, n_dict=N)
        log(f"[bench] tofl: tables over {N} pairs")
        g = GpuWorkload(wl, ctx=ctx)
        for cap in (0, 3 * wl.L):
            g.set_mode(cap=cap, rerank=0, proj=1, lle_fp64=1)
            for _ in range(args.warmup):
                g.zoom()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                g.zoom()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / args.steps
            if cap > 0:
                nc = g.results()["ncand"].astype(np.float64)
            else:
                # distinct IDs of the union, counted without a size limit
                cnt = torch.empty(g.Q, dtype=torch.int32, device="cuda")
                one = torch.empty((g.Q, 1), dtype=torch.int32, device="cuda")
                g.ctx.candidates_t(1, 1, cnt, one)
                nc = cnt.cpu().numpy().astype(np.float64)
            curve.append({"N": N, "early_stop": cap, "similarity_checks_per_patch": round(float(nc.mean()), 2),
                          "fewer_than_exhaustive": round(N / max(1e-9, float(nc.mean())), 1),
                          "ms_per_step": round(ms, 3), "patches": g.Q})
        if N == 200_000:
            g.set_mode(cap=0, rerank=0, proj=1, lle_fp64=1)
            g.zoom()
            Q = g.Q
            for t in (1, 2, 3, 4):
                cap_q = 4096
                counts = torch.empty(Q, dtype=torch.int32, device="cuda")
                ids = torch.empty((Q, cap_q), dtype=torch.int32, device="cuda")
                g.ctx.candidates_t(t, cap_q, counts, ids)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    g.ctx.candidates_t(t, cap_q, counts, ids)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / args.steps
                c = counts.cpu().numpy().astype(np.float64)
                tofl.append({"t": t, "mean_candidates": round(float(c.mean()), 2),
                             "patches_without_candidates": int((c == 0).sum()), "ms_per_call": round(ms, 3)})
    last = [r for r in curve if r["N"] == 200_000 and r["early_stop"] > 0][0]
    out = {"metric": "similarity checks per LR patch vs dictionary size (256^2 LR, L=16, w=32)",
           "value": last["fewer_than_exhaustive"], "unit": "x fewer checks than exhaustive at N=200k",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": last["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "diff: 256x256 LR x2, N in {25k, 50k, 100k, 200k} pairs, L=16 k=16 w=32 K=5; "
                                  "t-of-L at N=200k", "parallelism": "single GPU"},
           "roofline": None, "cpu_baseline": None, "extra": {"curve": curve, "t_of_L": tofl}}
    print(json.dumps(out), flush=True)


def bench_tools(args):
    """Dictionary-construction tools (off the per-image path): gradient-CDF
    sampling of 25 crops of 100 x 100 from each of 500 training images of
    512^2 (the paper's training-set recipe, synthetic images), and the bucket
    entropy of the 1024^2 workload's 24 tables over 2M pairs."""
    import torch
    import synthdata
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    n_img, side, per, H = 500, 100, 25, 512
    log(f"[bench] tools: {n_img} images of {H}^2, {per} crops of {side}^2 each")
    stack = torch.from_numpy(synthdata.image_stack(synthdata.SEED_BASE + 9000, n_img, H, H)).cuda()
    draws = torch.from_numpy(synthdata.crop_draws(synthdata.SEED_BASE + 9001, n_img, per).view(np.int64)).cuda()
    corners = torch.empty((n_img, per, 2), dtype=torch.int32, device="cuda")
    crops = torch.empty((n_img, per, side, side), dtype=torch.float32, device="cuda")
    ctx = zb.Context(0)

    def crop_call():
        ctx.sample_crops(stack, n_img, H, H, draws, per, side, corners, crops)

    for _ in range(args.warmup):
        crop_call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        crop_call()
    torch.cuda.synchronize()
    crop_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    # algorithmic bytes: the images read once, the crops written
    crop_bytes = n_img * H * H * 4 + n_img * per * side * side * 4
    wl = synthdata.WORKLOADS[args.workload]
    log(f"[bench] building {wl.name} tables for the entropy diagnostic")
    g = GpuWorkload(wl, device=0)
    for _ in range(args.warmup):
        g.ctx.table_entropy(wl.scale, wl.L)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ent = g.ctx.table_entropy(wl.scale, wl.L)
    ent_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    cap = 1 << (2 * wl.n_dict - 1).bit_length()
    ent_bytes = wl.L * cap * 16
    out = {"metric": "training crops/s (gradient-CDF sampling, 100x100 crops from 512^2 images)",
           "value": n_img * per / (crop_ms * 1e-3), "unit": "crops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": crop_ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64/u64", "data": "synthetic",
           "config": {"workload": f"{n_img} training images of {H}x{H}, {per} crops of {side}x{side} each; "
                                  f"bucket entropy of {wl.name} ({wl.L} tables, {wl.n_dict} pairs)",
                      "parallelism": "single GPU"},
           "roofline": {"bound": "hbm", "kernel": "crop sampling (whole call)",
                        "achieved": round(crop_bytes / (crop_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(crop_bytes / (crop_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": None, "algorithmic_bytes": crop_bytes},
           "cpu_baseline": None,
           "extra": {"entropy_ms_per_call": round(ent_ms, 4),
                     "entropy_directory_gbs": round(ent_bytes / (ent_ms * 1e-3) / 1e9, 1),
                     "entropy_bits": [round(float(v), 4) for v in ent],
                     "entropy_bound_bits": float(np.log2(wl.n_dict))}}
    print(json.dumps(out), flush=True)


def bench_batched(args):
    print(json.dumps(run_batched(args)), flush=True)


def run_batched(args):
    """64 LR images (sides 96..1024, aspect 0.5..2; 32 at x2, 32 at x3) against
    1M-pair dictionaries per zoom factor, screened form, 3 back-projection
    iterations: zh_run_batch (one captured graph, autotuned) against the same
    images launched one by one. Returns the bench record."""
    import torch
    import synthdata
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    ctx = zb.Context(0)
    t0 = time.perf_counter()
    dicts = {s: GpuWorkload(synthdata.BATCHED[s], ctx=ctx) for s in (2, 3)}
    wl = synthdata.BATCHED[2]
    ctx.set_query_opts(cap=wl.cap, rerank=wl.rerank, proj=1, lle_fp64=0)
    imgs = synthdata.batched_images()
    lrs = [torch.from_numpy(im).cuda() for im, _ in imgs]
    scales = [s for _, s in imgs]
    outs = [torch.empty((s * l.shape[0], s * l.shape[1]), device="cuda") for l, s in zip(lrs, scales)]
    ref = [torch.empty_like(o) for o in outs]
    torch.cuda.synchronize()
    log(f"[bench] batched: dictionaries and {len(imgs)} images ready in {time.perf_counter() - t0:.1f} s")
    Q = sum((l.shape[0] - 4) * (l.shape[1] - 4) for l in lrs)
    args_b = (lrs, outs, scales, wl.K, wl.lam, wl.bp_iters, wl.sigma_s, wl.sigma_r)

    def per_image(dst):
        for l, o, s in zip(lrs, dst, scales):
            ctx.query(l, l.shape[0], l.shape[1], s, wl.K)
            ctx.lle_weights(wl.lam)
            ctx.reconstruct(o)
            ctx.backproject(o, wl.bp_iters, wl.sigma_s, wl.sigma_r)

    steps, warm = max(1, args.steps // 2), max(1, args.warmup)
    # the tuned tile height of the fused synthesis and blend holds for both forms
    tuning = ctx.tune_batch(*args_b)
    for _ in range(warm):
        per_image(ref)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        per_image(ref)
    torch.cuda.synchronize()
    t_img = (time.perf_counter() - t0) / steps
    for _ in range(warm):
        ctx.run_batch(*args_b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run_batch(*args_b)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a, b) for a, b in zip(outs, ref))
    out = {"metric": "LR patches/s, batched form (64 images x2/x3, 1M-pair dictionaries, "
                     "hash+KNN+LLE+blend+3 BP iterations)",
           "value": Q / t_b, "unit": "LR patches/s", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": 1e3 * t_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16/fp32", "data": "synthetic",
           "config": {"workload": "batched: 64 LR images, sides U{96..1024}, aspect 0.5-2, 32 at x2 and 32 "
                                  "at x3, one 1,000,000-pair dictionary per zoom factor, L=24 k=20 w=32 K=8, "
                                  "early stop 72, screened form (R=32), 3 back-projection iterations",
                      "patches_per_step": Q, "parallelism": "single GPU"},
           "extra": {"per_image_launches": {"value": Q / t_img, "ms_per_step": 1e3 * t_img},
                     "speedup_vs_per_image": t_img / t_b, "outputs_equal_per_image": same,
                     "tuning": tuning}}
    del ctx, dicts, lrs, outs, ref
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def bench_diff(args):
    """Differentiation workload: 8 HR images 512^2 degraded to 256^2 LR (x2),
    200,000-pair fp32 dictionary, K = 5, 3 back-projection iterations;
    forward (query, weights, reconstruction, back-projection) and zh_backward
    of the MSE to the HR ground truth, per image."""
    import torch
    import synthdata
    from paper_1004_3980_amd.pipeline import GpuWorkload
    wl = synthdata.WORKLOADS["diff"]
    g = GpuWorkload(wl)
    g.set_mode(cap=wl.cap, rerank=0, proj=1, lle_fp64=1)
    imgs = []
    for i in range(8):
        gt = torch.from_numpy(synthdata.fractal_voronoi_image(wl.seed_test + i, 2 * wl.test_h,
                                                              2 * wl.test_w)).cuda()
        lr = torch.empty((wl.test_h, wl.test_w), device="cuda")
        g.ctx.degrade(gt, 1, gt.shape[0], gt.shape[1], wl.scale, wl.blur_sigma, lr)
        imgs.append((gt, lr))
    g_resid = torch.empty_like(g.resid)
    g_lam = torch.empty(1, device="cuda")
    acc = torch.zeros_like(g.resid)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_f = t_b = 0.0
    steps, warm = max(1, args.steps // 2), max(1, args.warmup)
    for it in range(warm + steps):
        for gt, lr in imgs:
            ev[0].record()
            out = g.forward_record(lr, wl.lam)
            ev[1].record()
            gout = (2.0 / gt.numel()) * (out - gt)
            g.ctx.backward(gout, g_resid, g_lam)
            ev[2].record()
            acc += g_resid
            torch.cuda.synchronize()
            if it >= warm:
                t_f += ev[0].elapsed_time(ev[1])
                t_b += ev[1].elapsed_time(ev[2])
    Q = 8 * (wl.test_h - 4) * (wl.test_w - 4)
    t_f /= steps
    t_b /= steps
    out = {"metric": "LR patches/s, forward + backward (differentiation form)",
           "value": Q / ((t_f + t_b) * 1e-3), "unit": "LR patches/s", "n_gpus": 1, "steps": steps,
           "warmup": warm, "ms_per_step": t_f + t_b, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32 (FP64 LLE)", "data": "synthetic",
           "config": {"workload": "diff: 8 HR 512^2 images degraded to 256^2 LR x2, 200,000-pair fp32 "
                                  "dictionary, L=16 k=16 w=32 K=5, early stop 48, 3 back-projection iterations, MSE to the HR "
                                  "ground truth; gradients for the residual patches and lambda",
                      "patches_per_step": Q, "parallelism": "single GPU"},
           "extra": {"forward_ms_8_images": t_f, "backward_ms_8_images": t_b,
                     "patches_without_neighbours_last": int((g.results()["m"] == 0).sum()),
                     "grad_lambda_last": float(g_lam.item()),
                     "grad_resid_rows_touched": int((acc.abs().sum(1) > 0).sum().item())}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
