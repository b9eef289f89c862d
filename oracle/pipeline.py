"""Oracle: the whole path, step by step, for one LR image.

    features -> hash codes -> bucket keys -> candidates (union over tables)
    -> K nearest (exact FP64 distance, ties by ID) -> LLE weights
    -> HR synthesis -> overlap blend -> back-projection

Test infrastructure only: used by tests/, the package smoke check and the
CPU baseline leg of the benchmark; never by the product path.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import imaging, lle, lsh
from .backproject import backproject


@dataclasses.dataclass
class Prepared:
    dictionary: imaging.Dictionary
    alpha: np.ndarray
    beta: np.ndarray
    tables: lsh.Tables
    dict_keys: np.ndarray
    L: int
    k: int
    w: float


def prepare(hr_stack, positions, scale, mode, L, k, w, seed, sigma=1.0) -> Prepared:
    d = imaging.build_dictionary(hr_stack, positions, scale, mode, sigma)
    alpha, beta = lsh.hash_params(seed, L, k, d.feat.shape[1], w)
    keys = lsh.bucket_keys(lsh.codes(d.feat, alpha, beta, w), L, k)
    return Prepared(d, alpha, beta, lsh.Tables(keys), keys, L, k, w)


@dataclasses.dataclass
class QueryResult:
    pos: np.ndarray          # [Q, 2] top-left LR corners
    feat: np.ndarray         # [Q, D] fp32
    mu: np.ndarray           # [Q] FP64 LR patch means
    codes: np.ndarray        # [Q, L*k] int32
    keys: np.ndarray         # [Q, L] uint64
    bucket_sizes: np.ndarray  # [Q, L]
    cand: list               # Q arrays of sorted unique IDs
    ids: np.ndarray          # [Q, K] int64, -1 past m
    d2: np.ndarray           # [Q, K] FP64, nan past m
    m: np.ndarray            # [Q] number of neighbours used (min(K, |C|))
    weights: np.ndarray      # [Q, K] FP64, 0 past m
    patches: list            # Q synthesised HR patches (FP64) or None
    all_weights: list = None  # all_matches: Q arrays of weights over cand[q] (in cand order)


def query(pre: Prepared, lr: np.ndarray, K: int, lam: float, pos=None,
          synthesize: bool = True, cap: int = 0, metric: str = "l2", t: int = 0,
          all_matches: bool = False) -> QueryResult:
    """metric "l2": neighbours by squared l2 distance (the LLE objective);
    "l1": by l1 distance (the hash's metric); the LLE weights are the same
    l2 solve for both. t > 0: the candidates are the IDs in at least t of the
    L bins (Section 4.1) instead of the union / early stop.
    all_matches: the weights are solved over all M matches of the patch
    (Eq. LinSys with m = 1..M, Section 4.2) and the HR patch is synthesised
    from all of them (Eq. HR_Rec); the K nearest are still reported."""
    mode = pre.dictionary.mode
    lr = np.asarray(lr, dtype=np.float32)
    if pos is None:
        pos = imaging.all_positions(*lr.shape)
    pos = np.asarray(pos, dtype=np.int64)
    feat = imaging.features(lr, pos, mode)
    mu = imaging.patch_mean(lr, pos)
    c = lsh.codes(feat, pre.alpha, pre.beta, pre.w)
    keys = lsh.bucket_keys(c, pre.L, pre.k)
    cand, bsz = pre.tables.candidates(keys, cap)
    if t > 0:
        cand = lsh.candidates_t(pre.tables, keys, t)
    Q = len(pos)
    ids = np.full((Q, K), -1, dtype=np.int64)
    d2 = np.full((Q, K), np.nan)
    m = np.zeros(Q, dtype=np.int64)
    wts = np.zeros((Q, K))
    patches = [None] * Q
    all_w = [None] * Q if all_matches else None
    D = pre.dictionary
    for q in range(Q):
        nid, nd = (lle.knn_l1 if metric == "l1" else lle.knn)(feat[q], D.feat, cand[q], K)
        mq = len(nid)
        m[q] = mq
        ids[q, :mq] = nid
        d2[q, :mq] = nd
        if mq == 0:
            continue
        if all_matches:
            wa = lle.lle_weights(feat[q], D.feat[cand[q]], lam)
            all_w[q] = wa
            if synthesize:
                patches[q] = lle.synthesize(mu[q], wa, D.resid[cand[q]])
            continue
        w = lle.lle_weights(feat[q], D.feat[nid], lam)
        wts[q, :mq] = w
        if synthesize:
            patches[q] = lle.synthesize(mu[q], w, D.resid[nid])
    return QueryResult(pos, feat, mu, c, keys, bsz, cand, ids, d2, m, wts, patches, all_w)


def prepare_interp(hr_stack, positions, scale, mode, L, k, w, seed, sigma=1.0) -> Prepared:
    """Tables over interpolated pairs (Section 2.1): positions on the HR
    grid, 5x5 HR patches (used at zoom factor 1)."""
    d = imaging.build_dictionary_interp(hr_stack, positions, scale, mode, sigma)
    alpha, beta = lsh.hash_params(seed, L, k, d.feat.shape[1], w)
    keys = lsh.bucket_keys(lsh.codes(d.feat, alpha, beta, w), L, k)
    return Prepared(d, alpha, beta, lsh.Tables(keys), keys, L, k, w)


def run_interp(pre: Prepared, lr, scale, K, lam, bp_iters, sigma_s=1.5, sigma_r=0.1, sigma=1.0, cap=0):
    """The interpolated pairing end to end: the LR image interpolated to the
    HR grid, queried at zoom factor 1 (5x5 HR patches, stride 1), blended,
    then back-projected against the LR image at its own zoom factor."""
    up = imaging.interpolated_lr(lr, scale)
    qr = query(pre, up, K, lam, cap=cap)
    hr, _ = reconstruct(qr, up, 1)
    return qr, up, hr, backproject(hr, lr, scale, bp_iters, sigma, sigma_s, sigma_r)


def reconstruct(qr: QueryResult, lr: np.ndarray, scale: int):
    return lle.blend(qr.patches, qr.pos, qr.m > 0, scale, np.asarray(lr, np.float32))


def run(pre: Prepared, lr, scale, K, lam, bp_iters, sigma_s=1.5, sigma_r=0.1, sigma=1.0, cap=0):
    qr = query(pre, lr, K, lam, cap=cap)
    hr, cnt = reconstruct(qr, lr, scale)
    hr_bp = backproject(hr, lr, scale, bp_iters, sigma, sigma_s, sigma_r)
    return qr, hr, hr_bp
