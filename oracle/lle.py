"""Oracle: nearest neighbours among the candidates, LLE weights, HR synthesis
and overlap blending (Section 3.1, Section 4.2 Eq. LinSys and Eq. HR_Rec,
Section 4 smoothness prior). FP64. Test infrastructure only."""
from __future__ import annotations

import numpy as np

from . import _clib
from .imaging import P, bicubic_up


def knn(qfeat: np.ndarray, dict_feat: np.ndarray, cand: np.ndarray, K: int):
    """The first min(K, |C|) candidates in (distance, ID) order, distance the
    squared l2 distance summed sequentially in FP64 (the LLE objective of
    Eq. LinSys is l2). Returns (ids int64, d2 float64)."""
    if len(cand) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.float64)
    d = _clib.sqdist(qfeat, dict_feat, cand)
    order = np.lexsort((cand, d))[:K]
    return cand[order], d[order]


def l1dist(qfeat: np.ndarray, dict_feat: np.ndarray, cand: np.ndarray) -> np.ndarray:
    """l1 distance of the query to each candidate row: sum over the
    coordinates, in index order, of |q_i - x_i|, in FP64 from the fp32
    values."""
    q = np.asarray(qfeat, dtype=np.float32).astype(np.float64)
    X = np.asarray(dict_feat[cand], dtype=np.float32).astype(np.float64)
    acc = np.zeros(len(cand), dtype=np.float64)
    for i in range(q.shape[0]):
        acc = acc + np.abs(q[i] - X[:, i])
    return acc


def knn_l1(qfeat: np.ndarray, dict_feat: np.ndarray, cand: np.ndarray, K: int):
    """K nearest candidates under l1, the metric the Cauchy hash is sensitive
    to (Section 4.1: the 1-stable distribution preserves l1 distances):
    the first min(K, |C|) in (l1 distance, ID) order."""
    if len(cand) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.float64)
    d = l1dist(qfeat, dict_feat, cand)
    order = np.lexsort((cand, d))[:K]
    return cand[order], d[order]


def lle_weights(qfeat: np.ndarray, nbr_feat: np.ndarray, lam: float) -> np.ndarray:
    """Weights minimising ||y - sum_m w_m y_m||^2 subject to sum_m w_m = 1
    (Eq. LinSys), regularised: with Z = y - Y (rows), G = Z Z^T,
    solve (G + lam * tr(G) * I) w~ = 1 by Cholesky and normalise
    w = w~ / sum(w~). If tr(G) = 0 every neighbour equals the query and the
    weights are uniform."""
    M = nbr_feat.shape[0]
    if M == 0:
        return np.zeros(0)
    Z = qfeat.astype(np.float64)[None, :] - nbr_feat.astype(np.float64)
    G = Z @ Z.T
    tau = float(np.trace(G))
    if tau == 0.0:
        return np.full(M, 1.0 / M)
    A = G + lam * tau * np.eye(M)
    Lc = np.linalg.cholesky(A)
    y = np.linalg.solve(Lc, np.ones(M))
    wt = np.linalg.solve(Lc.T, y)
    return wt / wt.sum()


def synthesize(mu_q: float, w: np.ndarray, nbr_resid: np.ndarray) -> np.ndarray:
    """HR patch x = mu_q + sum_m w_m r_m (Eq. HR_Rec applied to the residual
    patches; mu_q is the mean of the query's LR pixels, the DC that the
    features do not carry)."""
    return mu_q + (w[:, None] * nbr_resid.astype(np.float64)).sum(axis=0)


def blend(patches: list, pos: np.ndarray, valid: np.ndarray, scale: int, lr: np.ndarray):
    """Overlap blend: each HR pixel is the mean of the synthesised patches
    that cover it (the minimiser of the quadratic overlap prior of Section 4
    with equal weights); pixels that no patch covers take the bicubic
    interpolation of the LR image. Returns (hr float64, count int)."""
    h, w = lr.shape
    H, W = scale * h, scale * w
    ps = P * scale
    acc = np.zeros((H, W), dtype=np.float64)
    cnt = np.zeros((H, W), dtype=np.int64)
    for q in range(len(pos)):
        if not valid[q]:
            continue
        y0 = scale * pos[q, 0]
        x0 = scale * pos[q, 1]
        acc[y0:y0 + ps, x0:x0 + ps] += patches[q].reshape(ps, ps)
        cnt[y0:y0 + ps, x0:x0 + ps] += 1
    out = np.empty((H, W), dtype=np.float64)
    m = cnt > 0
    out[m] = acc[m] / cnt[m]
    if (~m).any():
        out[~m] = bicubic_up(lr, scale)[~m]
    return out, cnt
