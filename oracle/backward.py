"""Oracle: gradients of a scalar loss on the zoomed image with respect to the
dictionary's HR residual patches and the LLE regulariser lambda. FP64.
Test infrastructure only.

The forward path is the one of `pipeline`: neighbours (discrete, held at
their forward values), LLE weights of Eq. LinSys with the regulariser
lambda * tr(G), HR synthesis x_q = mu_q + sum_m w_qm r_{n_qm} (Eq. HR_Rec),
the overlap blend (per-pixel mean of the covering patches, bicubic where no
patch covers), and T back-projection iterations (Section 4, Eq. Err_img and
the update that follows it; Section 4.3, Eq. sx2 and Eq. bl_filter_3):

    I' = I + S(I) * F(I),   F = N( Up( I_L - Dec(Blur(I)) ) ),
    S = exp(-(I - Box(I))^2 / (2 sigma_r^2)).

Every linear operator of that iteration is separable: a matrix per axis
applied as A_y X A_x^T. The matrices below are built from the same
definitions as the forward functions of `imaging` and `backproject`, so the
adjoint of each is its transpose. The gradient of one iteration is

    g <- g - Dec_Blur^T Up^T N^T (S g) + (Id - Box)^T [ -(a / sigma_r^2) S F g ],

with a = I - Box(I). The blend's adjoint spreads g(X) / cnt(X) to every
covering patch; the synthesis gives dL/dr_n = sum over (q, m) with n_qm = n
of w_qm g_q, and dL/dw_qm = <g_q, r_{n_qm}>. For lambda, with tau = tr(G),
A = G + lambda tau I, w~ = A^-1 1, sigma = 1^T w~:
dw~/dlambda = -tau A^-1 w~ and dw/dlambda = (dw~/dlambda - w (1^T dw~/dlambda)) / sigma.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import imaging, lle, pipeline
from .imaging import P, gauss_weights, keys_cubic


# ---- one-axis operator matrices ---------------------------------------------
def axis_degrade(n_hr: int, scale: int, sigma: float = 1.0) -> np.ndarray:
    """[n_lr, n_hr]: blur with the Gaussian g (replicate border), keep every
    scale-th sample from 0."""
    g = gauss_weights(sigma)
    R = (len(g) - 1) // 2
    n_lr = (n_hr + scale - 1) // scale
    M = np.zeros((n_lr, n_hr))
    for i in range(n_lr):
        for ti, t in enumerate(range(-R, R + 1)):
            M[i, min(max(scale * i + t, 0), n_hr - 1)] += g[ti]
    return M


def axis_bicubic(n_lr: int, scale: int, n_out: int) -> np.ndarray:
    """[n_out, n_lr]: Keys' cubic (a = -0.5), output X samples X / scale,
    taps floor - 1 .. floor + 2, replicate border."""
    M = np.zeros((n_out, n_lr))
    for X in range(n_out):
        i0 = X // scale
        t = (X % scale) / scale
        for a in range(4):
            M[X, min(max(i0 - 1 + a, 0), n_lr - 1)] += keys_cubic(t - (a - 1))
    return M


def axis_gauss_normalised(n: int, sigma: float) -> np.ndarray:
    """[n, n]: Gaussian exp(-d^2 / (2 sigma^2)), |d| <= ceil(3 sigma), divided by
    the sum of the taps inside [0, n)."""
    R = int(math.ceil(3.0 * sigma))
    M = np.zeros((n, n))
    for X in range(n):
        for d in range(-R, R + 1):
            if 0 <= X + d < n:
                M[X, X + d] = math.exp(-(d * d) / (2.0 * sigma * sigma))
        M[X] /= M[X].sum()
    return M


def axis_box(n: int, R: int) -> np.ndarray:
    """[n, n]: mean over the in-range samples of [X - R, X + R]."""
    M = np.zeros((n, n))
    for X in range(n):
        lo, hi = max(0, X - R), min(n, X + R + 1)
        M[X, lo:hi] = 1.0 / (hi - lo)
    return M


def sep(Ay: np.ndarray, X: np.ndarray, Ax: np.ndarray) -> np.ndarray:
    return Ay @ X @ Ax.T


@dataclasses.dataclass
class BpOps:
    Dy: np.ndarray
    Dx: np.ndarray
    Uy: np.ndarray
    Ux: np.ndarray
    Ny: np.ndarray
    Nx: np.ndarray
    By: np.ndarray
    Bx: np.ndarray


def bp_ops(H: int, W: int, h: int, w: int, scale: int, sigma: float, sigma_s: float) -> BpOps:
    R = int(math.ceil(3.0 * sigma_s))
    return BpOps(axis_degrade(H, scale, sigma), axis_degrade(W, scale, sigma),
                 axis_bicubic(h, scale, H), axis_bicubic(w, scale, W),
                 axis_gauss_normalised(H, sigma_s), axis_gauss_normalised(W, sigma_s),
                 axis_box(H, R), axis_box(W, R))


def bp_terms(I: np.ndarray, lr: np.ndarray, ops: BpOps, sigma_r: float):
    """F, S and a = I - Box(I) of one iteration at the guide I."""
    e = np.asarray(lr, np.float64) - sep(ops.Dy, I, ops.Dx)
    F = sep(ops.Ny, sep(ops.Uy, e, ops.Ux), ops.Nx)
    a = I - sep(ops.By, I, ops.Bx)
    S = np.ones_like(I) if math.isinf(sigma_r) else np.exp(-(a * a) / (2.0 * sigma_r * sigma_r))
    return F, S, a


def bp_step_adjoint(I: np.ndarray, lr: np.ndarray, ops: BpOps, sigma_r: float,
                    g: np.ndarray) -> np.ndarray:
    """dL/dI of one iteration I' = I + S(I) F(I), given g = dL/dI'."""
    F, S, a = bp_terms(I, lr, ops, sigma_r)
    u = S * g
    v = sep(ops.Dy.T, sep(ops.Uy.T, sep(ops.Ny.T, u, ops.Nx.T), ops.Ux.T), ops.Dx.T)
    out = g - v
    if not math.isinf(sigma_r):
        z = -(a / (sigma_r * sigma_r)) * S * F * g
        out = out + z - sep(ops.By.T, z, ops.Bx.T)
    return out


# ---- forward with the records the backward needs ----------------------------
@dataclasses.dataclass
class Record:
    qr: pipeline.QueryResult
    lr: np.ndarray
    scale: int
    lam: float
    sigma: float
    sigma_s: float
    sigma_r: float
    cnt: np.ndarray          # [H, W] patches covering each HR pixel
    guides: list             # I^0 .. I^{T-1}
    out: np.ndarray          # I^T


def forward(pre: pipeline.Prepared, lr: np.ndarray, scale: int, K: int, lam: float, bp_iters: int,
            sigma_s: float = 1.5, sigma_r: float = 0.1, sigma: float = 1.0, cap: int = 0) -> Record:
    from .backproject import bp_step
    qr = pipeline.query(pre, lr, K, lam, cap=cap)
    hr0, cnt = pipeline.reconstruct(qr, lr, scale)
    guides, I = [], hr0
    for _ in range(bp_iters):
        guides.append(I)
        I = bp_step(I, lr, scale, sigma, sigma_s, sigma_r)
    return Record(qr, np.asarray(lr, np.float32), scale, lam, sigma, sigma_s, sigma_r, cnt, guides, I)


def output_given(rec: Record, pre: pipeline.Prepared, resid: np.ndarray, lam: float) -> np.ndarray:
    """The forward output with the neighbours of `rec` held fixed, for other
    residual patches and another lambda (finite differences)."""
    from .backproject import bp_step
    qr = rec.qr
    patches = [None] * len(qr.pos)
    for q in range(len(qr.pos)):
        mq = int(qr.m[q])
        if mq == 0:
            continue
        nid = qr.ids[q, :mq]
        w = lle.lle_weights(qr.feat[q], pre.dictionary.feat[nid], lam)
        patches[q] = lle.synthesize(qr.mu[q], w, resid[nid])
    I, _ = lle.blend(patches, qr.pos, qr.m > 0, rec.scale, rec.lr)
    for _ in range(len(rec.guides)):
        I = bp_step(I, rec.lr, rec.scale, rec.sigma, rec.sigma_s, rec.sigma_r)
    return I


def lle_dw_dlambda(qfeat: np.ndarray, nbr_feat: np.ndarray, lam: float):
    """(w, dw/dlambda) of one patch, FP64."""
    M = nbr_feat.shape[0]
    Z = qfeat.astype(np.float64)[None, :] - nbr_feat.astype(np.float64)
    G = Z @ Z.T
    tau = float(np.trace(G))
    if tau == 0.0:
        return np.full(M, 1.0 / M), np.zeros(M)
    A = G + lam * tau * np.eye(M)
    wt = np.linalg.solve(A, np.ones(M))
    s = wt.sum()
    w = wt / s
    dwt = -tau * np.linalg.solve(A, wt)
    return w, (dwt - w * dwt.sum()) / s


def backward(rec: Record, pre: pipeline.Prepared, g_out: np.ndarray):
    """(dL/dr [N, (5s)^2], dL/dlambda) for dL/dI_out = g_out."""
    H, W = rec.out.shape
    h, w = rec.lr.shape
    g = np.asarray(g_out, np.float64)
    if rec.guides:
        ops = bp_ops(H, W, h, w, rec.scale, rec.sigma, rec.sigma_s)
        for I in reversed(rec.guides):
            g = bp_step_adjoint(I, rec.lr, ops, rec.sigma_r, g)
    # blend: covered pixels are the mean of their patches
    gp = np.where(rec.cnt > 0, g / np.maximum(rec.cnt, 1), 0.0)
    qr = rec.qr
    s = rec.scale
    ps = P * s
    resid = pre.dictionary.resid
    g_r = np.zeros(resid.shape, np.float64)
    g_lam = 0.0
    for q in range(len(qr.pos)):
        mq = int(qr.m[q])
        if mq == 0:
            continue
        y0, x0 = s * int(qr.pos[q, 0]), s * int(qr.pos[q, 1])
        gq = gp[y0:y0 + ps, x0:x0 + ps].reshape(-1)
        nid = qr.ids[q, :mq]
        wq, dw = lle_dw_dlambda(qr.feat[q], pre.dictionary.feat[nid], rec.lam)
        for mi in range(mq):
            g_r[nid[mi]] += wq[mi] * gq
        gw = resid[nid].astype(np.float64) @ gq
        g_lam += float(gw @ dw)
    return g_r, g_lam
