"""Oracle: iterative error back-projection with the approximate cross
bilateral filter (Section 4, Eq. Err_img and the update that follows it;
Section 4.3, Eq. sx2, Eq. bl_filter_2, Eq. bl_filter_3). FP64.
Test infrastructure only.

Readings (the paper is ambiguous here):
 - the LR error is I_L - (g * I_H) decimated, so that adding its upsampled,
   filtered version moves the estimate towards consistency (Irani's update);
 - the upsampler is bicubic (Keys, a = -0.5, phase 0, replicate border);
 - the spatial kernel C is a Gaussian of sigma_s over a (2R+1)^2 window,
   R = ceil(3 sigma_s), normalised over the taps that fall inside the image;
 - the range weight compares the current HR estimate at x with the mean of
   the current HR estimate over the same window (in-image pixels only):
   S(x) = exp(-(I(x) - mean_Gamma I)^2 / (2 sigma_r^2));
 - the update is I <- I + S (elementwise) * (C * E), E the upsampled error.
"""
from __future__ import annotations

import math

import numpy as np

from .imaging import bicubic_up, degrade


def _taps(sigma: float):
    R = int(math.ceil(3.0 * sigma))
    c = np.array([math.exp(-(d * d) / (2.0 * sigma * sigma)) for d in range(-R, R + 1)])
    return R, c


def gauss_filter_normalised(E: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian smoothing normalised by the weight of the in-image taps
    (separable: the in-image window is a rectangle)."""
    R, c = _taps(sigma)
    H, W = E.shape
    out = np.zeros_like(E, dtype=np.float64)
    nrm = np.zeros(W)
    tmp = np.zeros((H, W))
    for ti, d in enumerate(range(-R, R + 1)):
        lo, hi = max(0, -d), min(W, W - d)
        tmp[:, lo:hi] += c[ti] * E[:, lo + d:hi + d]
        nrm[lo:hi] += c[ti]
    tmp /= nrm[None, :]
    nrm = np.zeros(H)
    for ti, d in enumerate(range(-R, R + 1)):
        lo, hi = max(0, -d), min(H, H - d)
        out[lo:hi, :] += c[ti] * tmp[lo + d:hi + d, :]
        nrm[lo:hi] += c[ti]
    return out / nrm[:, None]


def box_mean(I: np.ndarray, R: int) -> np.ndarray:
    """Mean over the in-image pixels of the (2R+1)^2 window (the mean of
    Eq. sx2; the paper evaluates it with an integral image)."""
    H, W = I.shape
    S = np.zeros((H + 1, W + 1))
    S[1:, 1:] = np.cumsum(np.cumsum(I, axis=0), axis=1)
    y = np.arange(H)
    x = np.arange(W)
    y0 = np.clip(y - R, 0, H)[:, None]
    y1 = np.clip(y + R + 1, 0, H)[:, None]
    x0 = np.clip(x - R, 0, W)[None, :]
    x1 = np.clip(x + R + 1, 0, W)[None, :]
    tot = S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]
    return tot / ((y1 - y0) * (x1 - x0))


def range_weight(I: np.ndarray, sigma_s: float, sigma_r: float) -> np.ndarray:
    R = int(math.ceil(3.0 * sigma_s))
    mu = box_mean(I, R)
    return np.exp(-((I - mu) ** 2) / (2.0 * sigma_r * sigma_r))


def bp_step(I: np.ndarray, lr: np.ndarray, scale: int, sigma_blur: float, sigma_s: float,
            sigma_r: float) -> np.ndarray:
    """One back-projection iteration."""
    sim = degrade(I, scale, sigma_blur, to_f32=False)
    e = np.asarray(lr, dtype=np.float64) - sim
    E = bicubic_up(e, scale, I.shape[0], I.shape[1])
    F = gauss_filter_normalised(E, sigma_s)
    if math.isinf(sigma_r):
        S = np.ones_like(I)
    else:
        S = range_weight(I, sigma_s, sigma_r)
    return I + S * F


def backproject(I0: np.ndarray, lr: np.ndarray, scale: int, iters: int, sigma_blur: float = 1.0,
                sigma_s: float = 1.5, sigma_r: float = 0.1) -> np.ndarray:
    I = np.asarray(I0, dtype=np.float64).copy()
    for _ in range(iters):
        I = bp_step(I, lr, scale, sigma_blur, sigma_s, sigma_r)
    return I


def exact_cross_bilateral(E: np.ndarray, I: np.ndarray, sigma_s: float,
                          sigma_r: float) -> np.ndarray:
    """The O(r^2) cross bilateral filter of Eq. bl_filter / Eq. normalization
    with the range kernel on the guide I, filtering E. Used only to quantify
    the approximation of Section 4.3 (small images)."""
    R, c = _taps(sigma_s)
    H, W = E.shape
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    for a, dy in enumerate(range(-R, R + 1)):
        for b, dx in enumerate(range(-R, R + 1)):
            y0, y1 = max(0, -dy), min(H, H - dy)
            x0, x1 = max(0, -dx), min(W, W - dx)
            Iy = I[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
            wgt = c[a] * c[b] * np.exp(-((I[y0:y1, x0:x1] - Iy) ** 2) / (2.0 * sigma_r ** 2))
            num[y0:y1, x0:x1] += wgt * E[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
            den[y0:y1, x0:x1] += wgt
    return num / den


def backproject_exact(I0: np.ndarray, lr: np.ndarray, scale: int, iters: int, sigma_blur: float = 1.0,
                      sigma_s: float = 1.5, sigma_r: float = 0.1) -> np.ndarray:
    """Back-projection with the filter that Section 4.3 approximates: each
    iteration adds the exact cross bilateral filter of the upsampled error
    (guide: the current estimate) instead of S * (C * E). Used only to report
    the effect of the approximation on the result (small images)."""
    I = np.asarray(I0, dtype=np.float64).copy()
    for _ in range(iters):
        sim = degrade(I, scale, sigma_blur, to_f32=False)
        E = bicubic_up(np.asarray(lr, dtype=np.float64) - sim, scale, I.shape[0], I.shape[1])
        I = I + exact_cross_bilateral(E, I, sigma_s, sigma_r)
    return I
