"""Oracle: degradation model, bicubic upsampling, patch features, dictionary.

FP64 throughout; the fp32 roundings stated below are part of the definition
(the stored LR images, features and HR residuals are fp32 arrays).
Test infrastructure only.
"""
from __future__ import annotations

import math

import numpy as np

P = 5  # LR patch side (Section 4.2: 5x5 patches)


# ---------------------------------------------------------------------------
# Degradation: LR = (HR * K(sigma^2)) decimated by D (Section 2.1 Notations)
# ---------------------------------------------------------------------------
def gauss_weights(sigma: float, radius: int | None = None) -> np.ndarray:
    """Normalised 1-D Gaussian taps for offsets -R..R, R = ceil(3 sigma).
    Each tap exp(-(t*t) / (2 sigma sigma)) uses host libm's exp; the taps are
    summed in ascending offset order and each is divided by that sum."""
    R = int(math.ceil(3.0 * sigma)) if radius is None else radius
    e = [math.exp(-(t * t) / (2.0 * sigma * sigma)) for t in range(-R, R + 1)]
    s = 0.0
    for x in e:
        s = s + x
    return np.array([x / s for x in e], dtype=np.float64)


def _clampi(idx: np.ndarray, n: int) -> np.ndarray:
    return np.clip(idx, 0, n - 1)


def degrade(hr: np.ndarray, scale: int, sigma: float = 1.0, to_f32: bool = True) -> np.ndarray:
    """Blur with the Gaussian g (replicate border) then keep every scale-th
    pixel starting at 0 (phase 0): LR[i, j] = (g * HR)[s i, s j].

    Fixed evaluation order (so that an exact re-implementation reproduces the
    same FP64 value): horizontal pass first, H(r, c) = sum over t ascending of
    g_t * HR[r, clamp(c + t)], then the vertical pass at the kept rows,
    V(i, j) = sum over t ascending of g_t * H(clamp(s i + t), s j); every
    product and every addition rounded in FP64, accumulation starting at 0.
    With to_f32 the result is rounded once to fp32."""
    hr = np.asarray(hr, dtype=np.float64)
    Hh, Wh = hr.shape
    g = gauss_weights(sigma)
    R = (len(g) - 1) // 2
    h = (Hh + scale - 1) // scale
    w = (Wh + scale - 1) // scale
    cols = np.arange(w) * scale
    # horizontal pass at the kept columns, all rows
    Hp = np.zeros((Hh, w), dtype=np.float64)
    for ti, t in enumerate(range(-R, R + 1)):
        Hp = Hp + g[ti] * hr[:, _clampi(cols + t, Wh)]
    rows = np.arange(h) * scale
    V = np.zeros((h, w), dtype=np.float64)
    for ti, t in enumerate(range(-R, R + 1)):
        V = V + g[ti] * Hp[_clampi(rows + t, Hh), :]
    return V.astype(np.float32) if to_f32 else V


def degrade_images(hr_stack: np.ndarray, scale: int, sigma: float = 1.0) -> np.ndarray:
    return np.stack([degrade(x, scale, sigma) for x in hr_stack])


# ---------------------------------------------------------------------------
# Bicubic interpolation (the upsampler of the back-projection, Section 4 and
# Section 4.3; also the fill for HR pixels that no patch covers)
# ---------------------------------------------------------------------------
def keys_cubic(x: float, a: float = -0.5) -> float:
    """Keys' cubic convolution kernel with a = -0.5."""
    x = abs(x)
    if x <= 1.0:
        return (a + 2.0) * x ** 3 - (a + 3.0) * x ** 2 + 1.0
    if x < 2.0:
        return a * x ** 3 - 5.0 * a * x ** 2 + 8.0 * a * x - 4.0 * a
    return 0.0


def bicubic_up(lr: np.ndarray, scale: int, out_h: int | None = None,
               out_w: int | None = None) -> np.ndarray:
    """HR pixel X samples LR coordinate X / scale (phase 0); four taps at
    floor - 1 .. floor + 2 per axis, replicate border. FP64."""
    lr = np.asarray(lr, dtype=np.float64)
    h, w = lr.shape
    H = scale * h if out_h is None else out_h
    W = scale * w if out_w is None else out_w

    def axis(n_out, n_in):
        idx = np.zeros((n_out, 4), dtype=np.int64)
        wt = np.zeros((n_out, 4), dtype=np.float64)
        for X in range(n_out):
            i0 = X // scale
            t = (X % scale) / scale
            for a in range(4):
                idx[X, a] = min(max(i0 - 1 + a, 0), n_in - 1)
                wt[X, a] = keys_cubic(t - (a - 1))
        return idx, wt

    iy, wy = axis(H, h)
    ix, wx = axis(W, w)
    # along x for every LR row, then along y
    tmp = np.zeros((h, W), dtype=np.float64)
    for b in range(4):
        tmp += wx[:, b][None, :] * lr[:, ix[:, b]]
    out = np.zeros((H, W), dtype=np.float64)
    for a in range(4):
        out += wy[:, a][:, None] * tmp[iy[:, a], :]
    return out


# ---------------------------------------------------------------------------
# Patch features (Section 4.1, "Feature representation")
# ---------------------------------------------------------------------------
FEAT_MEANREM = 0
FEAT_GRAD4 = 1


def feature_dim(mode: int) -> int:
    return 25 if mode == FEAT_MEANREM else 100


def patch_mean(lr: np.ndarray, ij: np.ndarray) -> np.ndarray:
    """Mean of each 5x5 LR patch: FP64 sum in row-major order, then / 25."""
    lr = np.asarray(lr, dtype=np.float64)
    i = ij[:, 0]
    j = ij[:, 1]
    s = np.zeros(len(ij), dtype=np.float64)
    for a in range(P):
        for b in range(P):
            s = s + lr[i + a, j + b]
    return s / float(P * P)


def gradient_maps(lr: np.ndarray) -> np.ndarray:
    """The four gradient maps of the LR image, fp32 [4, h, w]: correlation with
    [-1, 0, 1] along x and y (first order) and [-1, 0, 2, 0, -1] along x and y
    (second order), replicate border. Evaluated in FP64 from the fp32 pixels
    in the order  dx = I(c+1) - I(c-1),  dxx = (2 I(c) - I(c-2)) - I(c+2),
    then rounded once to fp32."""
    I = np.asarray(lr, dtype=np.float64)
    h, w = I.shape
    c = np.arange(w)
    r = np.arange(h)
    dx = I[:, _clampi(c + 1, w)] - I[:, _clampi(c - 1, w)]
    dy = I[_clampi(r + 1, h), :] - I[_clampi(r - 1, h), :]
    dxx = (2.0 * I - I[:, _clampi(c - 2, w)]) - I[:, _clampi(c + 2, w)]
    dyy = (2.0 * I - I[_clampi(r - 2, h), :]) - I[_clampi(r + 2, h), :]
    return np.stack([dx, dy, dxx, dyy]).astype(np.float32)


def features(lr: np.ndarray, ij: np.ndarray, mode: int) -> np.ndarray:
    """Feature vectors of the 5x5 LR patches with top-left corners ij [n, 2].

    mode 0: the 25 pixels minus the patch mean (FP64), rounded to fp32.
    mode 1: the 5x5 windows of the four gradient maps, channel-major
            [dx, dy, dxx, dyy], row-major within a channel (D = 100)."""
    ij = np.asarray(ij, dtype=np.int64)
    i = ij[:, 0]
    j = ij[:, 1]
    lr = np.asarray(lr, dtype=np.float32)
    if mode == FEAT_MEANREM:
        mu = patch_mean(lr, ij)
        out = np.empty((len(ij), 25), dtype=np.float32)
        for a in range(P):
            for b in range(P):
                out[:, a * P + b] = (lr[i + a, j + b].astype(np.float64) - mu).astype(np.float32)
        return out
    maps = gradient_maps(lr)
    out = np.empty((len(ij), 100), dtype=np.float32)
    for ch in range(4):
        for a in range(P):
            for b in range(P):
                out[:, ch * 25 + a * P + b] = maps[ch, i + a, j + b]
    return out


def all_positions(h: int, w: int) -> np.ndarray:
    """Top-left corners of every stride-1 5x5 patch in row-major order."""
    ii, jj = np.meshgrid(np.arange(h - P + 1), np.arange(w - P + 1), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel()], axis=1).astype(np.int64)


# ---------------------------------------------------------------------------
# Training dictionary (Section 2.1): LR/HR patch pairs with unique integer IDs
# ---------------------------------------------------------------------------
class Dictionary:
    """feat  fp32 [N, D]       features of the LR patches
       resid fp32 [N, (5s)^2]  HR patch minus the mean of its LR patch
       The HR patch of pair n is recovered as resid[n] + mean(LR patch n)."""

    def __init__(self, feat, resid, scale, mode, lr_mean=None):
        self.feat = feat
        self.resid = resid
        self.scale = scale
        self.mode = mode
        self.lr_mean = lr_mean

    @property
    def n(self):
        return self.feat.shape[0]


def build_dictionary(hr_stack: np.ndarray, positions: np.ndarray, scale: int, mode: int,
                     sigma: float = 1.0, lr_stack: np.ndarray | None = None) -> Dictionary:
    """Cut the pairs at `positions` (image, i, j) (row index = ID). The LR
    training images are the degraded HR images; each HR patch is the
    5s x 5s block at (s i, s j). Residual = fp32(HR - mean(LR patch))."""
    n = len(positions)
    D = feature_dim(mode)
    ps = P * scale
    feat = np.empty((n, D), dtype=np.float32)
    resid = np.empty((n, ps * ps), dtype=np.float32)
    lr_mean = np.empty(n, dtype=np.float64)
    imgs = positions[:, 0]
    for im in np.unique(imgs):
        sel = np.nonzero(imgs == im)[0]
        hr = hr_stack[im]
        lr = degrade(hr, scale, sigma) if lr_stack is None else lr_stack[im]
        ij = positions[sel, 1:3]
        feat[sel] = features(lr, ij, mode)
        mu = patch_mean(lr, ij)
        lr_mean[sel] = mu
        hp = np.empty((len(sel), ps * ps), dtype=np.float64)
        for a in range(ps):
            for b in range(ps):
                hp[:, a * ps + b] = hr[scale * ij[:, 0] + a, scale * ij[:, 1] + b]
        resid[sel] = (hp - mu[:, None]).astype(np.float32)
    return Dictionary(feat, resid, scale, mode, lr_mean)


# ---------------------------------------------------------------------------
# Interpolated pairing (Section 2.1): the LR training images are interpolated
# back to the size of the HR images and both are cut at the same places
# ---------------------------------------------------------------------------
def interpolated_lr(lr: np.ndarray, scale: int) -> np.ndarray:
    """The LR image brought back to the HR grid: bicubic_up (FP64) of the fp32
    LR image, rounded once to fp32."""
    return bicubic_up(np.asarray(lr, dtype=np.float32), scale).astype(np.float32)


def build_dictionary_interp(hr_stack: np.ndarray, positions: np.ndarray, scale: int, mode: int,
                            sigma: float = 1.0) -> Dictionary:
    """Pairs of 5x5 patches at HR-grid positions (image, r, c): the LR patch
    from the degraded image interpolated back to the HR size, the HR patch
    from the HR image at the same place (a dictionary of HR patch side 5,
    queried at zoom factor 1). H and W must be multiples of the scale."""
    H, W = hr_stack.shape[1:]
    assert H % scale == 0 and W % scale == 0
    ups = {}
    for im in np.unique(positions[:, 0]):
        ups[im] = interpolated_lr(degrade(hr_stack[im], scale, sigma), scale)
    lr_stack = np.zeros(hr_stack.shape, dtype=np.float32)
    for im, u in ups.items():
        lr_stack[im] = u
    return build_dictionary(hr_stack, positions, 1, mode, sigma, lr_stack=lr_stack)
