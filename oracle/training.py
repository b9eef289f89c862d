"""Oracle: training-data and table-quality tools of the method.

Training crops (Section 5, "Training Data Generation"): the first-order
gradients (taps [-1, 0, 1] along each axis) of a training image define a
cumulative distribution over its pixels; crop centres are drawn from it and
a fixed-size sub-image around each centre becomes a training image.

Readings (the section gives no formula):
  - the weight of a pixel is its l1 gradient magnitude |dx| + |dy| (FP64 from
    the fp32 pixels, replicate border), quantised to an integer
    q = floor(g * 2^20), saturated at 2^32 - 1 (also for non-finite g), so
    that the cumulative distribution is an exact integer sum whatever the
    summation order;
  - a draw is a 64-bit integer x; with T the sum of the weights, the centre
    is the first pixel (row-major) whose inclusive cumulative weight exceeds
    x mod T; an image without gradient (T = 0) takes pixel x mod (H W);
  - the crop of side S has its top-left corner at the centre minus S // 2,
    clamped so that the crop lies inside the image.

Hashing quality (Section 4.1, "Hashing Quality (determining r)"): the
entropy of a table's bucket occupancy, H = -sum_b p_b log2 p_b with p_b the
fraction of the dictionary in bucket b; the bin width r trades it against
reconstruction quality.

Test infrastructure only: plain numpy, no blocking or reordering beyond the
definitions above.
"""
from __future__ import annotations

import math

import numpy as np

QSHIFT = 20                 # weights are multiples of 2^-20 of a gradient unit
QMAX = (1 << 32) - 1        # saturation of one pixel's weight


def gradient_weights(img: np.ndarray) -> np.ndarray:
    """Integer weight of every pixel of img [H, W] (uint64 [H, W])."""
    x = img.astype(np.float32).astype(np.float64)
    H, W = x.shape
    cols = np.arange(W)
    rows = np.arange(H)
    dx = x[:, np.minimum(cols + 1, W - 1)] - x[:, np.maximum(cols - 1, 0)]
    dy = x[np.minimum(rows + 1, H - 1), :] - x[np.maximum(rows - 1, 0), :]
    g = np.abs(dx) + np.abs(dy)
    scaled = g * float(1 << QSHIFT)
    q = np.full(g.shape, QMAX, dtype=np.uint64)
    ok = scaled < float(QMAX)          # false for NaN and infinities
    q[ok] = np.floor(scaled[ok]).astype(np.uint64)
    return q


def sample_centres(img: np.ndarray, draws: np.ndarray) -> np.ndarray:
    """Row-major pixel index of the centre of each draw (int64 [n])."""
    q = gradient_weights(img).ravel()
    c = np.cumsum(q, dtype=np.uint64)          # inclusive cumulative weights
    T = int(c[-1]) if c.size else 0
    d = draws.astype(np.uint64)
    if T == 0:
        return (d % np.uint64(q.size)).astype(np.int64)
    t = d % np.uint64(T)
    return np.searchsorted(c, t, side="right").astype(np.int64)


def crop_corners(centres: np.ndarray, H: int, W: int, side: int) -> np.ndarray:
    """Top-left corner (row, col) of the side x side crop around each centre,
    clamped inside the H x W image (int64 [n, 2])."""
    r = centres // W - side // 2
    c = centres % W - side // 2
    return np.stack([np.clip(r, 0, H - side), np.clip(c, 0, W - side)], axis=1)


def sample_crops(stack: np.ndarray, draws: np.ndarray, side: int):
    """Crops of every image of stack [n_img, H, W] for its row of draws
    [n_img, m]: corners int64 [n_img, m, 2] and crops fp32 [n_img, m, side, side]."""
    n_img, H, W = stack.shape
    m = draws.shape[1]
    corners = np.zeros((n_img, m, 2), dtype=np.int64)
    crops = np.zeros((n_img, m, side, side), dtype=np.float32)
    for i in range(n_img):
        cen = sample_centres(stack[i], draws[i])
        corners[i] = crop_corners(cen, H, W, side)
        for j in range(m):
            r0, c0 = corners[i, j]
            crops[i, j] = stack[i, r0:r0 + side, c0:c0 + side]
    return corners, crops


def bucket_entropy(keys: np.ndarray) -> np.ndarray:
    """Entropy in bits of each table's bucket occupancy; keys [N, L] are the
    bucket keys of the dictionary's N rows (FP64 [L])."""
    N, L = keys.shape
    out = np.zeros(L, dtype=np.float64)
    for l in range(L):
        _, counts = np.unique(keys[:, l], return_counts=True)
        p = counts.astype(np.float64) / N
        out[l] = -float(np.sum(p * np.log2(p)))
    return out


def entropy_bound(N: int) -> float:
    """Largest possible entropy of N rows: every row in a bucket of its own."""
    return math.log2(N) if N > 0 else 0.0
