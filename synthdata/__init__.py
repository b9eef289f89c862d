"""Seeded synthetic inputs for the patch-hashing zoom path.

This module is shared by the HIP path's tests/bench and by the FP64 oracle.
It holds NONE of the method's arithmetic: no blur, no decimation, no features,
no hashing, no LLE. It only draws images and sampling positions from seeds and
records the workload parameters (sizes, L, k, w, K, ...).

Images stand in for the natural-image training set and test images of the
paper (Section 5.1 uses 500 images of a public image database that is not
available here). Each image is 1/f^2 Gaussian noise (power spectrum
proportional to 1/f^2, i.e. amplitude proportional to 1/f, DC removed,
normalised to standard deviation `amp`) added to a piecewise-constant Voronoi
map of `cells` cells whose values are uniform in [0, 1]; the sum is clipped to
[0, 1] and stored as float32. The 1/f^2 spectrum follows natural-image power
laws; the Voronoi edges supply the sparse, heavy-tailed derivatives that the
paper's choice of a Cauchy (l1) hash relies on (Section 4.1, Hashing).
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = 10043980


def fractal_voronoi_image(seed: int, h: int, w: int, amp: float = 0.2,
                          cells: int = 16) -> np.ndarray:
    """One synthetic grayscale image, float32 [h, w] in [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    # 1/f^2 power spectrum noise
    spec = rng.standard_normal((h, w)) + 1j * rng.standard_normal((h, w))
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    f = np.sqrt(fy * fy + fx * fx)
    f[0, 0] = 1.0
    amp_f = 1.0 / f
    amp_f[0, 0] = 0.0
    noise = np.fft.ifft2(spec * amp_f).real
    noise -= noise.mean()
    sd = noise.std()
    if sd > 0:
        noise *= amp / sd
    # Voronoi piecewise-constant map: nearest seed, lower index on ties
    sy = rng.uniform(0.0, h, size=cells)
    sx = rng.uniform(0.0, w, size=cells)
    vals = rng.uniform(0.0, 1.0, size=cells)
    yy = np.arange(h, dtype=np.float64)[:, None]
    xx = np.arange(w, dtype=np.float64)[None, :]
    best = np.full((h, w), np.inf)
    lab = np.zeros((h, w), dtype=np.int64)
    for c in range(cells):
        d = (yy - sy[c]) ** 2 + (xx - sx[c]) ** 2
        m = d < best
        best[m] = d[m]
        lab[m] = c
    img = vals[lab] + noise
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def image_stack(seed0: int, count: int, h: int, w: int, amp: float = 0.2) -> np.ndarray:
    """`count` images with seeds seed0, seed0+1, ...; float32 [count, h, w]."""
    out = np.empty((count, h, w), dtype=np.float32)
    for i in range(count):
        out[i] = fractal_voronoi_image(seed0 + i, h, w, amp=amp)
    return out


def sample_positions(seed: int, n_images: int, h_lr: int, w_lr: int, p: int,
                     n: int) -> np.ndarray:
    """Draw n distinct patch positions (image, i, j) without replacement over
    every image and every top-left LR position i in [0, h_lr-p], j in
    [0, w_lr-p]. Returned int64 [n, 3] in lexicographic (image, i, j) order,
    so that the row index is the patch's unique integer ID (IDs run over all
    images in row-major order, Section 2.1 Notations)."""
    ni = h_lr - p + 1
    nj = w_lr - p + 1
    per = ni * nj
    total = n_images * per
    if n > total:
        raise ValueError(f"n={n} > {total} available positions")
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = np.sort(rng.choice(total, size=n, replace=False))
    img = flat // per
    rem = flat % per
    return np.stack([img, rem // nj, rem % nj], axis=1).astype(np.int64)


@dataclasses.dataclass
class Workload:
    """Sizes, seeds and method parameters of one workload.

    test_lr_direct: the LR test image is drawn directly (True) or an HR
    ground-truth image of size scale*test_h x scale*test_w is drawn and the
    method's degradation makes the LR test image (False)."""
    name: str
    test_h: int
    test_w: int
    scale: int
    feat_mode: int          # 0 = mean-removed pixels (D=25), 1 = 4 gradient channels (D=100)
    dict_images: int
    dict_hr: int            # training HR images are dict_hr x dict_hr
    n_dict: int
    L: int
    k: int
    w: float
    K: int
    lam: float
    bp_iters: int
    sigma_s: float
    sigma_r: float
    test_lr_direct: bool
    seed_test: int
    seed_dict_images: int
    seed_positions: int
    hash_seed: int
    p: int = 5
    blur_sigma: float = 1.0
    rerank: int = 0         # 0 = exact FP32 rank of every candidate; >0 = BF16 screen to this many
    feat_bf16: bool = False
    cap: int = 0            # 0 = union of all bins; >0 = early stop at this many matches
    amp: float = 0.2        # noise amplitude of the images (0: piecewise constant)

    @property
    def D(self) -> int:
        return 25 if self.feat_mode == 0 else 100

    @property
    def Q(self) -> int:
        return (self.test_h - self.p + 1) * (self.test_w - self.p + 1)

    def test_image(self) -> np.ndarray:
        if self.test_lr_direct:
            return fractal_voronoi_image(self.seed_test, self.test_h, self.test_w, amp=self.amp)
        return fractal_voronoi_image(self.seed_test, self.scale * self.test_h,
                                     self.scale * self.test_w, amp=self.amp)

    def dictionary_images(self) -> np.ndarray:
        return image_stack(self.seed_dict_images, self.dict_images, self.dict_hr, self.dict_hr, amp=self.amp)

    def positions(self) -> np.ndarray:
        h_lr = self.dict_hr // self.scale
        return sample_positions(self.seed_positions, self.dict_images, h_lr, h_lr,
                                self.p, self.n_dict)


B = SEED_BASE

WORKLOADS = {
    # one 64x64 LR image, 20k pairs from 8 x 128^2 HR images, mean-removed pixels
    "tiny": Workload("tiny", 64, 64, 2, 0, 8, 128, 20_000, L=8, k=12, w=4.0, K=5,
                     lam=1e-3, bp_iters=1, sigma_s=1.5, sigma_r=0.1, test_lr_direct=True,
                     seed_test=B + 1, seed_dict_images=B + 100, seed_positions=B + 200,
                     hash_seed=1),
    # 256^2 LR -> 512^2, 200k pairs from 64 x 512^2 HR images, 4 gradient channels
    "mid": Workload("mid", 256, 256, 2, 1, 64, 512, 200_000, L=16, k=16, w=4.0, K=5,
                    lam=1e-3, bp_iters=3, sigma_s=1.5, sigma_r=0.1, test_lr_direct=True,
                    seed_test=B + 2, seed_dict_images=B + 300, seed_positions=B + 400,
                    hash_seed=2),
    # 1024^2 LR (degraded from a 2048^2 HR ground truth), 2M pairs from 128 x 512^2
    # (w is not fixed for this workload: 32 is the smallest power of two for
    # which at least 95% of the test patches find K candidates; the early stop
    # at 3L matches bounds the candidates of near-flat patches)
    "precision": Workload("precision", 1024, 1024, 2, 1, 128, 512, 2_000_000, L=24, k=20,
                          w=32.0, K=8, cap=72, lam=1e-3, bp_iters=3, sigma_s=1.5, sigma_r=0.1,
                          test_lr_direct=False, seed_test=B + 3, seed_dict_images=B + 500,
                          seed_positions=B + 600, hash_seed=3, rerank=32, feat_bf16=True),
    # one batch image of the differentiation workload; 200k fp32 pairs (w and
    # the early stop at 3L chosen as for the 1024^2 workload)
    "diff": Workload("diff", 256, 256, 2, 1, 64, 512, 200_000, L=16, k=16, w=32.0, K=5,
                     lam=1e-3, bp_iters=3, sigma_s=1.5, sigma_r=0.1, test_lr_direct=False,
                     seed_test=B + 1000, seed_dict_images=B + 1100, seed_positions=B + 1150,
                     hash_seed=4, cap=48),
}


def scaled(wl: Workload, **kw) -> Workload:
    """A copy of a workload with some fields replaced (smaller test sizes)."""
    return dataclasses.replace(wl, **kw)


def at_scale(wl: Workload, s: int) -> Workload:
    """The workload at zoom factor s: the same LR test size, dictionary size
    and seeds; training images are added while their LR grids hold fewer
    than n_dict patch positions (at x4 a 512^2 HR image gives 124^2)."""
    per = (wl.dict_hr // s - wl.p + 1) ** 2
    need = -(-wl.n_dict // per)
    return dataclasses.replace(wl, name=f"{wl.name}_x{s}", scale=s, dict_images=max(wl.dict_images, need))


# dictionaries of the batched workload: 1M pairs per zoom factor from 64
# seeded 512^2 HR images each; method parameters as the precision workload
BATCHED = {
    s: Workload(f"batched_x{s}", 0, 0, s, 1, 64, 512, 1_000_000, L=24, k=20, w=32.0, K=8, cap=72, lam=1e-3,
                bp_iters=3, sigma_s=1.5, sigma_r=0.1, test_lr_direct=True, seed_test=B + 4,
                seed_dict_images=B + 700 + 100 * s, seed_positions=B + 750 + 100 * s, hash_seed=10 + s,
                rerank=32, feat_bf16=True)
    for s in (2, 3)
}


def batched_images(seed: int = B + 4, count: int = 64):
    """The LR images of the batched workload (drawn directly at LR) with their
    zoom factors: a list of (image float32 [h, w], scale)."""
    return [(fractal_voronoi_image(seed + 1000 + i, h, w), s)
            for i, (h, w, s) in enumerate(batched_sizes(seed, count))]


def batched_sizes(seed: int = B + 4, count: int = 64):
    """Image sizes of the batched workload: side a ~ U{96..1024}, aspect
    rho ~ log-uniform[0.5, 2], b = clamp(round(a*rho), 96, 1024); the first
    half at x2, the second half at x3. Returns a list of (h, w, scale)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        a = int(rng.integers(96, 1025))
        rho = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        b = int(min(1024, max(96, round(a * rho))))
        out.append((a, b, 2 if i < count // 2 else 3))
    return out


def crop_draws(seed: int, n_images: int, per_image: int) -> np.ndarray:
    """64-bit integer draws [n_images, per_image] for the training-crop sampler."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, np.iinfo(np.uint64).max, size=(n_images, per_image), dtype=np.uint64,
                        endpoint=True)
