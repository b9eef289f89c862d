"""Oracle: p-stable (Cauchy) LSH of Section 3.2 and Section 4.1.

Hash parameters come from a counter-based SplitMix64 stream (Steele, Lea and
Flood, 2014) with normal variates by Marsaglia's polar method; the library
implements the same published generators on its own, so both sides draw the
same alpha and beta from the same seed. Test infrastructure only.
"""
from __future__ import annotations

import math

import numpy as np

from . import _clib

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
EMPTY_KEY = MASK64


def fmix64(z: int) -> int:
    """SplitMix64 output function."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    def __init__(self, state: int):
        self.s = state & MASK64

    def next_u64(self) -> int:
        self.s = (self.s + GOLDEN) & MASK64
        return fmix64(self.s)

    def uniform(self) -> float:
        """Uniform in [0, 1): top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def normal(self) -> float:
        """Standard normal by the polar method; the first variate of each
        accepted pair is returned and the second discarded."""
        while True:
            u1 = 2.0 * self.uniform() - 1.0
            u2 = 2.0 * self.uniform() - 1.0
            s = u1 * u1 + u2 * u2
            if 0.0 < s < 1.0:
                return u1 * math.sqrt(-2.0 * math.log(s) / s)


def table_stream(seed: int, l: int) -> SplitMix64:
    """Independent stream of table l: state fmix64(seed + GOLDEN*(l+1)).
    Tables are nested: the first L tables of an L' > L build are the L-table
    build."""
    return SplitMix64(fmix64((seed + GOLDEN * (l + 1)) & MASK64))


def hash_params(seed: int, L: int, k: int, D: int, w: float, eps: float = 1e-3):
    """alpha [L*k, D] fp32 and beta [L*k] fp32 (Eq. cauchy, Eq. hash_fn).

    Per table l, in order: for each of its k hashes and each of the D
    coordinates, a ~ N(0,1), then b ~ N(0,1) redrawn while |b| < eps,
    alpha = a / b; after the k*D alphas, beta_j = u * w with u ~ U[0,1), one
    per hash. All in FP64, rounded once to fp32."""
    alpha = np.empty((L * k, D), dtype=np.float32)
    beta = np.empty(L * k, dtype=np.float32)
    for l in range(L):
        g = table_stream(seed, l)
        for j in range(k):
            row = alpha[l * k + j]
            for i in range(D):
                a = g.normal()
                b = g.normal()
                while abs(b) < eps:
                    b = g.normal()
                row[i] = np.float32(a / b)
        for j in range(k):
            beta[l * k + j] = np.float32(g.uniform() * w)
    return alpha, beta


def codes(V: np.ndarray, alpha: np.ndarray, beta: np.ndarray, w: float) -> np.ndarray:
    """h = floor((alpha . v + beta) / w) for every row of V and every hash;
    dot product summed sequentially in FP64 (Eq. hash_fn). int32 [n, L*k]."""
    return _clib.codes(V, alpha, beta, w)


def _fmix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def key_multipliers(L: int, k: int) -> np.ndarray:
    """Multipliers of the bucket key: entry (l, j) is output number
    64 l + j + 1 of SplitMix64 started from state 0; columns 0..k-1 weigh the
    k codes of table l and the last column (output 64 l + 64) starts the sum
    (k <= 32). uint64 [L, k + 1]."""
    gen = SplitMix64(0)
    outs = [gen.next_u64() for _ in range(64 * L)]
    return np.array([[outs[64 * l + j] for j in range(k)] + [outs[64 * l + 63]] for l in range(L)],
                    dtype=np.uint64)


def bucket_keys(c: np.ndarray, L: int, k: int) -> np.ndarray:
    """64-bit key of each table's k-tuple of codes (the bin of Section 4.1):
    the start value of table l plus the sum over j of uint32(c_j) times the
    multiplier M_lj, modulo 2^64, through the SplitMix64 output function; a
    key equal to all-ones becomes all-ones minus one. uint64 [n, L]."""
    n = c.shape[0]
    M = key_multipliers(L, k)
    out = np.empty((n, L), dtype=np.uint64)
    with np.errstate(over="ignore"):
        for l in range(L):
            s = np.full(n, M[l, k], dtype=np.uint64)
            for j in range(k):
                cj = (c[:, l * k + j].astype(np.int64) & 0xFFFFFFFF).astype(np.uint64)
                s = s + cj * M[l, j]
            h = _fmix64_np(s)
            h[h == np.uint64(EMPTY_KEY)] = np.uint64(EMPTY_KEY - 1)
            out[:, l] = h
    return out


class Tables:
    """L hash tables over the dictionary: per table the keys sorted ascending
    and the IDs in that order (IDs ascending inside a bin)."""

    def __init__(self, keys: np.ndarray):
        self.L = keys.shape[1]
        self.sorted_keys = []
        self.sorted_ids = []
        for l in range(self.L):
            order = np.argsort(keys[:, l], kind="stable")
            self.sorted_keys.append(keys[order, l])
            self.sorted_ids.append(order.astype(np.int64))

    def bucket_ranges(self, qkeys: np.ndarray):
        """(lo, hi) [Q, L]: bin of each query key inside each table."""
        Q = qkeys.shape[0]
        lo = np.empty((Q, self.L), dtype=np.int64)
        hi = np.empty((Q, self.L), dtype=np.int64)
        for l in range(self.L):
            lo[:, l] = np.searchsorted(self.sorted_keys[l], qkeys[:, l], side="left")
            hi[:, l] = np.searchsorted(self.sorted_keys[l], qkeys[:, l], side="right")
        return lo, hi

    def candidates(self, qkeys: np.ndarray, cap: int = 0):
        """Candidate set of every query: the IDs found in at least one of the
        L tables (t = 1), each once, ascending (Section 3.2; Section 4.2).

        cap > 0 is the early stop of Section 4.2 (searching stops once the
        number of matches reaches the limit): tables are visited in order
        0..L-1 and each bin's IDs in ascending order; an ID already collected
        is skipped; collection stops as soon as `cap` distinct IDs are held."""
        lo, hi = self.bucket_ranges(qkeys)
        out = []
        for q in range(qkeys.shape[0]):
            if cap <= 0:
                parts = [self.sorted_ids[l][lo[q, l]:hi[q, l]] for l in range(self.L)]
                ids = np.concatenate(parts) if parts else np.zeros(0, np.int64)
                out.append(np.unique(ids))
                continue
            got = []
            seen = set()
            for l in range(self.L):
                for i in self.sorted_ids[l][lo[q, l]:hi[q, l]]:
                    i = int(i)
                    if i in seen:
                        continue
                    seen.add(i)
                    got.append(i)
                    if len(got) == cap:
                        break
                if len(got) == cap:
                    break
            out.append(np.array(sorted(got), dtype=np.int64))
        return out, (hi - lo)


def candidates_t(tables: Tables, qkeys: np.ndarray, t: int):
    """The IDs present in at least t of the L tables' bins of each query
    (Section 4.1: a training patch is a match when it shares the query's
    bucket in at least t out of L tables), ascending. t = 1 is the union."""
    lo, hi = tables.bucket_ranges(qkeys)
    out = []
    for q in range(qkeys.shape[0]):
        parts = [tables.sorted_ids[l][lo[q, l]:hi[q, l]] for l in range(tables.L)]
        ids = np.concatenate(parts) if parts else np.zeros(0, np.int64)
        u, c = np.unique(ids, return_counts=True)
        out.append(u[c >= t])
    return out


def build_tables(feat: np.ndarray, alpha: np.ndarray, beta: np.ndarray, w: float, L: int,
                 k: int) -> Tables:
    return Tables(bucket_keys(codes(feat, alpha, beta, w), L, k))
