"""Pins of the oracle's hashing (Section 3.2, Section 4.1 Eq. hash_fn and
Eq. cauchy) against things other than itself: published generator outputs,
distribution laws, exact rational arithmetic, Datar et al.'s collision
probability for 1-stable projections, brute-force bucket matching."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import lsh, lle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    g = lsh.SplitMix64(1234567)
    assert [g.next_u64() for _ in range(len(vals))] == vals


def test_polar_normals_are_standard_normal():
    g = lsh.SplitMix64(77)
    z = np.array([g.normal() for _ in range(20000)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.05 and abs(z.var() - 1.0) < 0.05


def test_alpha_is_cauchy_beta_uniform():
    w = 4.0
    alpha, beta = lsh.hash_params(5, L=40, k=10, D=50, w=w)
    a = alpha.astype(np.float64).ravel()
    # ratio of two independent standard normals is standard Cauchy (Eq. cauchy)
    assert stats.kstest(a, "cauchy").pvalue > 1e-3
    assert abs(np.median(np.abs(a)) - 1.0) < 0.03
    # |b| >= eps bounds |alpha| by max|a| / eps
    assert np.abs(a).max() < 10.0 / 1e-3
    b = beta.astype(np.float64)
    assert b.min() >= 0.0 and b.max() <= w
    assert stats.kstest(b / w, "uniform").pvalue > 1e-3


def test_tables_are_nested_and_seeded():
    a2, b2 = lsh.hash_params(9, L=2, k=3, D=7, w=4.0)
    a4, b4 = lsh.hash_params(9, L=4, k=3, D=7, w=4.0)
    assert np.array_equal(a2, a4[:6]) and np.array_equal(b2, b4[:6])
    a2s, _ = lsh.hash_params(10, L=2, k=3, D=7, w=4.0)
    assert not np.array_equal(a2, a2s)


def test_codes_match_exact_rational_floor():
    rng = np.random.default_rng(3)
    D, m, n, w = 25, 40, 60, 4.0
    V = rng.standard_normal((n, D)).astype(np.float32)
    A, beta = lsh.hash_params(11, L=4, k=10, D=D, w=w)
    c = lsh.codes(V, A, beta, w)
    for r in range(n):
        for j in range(m):
            s = sum(Fraction(float(A[j, i])) * Fraction(float(V[r, i])) for i in range(D))
            t = (s + Fraction(float(beta[j]))) / Fraction(w)
            exact = math.floor(t)
            # the FP64 sum differs from the exact value by ~1e-13 at most
            if abs(float(t - round(t))) > 1e-9:
                assert c[r, j] == exact, (r, j)


def _datar_cauchy(c, w):
    x = w / c
    return 2.0 * math.atan(x) / math.pi - (1.0 / (math.pi * x)) * math.log(1.0 + x * x)


@pytest.mark.parametrize("cdist", [0.5, 2.0, 6.0])
def test_collision_rate_matches_datar_cauchy_formula(cdist):
    """For a fixed pair at l1 distance c and random (alpha, beta) the event
    h(u) == h(v) has probability p(c) of Datar et al. (1-stable case)."""
    w = 4.0
    D = 16
    rng = np.random.default_rng(int(cdist * 10))
    u = rng.standard_normal(D)
    d = rng.standard_normal(D)
    d *= cdist / np.abs(d).sum()
    v = u + d
    A, beta = lsh.hash_params(21, L=400, k=50, D=D, w=w)
    cu = lsh.codes(u[None].astype(np.float32), A, beta, w)[0]
    cv = lsh.codes(v[None].astype(np.float32), A, beta, w)[0]
    # fp32 rounding of u, v shifts c by ~1e-7 relative
    c32 = float(np.abs(u.astype(np.float32).astype(np.float64) -
                       v.astype(np.float32).astype(np.float64)).sum())
    p = _datar_cauchy(c32, w)
    n = len(cu)
    rate = (cu == cv).mean()
    assert abs(rate - p) < 4.5 * math.sqrt(p * (1 - p) / n) + 1e-3, (rate, p)


def test_keys_identify_code_tuples():
    rng = np.random.default_rng(4)
    c = rng.integers(-3, 3, size=(3000, 2 * 5)).astype(np.int32)
    keys = lsh.bucket_keys(c, L=2, k=5)
    for l in range(2):
        tup = {}
        for r in range(len(c)):
            t = tuple(c[r, l * 5:(l + 1) * 5])
            tup.setdefault(t, set()).add(int(keys[r, l]))
        assert all(len(s) == 1 for s in tup.values())          # equal tuple -> equal key
        assert len({next(iter(s)) for s in tup.values()}) == len(tup)  # distinct -> distinct
    assert not (keys == np.uint64(lsh.EMPTY_KEY)).any()
    # the same tuple in two different tables gets different keys
    same = np.zeros((1, 10), np.int32)
    k2 = lsh.bucket_keys(same, 2, 5)
    assert k2[0, 0] != k2[0, 1]


def test_key_depends_on_every_position_and_the_order():
    rng = np.random.default_rng(11)
    L, k = 3, 7
    c = rng.integers(-50, 50, size=(200, L * k)).astype(np.int32)
    base = lsh.bucket_keys(c, L, k)
    for j in range(L * k):
        d = c.copy()
        d[:, j] += 1
        assert (lsh.bucket_keys(d, L, k)[:, j // k] != base[:, j // k]).all()
        others = [l for l in range(L) if l != j // k]
        assert (lsh.bucket_keys(d, L, k)[:, others] == base[:, others]).all()
    # swapping two unequal codes of a table changes its key
    s = c.copy()
    s[:, [0, 1]] = s[:, [1, 0]]
    diff = c[:, 0] != c[:, 1]
    assert (lsh.bucket_keys(s, L, k)[diff, 0] != base[diff, 0]).all()
    # the multipliers are the SplitMix64 stream from state 0, 64 per table
    gen = lsh.SplitMix64(0)
    first = [gen.next_u64() for _ in range(64 + 2)]
    M = lsh.key_multipliers(2, 3)
    assert int(M[0, 0]) == first[0] and int(M[0, 2]) == first[2] and int(M[1, 1]) == first[65]
    assert int(M[0, 3]) == first[63] and M.shape == (2, 4)


def _brute_candidates(qc, dc, L, k, cap=0):
    """Candidates by comparing the k-tuples of codes directly (no keys)."""
    out = []
    for q in range(len(qc)):
        got = []
        seen = set()
        for l in range(L):
            hit = np.nonzero((dc[:, l * k:(l + 1) * k] == qc[q, l * k:(l + 1) * k]).all(1))[0]
            for i in hit:
                if int(i) not in seen:
                    seen.add(int(i))
                    got.append(int(i))
                    if cap and len(got) == cap:
                        break
            if cap and len(got) == cap:
                break
        out.append(np.array(sorted(got), dtype=np.int64))
    return out


@pytest.mark.parametrize("cap", [0, 7])
def test_candidates_equal_brute_force_tuple_matching(cap):
    rng = np.random.default_rng(5)
    D, L, k, w = 10, 6, 3, 2.0
    Y = rng.standard_normal((400, D)).astype(np.float32)
    Qf = (Y[rng.integers(0, 400, 50)] + 0.3 * rng.standard_normal((50, D))).astype(np.float32)
    A, beta = lsh.hash_params(2, L, k, D, w)
    dc = lsh.codes(Y, A, beta, w)
    qc = lsh.codes(Qf, A, beta, w)
    tabs = lsh.Tables(lsh.bucket_keys(dc, L, k))
    cand, _ = tabs.candidates(lsh.bucket_keys(qc, L, k), cap)
    ref = _brute_candidates(qc, dc, L, k, cap)
    assert sum(len(c) for c in cand) > 0
    for a, b in zip(cand, ref):
        assert np.array_equal(a, b)


def test_capped_candidates_first_occurrence_reference():
    """Second construction of the early stop: first occurrences of the
    table-ordered concatenation of the bins, truncated."""
    rng = np.random.default_rng(6)
    D, L, k, w = 8, 5, 2, 3.0
    Y = rng.standard_normal((600, D)).astype(np.float32)
    A, beta = lsh.hash_params(3, L, k, D, w)
    tabs = lsh.Tables(lsh.bucket_keys(lsh.codes(Y, A, beta, w), L, k))
    qk = lsh.bucket_keys(lsh.codes(Y[:40], A, beta, w), L, k)
    lo, hi = tabs.bucket_ranges(qk)
    for cap in (1, 5, 30):
        cand, _ = tabs.candidates(qk, cap)
        full, _ = tabs.candidates(qk, 0)
        for q in range(40):
            cat = np.concatenate([tabs.sorted_ids[l][lo[q, l]:hi[q, l]] for l in range(L)])
            _, first = np.unique(cat, return_index=True)
            ref = np.sort(cat[np.sort(first)][:cap])
            assert np.array_equal(cand[q], ref)
            assert len(cand[q]) == min(cap, len(full[q]))
            assert np.isin(cand[q], full[q]).all()


def test_huge_w_gives_exhaustive_knn():
    """w -> infinity puts every point in one bin, so LSH k-NN is exhaustive
    k-NN."""
    rng = np.random.default_rng(7)
    D, L, k, w, K = 12, 2, 4, 1e30, 5
    Y = rng.random((300, D)).astype(np.float32)
    Qf = rng.random((20, D)).astype(np.float32)
    A, beta = lsh.hash_params(4, L, k, D, w)
    tabs = lsh.Tables(lsh.bucket_keys(lsh.codes(Y, A, beta, w), L, k))
    cand, _ = tabs.candidates(lsh.bucket_keys(lsh.codes(Qf, A, beta, w), L, k))
    for q in range(20):
        assert len(cand[q]) == 300
        ids, d2 = lle.knn(Qf[q], Y, cand[q], K)
        full = ((Y.astype(np.float64) - Qf[q].astype(np.float64)) ** 2).sum(1)
        ref = np.argsort(full, kind="stable")[:K]
        assert np.array_equal(ids, ref)
        assert np.allclose(d2, full[ref], rtol=1e-12)


def test_recall_is_monotone_in_L_and_nested():
    rng = np.random.default_rng(8)
    D, k, w, K = 16, 4, 12.0, 4
    centers = rng.standard_normal((40, D))
    Y = (centers[rng.integers(0, 40, 3000)] + 0.2 * rng.standard_normal((3000, D))).astype(np.float32)
    Qf = (centers[rng.integers(0, 40, 60)] + 0.2 * rng.standard_normal((60, D))).astype(np.float32)
    true = [np.argsort(((Y.astype(np.float64) - q) ** 2).sum(1), kind="stable")[:K] for q in Qf]
    prev_c, prev_r = None, -1.0
    for L in (1, 2, 4, 8, 16, 32):
        A, beta = lsh.hash_params(6, L, k, D, w)
        tabs = lsh.Tables(lsh.bucket_keys(lsh.codes(Y, A, beta, w), L, k))
        cand, _ = tabs.candidates(lsh.bucket_keys(lsh.codes(Qf, A, beta, w), L, k))
        rec = np.mean([len(np.intersect1d(lle.knn(Qf[q], Y, cand[q], K)[0], true[q])) / K
                       for q in range(60)])
        if prev_c is not None:
            assert all(np.isin(p, c).all() for p, c in zip(prev_c, cand))
        assert rec >= prev_r
        prev_c, prev_r = cand, rec
    assert prev_r > 0.9


def test_t_of_l_candidates_pins():
    rng = np.random.default_rng(51)
    N, L, Q = 400, 6, 30
    keys = rng.integers(0, 5, (N, L)).astype(np.uint64)       # few, large buckets
    tables = lsh.Tables(keys)
    qkeys = rng.integers(0, 5, (Q, L)).astype(np.uint64)
    union, _ = tables.candidates(qkeys, 0)
    c1 = lsh.candidates_t(tables, qkeys, 1)
    assert all(np.array_equal(a, b) for a, b in zip(c1, union))
    prev = c1
    for t in range(2, L + 1):
        ct = lsh.candidates_t(tables, qkeys, t)
        assert all(np.all(np.isin(a, b)) for a, b in zip(ct, prev))      # nested
        prev = ct
    # t = L: the intersection of the L bins
    for q in range(Q):
        inter = np.arange(N)
        for l in range(L):
            inter = np.intersect1d(inter, np.nonzero(keys[:, l] == qkeys[q, l])[0])
        assert np.array_equal(prev[q], inter)
    # brute force at t = 3
    c3 = lsh.candidates_t(tables, qkeys, 3)
    for q in range(Q):
        hits = (keys == qkeys[q]).sum(axis=1)
        assert np.array_equal(c3[q], np.nonzero(hits >= 3)[0])
