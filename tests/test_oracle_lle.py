"""Pins of the oracle's LLE weights (Eq. LinSys with the trace regulariser),
synthesis (Eq. HR_Rec) and overlap blend (the quadratic overlap prior of
Section 4) against closed forms, a KKT solve and self-reproduction."""
import numpy as np
import pytest

import synthdata
from oracle import imaging, lle, pipeline


def test_weights_sum_to_one_and_small_cases():
    rng = np.random.default_rng(0)
    q = rng.standard_normal(25)
    Y = rng.standard_normal((6, 25))
    w = lle.lle_weights(q, Y, 1e-3)
    assert abs(w.sum() - 1.0) < 1e-12
    assert np.array_equal(lle.lle_weights(q, Y[:1], 1e-3), np.array([1.0]))
    # K = 2 closed form: w1 = (G22 + e - G12) / (G11 + G22 + 2e - 2 G12), e = lam tr G
    lam = 1e-3
    Z = q[None] - Y[:2]
    G = Z @ Z.T
    e = lam * np.trace(G)
    w1 = (G[1, 1] + e - G[0, 1]) / (G[0, 0] + G[1, 1] + 2 * e - 2 * G[0, 1])
    assert np.allclose(lle.lle_weights(q, Y[:2], lam), [w1, 1 - w1], rtol=0, atol=1e-13)


def test_weights_equal_kkt_solution_and_invariances():
    rng = np.random.default_rng(1)
    q = rng.standard_normal(100)
    Y = q[None] + 0.3 * rng.standard_normal((8, 100))
    lam = 1e-3
    w = lle.lle_weights(q, Y, lam)
    # KKT system of min w^T A w s.t. 1^T w = 1
    Z = q[None] - Y
    A = Z @ Z.T + lam * np.trace(Z @ Z.T) * np.eye(8)
    kkt = np.block([[2 * A, np.ones((8, 1))], [np.ones((1, 8)), np.zeros((1, 1))]])
    sol = np.linalg.solve(kkt, np.r_[np.zeros(8), 1.0])
    assert np.allclose(w, sol[:8], rtol=0, atol=1e-12)
    perm = rng.permutation(8)
    assert np.allclose(lle.lle_weights(q, Y[perm], lam), w[perm], atol=1e-12)
    shift = rng.standard_normal(100)
    assert np.allclose(lle.lle_weights(q + shift, Y + shift[None], lam), w, atol=1e-12)


def test_affine_combination_is_recovered_as_lambda_vanishes():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((5, 30))
    c = np.array([0.4, 0.3, -0.2, 0.25, 0.25])
    q = c @ Y
    assert np.allclose(lle.lle_weights(q, Y, 1e-12), c, atol=1e-8)


def test_degenerate_weights():
    q = np.ones(10)
    assert np.array_equal(lle.lle_weights(q, np.ones((3, 10)), 1e-3), np.full(3, 1 / 3))
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((4, 10))
    assert np.allclose(lle.lle_weights(q, Y, 1e9), np.full(4, 0.25), atol=1e-8)


def test_blend_is_least_squares_minimiser_and_counts():
    rng = np.random.default_rng(4)
    h, w, s = 9, 8, 2
    lr = rng.random((h, w)).astype(np.float32)
    pos = imaging.all_positions(h, w)
    valid = rng.random(len(pos)) > 0.2
    patches = [rng.random(100) for _ in range(len(pos))]
    out, cnt = lle.blend(patches, pos, valid, s, lr)
    # closed-form coverage when every patch is valid
    _, cnt_all = lle.blend(patches, pos, np.ones(len(pos), bool), s, lr)
    for Y in range(s * h):
        ny = sum(1 for i in range(h - 4) if s * i <= Y < s * i + 10)
        for X in range(s * w):
            nx = sum(1 for j in range(w - 4) if s * j <= X < s * j + 10)
            assert cnt_all[Y, X] == ny * nx
    # least squares: minimise sum_q ||R_q I - x_q||^2 over the covered pixels
    H, W = s * h, s * w
    rows, rhs = [], []
    for q in np.nonzero(valid)[0]:
        y0, x0 = s * pos[q]
        for a in range(10):
            for b in range(10):
                r = np.zeros(H * W)
                r[(y0 + a) * W + x0 + b] = 1.0
                rows.append(r)
                rhs.append(patches[q][a * 10 + b])
    Amat = np.array(rows)
    cov = cnt.ravel() > 0
    sol = np.linalg.lstsq(Amat[:, cov], np.array(rhs), rcond=None)[0]
    assert np.allclose(out.ravel()[cov], sol, atol=1e-12)
    bic = imaging.bicubic_up(lr, s)
    assert np.array_equal(out[cnt == 0], bic[cnt == 0])


def test_constant_patches_give_constant_image():
    h, w = 10, 11
    pos = imaging.all_positions(h, w)
    out, _ = lle.blend([np.full(100, 0.3)] * len(pos), pos, np.ones(len(pos), bool), 2,
                       np.zeros((h, w), np.float32))
    assert np.abs(out - 0.3).max() < 1e-15


@pytest.mark.parametrize("mode", [0, 1])
def test_full_image_self_reproduction(mode):
    """A dictionary holding every patch pair of (HR, degraded HR): each query
    patch of the degraded HR finds itself at distance 0 and K = 1
    reconstructs its own HR patch, so the blend returns HR (up to the fp32
    rounding of the stored residuals). The paper adds part of the test image
    to the training set for the same effect (Section 5.1)."""
    hr = synthdata.fractal_voronoi_image(40, 48, 48)
    lr = imaging.degrade(hr, 2)
    pos = np.concatenate([np.zeros((len(imaging.all_positions(24, 24)), 1), np.int64),
                          imaging.all_positions(24, 24)], axis=1)
    pre = pipeline.prepare(hr[None], pos, 2, mode, L=4, k=6, w=4.0, seed=7)
    qr = pipeline.query(pre, lr, K=1, lam=1e-3)
    # own patch is a candidate and at distance zero
    for q in range(len(pos)):
        assert q in set(qr.cand[q].tolist())
    assert np.all(qr.d2[:, 0] == 0.0)
    out, cnt = pipeline.reconstruct(qr, lr, 2)
    assert cnt.min() > 0
    assert np.abs(out - hr.astype(np.float64)).max() < 1e-6


def test_l1_distance_pins():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(41)
    X = rng.standard_normal((300, 100)).astype(np.float32)
    q = rng.standard_normal(100).astype(np.float32)
    cand = np.arange(0, 300, 3)
    d = lle.l1dist(q, X, cand)
    ref = cdist(q[None].astype(np.float64), X[cand].astype(np.float64), "cityblock")[0]
    assert np.allclose(d, ref, rtol=1e-13, atol=0)
    # integer-valued features: every partial sum exact, so any order agrees exactly
    Xi = rng.integers(-50, 50, (40, 25)).astype(np.float32)
    qi = rng.integers(-50, 50, 25).astype(np.float32)
    assert np.array_equal(lle.l1dist(qi, Xi, np.arange(40)), np.abs(Xi - qi).sum(axis=1).astype(np.float64))
    # l1 >= l2, and the l1 distance ignores the order of the coordinates
    l2 = np.sqrt(((X[cand].astype(np.float64) - q) ** 2).sum(axis=1))
    assert np.all(d >= l2 * (1 - 1e-12))
    perm = rng.permutation(100)
    assert np.allclose(lle.l1dist(q[perm], X[:, perm], cand), d, rtol=1e-13)


def test_knn_l1_brute_force_and_ties():
    rng = np.random.default_rng(42)
    X = rng.integers(0, 4, (60, 6)).astype(np.float32)       # many ties
    q = rng.integers(0, 4, 6).astype(np.float32)
    cand = np.sort(rng.choice(60, 35, replace=False))
    ids, d = lle.knn_l1(q, X, cand, 7)
    ref = sorted((float(np.abs(X[i] - q).sum()), int(i)) for i in cand)[:7]
    assert [int(i) for i in ids] == [i for _, i in ref]
    assert np.array_equal(d, np.array([v for v, _ in ref]))
    # a dictionary row queried against itself comes first at distance 0
    ids0, d0 = lle.knn_l1(X[cand[5]], X, cand, 3)
    assert d0[0] == 0.0 and (ids0[0] == cand[5] or np.array_equal(X[ids0[0]], X[cand[5]]))
    # fewer candidates than K: all of them
    assert len(lle.knn_l1(q, X, cand[:4], 7)[0]) == 4


@pytest.mark.parametrize("K", [2, 5, 8])
def test_synthesis_of_an_affine_combination(K):
    """Eq. LinSys then Eq. HR_Rec with K > 1: a query feature that is an
    affine combination sum_m c_m y_m (sum c = 1) of its neighbours, whose HR
    residuals follow the same combination, is synthesised as
    mu_q + sum_m c_m r_m as lambda -> 0 (the weights recover c and the HR
    patch is built with them). A dropped mean, a transposed weight/residual
    product or weights that are not renormalised fail it."""
    rng = np.random.default_rng(50 + K)
    Y = rng.standard_normal((K, 100))
    R = rng.standard_normal((K, 100))
    c = rng.uniform(-0.5, 1.0, K)
    c /= c.sum()
    q = c @ Y
    w = lle.lle_weights(q, Y, 1e-13)
    assert np.abs(w - c).max() < 1e-7
    mu = 0.37
    x = lle.synthesize(mu, w, R)
    assert x.shape == (100,)
    assert np.abs(x - (mu + c @ R)).max() < 1e-6
    # a larger lambda pulls the weights towards uniform; the patch follows them
    w2 = lle.lle_weights(q, Y, 0.5)
    assert np.abs(w2 - c).max() > 1e-3
    assert np.abs(lle.synthesize(mu, w2, R) - (mu + w2 @ R)).max() < 1e-12


def test_all_matches_equals_k_nearest_when_every_set_is_small():
    """LLE over all M matches (Eq. LinSys with m = 1..M): when no patch has
    more than K candidates the K nearest are all of them, and the weights
    (a permutation of the K-NN ones: the solve is equivariant under a
    reordering of the neighbours) and the image agree with the K-NN path."""
    wl = synthdata.WORKLOADS["tiny"]
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, 4, 12, 4.0,
                           wl.hash_seed)
    lr = wl.test_image()
    K = 400      # above the largest candidate set
    a = pipeline.query(pre, lr, K, wl.lam, cap=0)
    b = pipeline.query(pre, lr, K, wl.lam, cap=0, all_matches=True)
    assert max(len(c) for c in a.cand) < K and (a.m > 1).sum() > 100
    for q in np.nonzero(a.m > 0)[0]:
        order = np.argsort(a.ids[q, :a.m[q]])
        assert np.allclose(b.all_weights[q], a.weights[q, :a.m[q]][order], rtol=0, atol=1e-9)
    ha, _ = pipeline.reconstruct(a, lr, wl.scale)
    hb, _ = pipeline.reconstruct(b, lr, wl.scale)
    assert np.abs(ha - hb).max() < 1e-9


def test_all_matches_uses_every_candidate():
    """With the early stop at 24 and K = 5, the all-M weights of a patch are
    the LLE solve over its whole candidate list (checked against the KKT
    system of Eq. LinSys with the trace regulariser) and its HR patch the
    weighted sum of all M residuals."""
    wl = synthdata.WORKLOADS["tiny"]
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, 16.0,
                           wl.hash_seed)
    lr = wl.test_image()
    b = pipeline.query(pre, lr, 5, wl.lam, cap=24, all_matches=True)
    big = [q for q in range(len(b.cand)) if len(b.cand[q]) == 24][:5]
    assert len(big) == 5
    for q in big:
        Y = pre.dictionary.feat[b.cand[q]].astype(np.float64)
        Z = b.feat[q].astype(np.float64)[None] - Y
        G = Z @ Z.T
        A = G + wl.lam * np.trace(G) * np.eye(24)
        kkt = np.block([[2 * A, np.ones((24, 1))], [np.ones((1, 24)), np.zeros((1, 1))]])
        sol = np.linalg.solve(kkt, np.r_[np.zeros(24), 1.0])
        assert np.allclose(b.all_weights[q], sol[:24], rtol=0, atol=1e-8)
        R = pre.dictionary.resid[b.cand[q]].astype(np.float64)
        assert np.allclose(b.patches[q], b.mu[q] + sol[:24] @ R, rtol=0, atol=1e-7)
