"""Pins of the KDE-tree edge-sampler oracle (Sec. "The MS Algorithm": edges
drawn with probability close to eq. (sampling_prob), the kernel sums coming
from a KDE algorithm used as a black box, here random sampling per tree node).

What fixes the oracle independently of its own code:
- where every node estimate is exact (children of at most t rows, or a child
  of identical points not holding the query row) the descent telescopes to
  P_i(j) = k_ij / rest_i, rest_i = sum_{j != i} k_ij: chi-square against the
  brute-force kernel row;
- the random-sampling estimator is unbiased for rest_i (mean over seeds);
- with every kernel value 0 the descent follows the row-count rule and the
  leaf picks the floor(u m)-th row other than i (brute force of the rule);
- the weight is 1/(s (1/rest_i + 1/rest_j)) with exact degrees when
  t_deg >= n (brute force), which gives every pair expected weight k_ij;
- no draw returns its own row; every index is in range."""
import math

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle


def _kernel_rows(X, a):
    X = X.astype(np.float64)
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    K = np.exp(-a * D)
    np.fill_diagonal(K, 0.0)
    return K


def _chi2_rows(X, a, s, t, rows, seed):
    n = len(X)
    K = _kernel_rows(X, a)
    src, dst, w, deg, _ = oracle.simgraph_tree(X, a, s, t, n, seed)
    assert np.array_equal(src, np.repeat(np.arange(n), s))
    for i in rows:
        got = np.bincount(dst[i * s:(i + 1) * s], minlength=n).astype(np.float64)
        p = K[i] / K[i].sum()
        assert got[i] == 0
        keep = np.arange(n) != i
        res = chisquare(got[keep], p[keep] * s)
        assert res.pvalue > 1e-4, (i, res)


@pytest.mark.parametrize("n", [64, 40])
def test_exact_nodes_give_sampling_prob(n):
    # t = 32: the two children of the root are single leaves, so every
    # estimate is the exact sum and P_i(j) = k_ij / rest_i
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 2)).astype(np.float32)
    _chi2_rows(X, 0.5, 20000, 32, rows=[0, 5, n - 1, n // 2], seed=3)


def test_sampled_node_of_identical_points():
    # n = 96: leaves [0,32) [32,64) [64,96), root children [0,64) (64 rows > t,
    # sampled) and [64,96).  Rows 0..63 are one point p, so for a query row i
    # >= 64 the sampled estimate of [0,64) is exactly 64 k(x_i, p) whatever
    # rows it draws: the descent is exact again and P_i(j) = k_ij / rest_i.
    # A wrong scale P/t or a wrong node range changes the law.
    rng = np.random.default_rng(9)
    X = np.zeros((96, 2), dtype=np.float32)
    X[:64] = [0.2, -0.1]
    X[64:] = (rng.normal(size=(32, 2)) * 0.7 + 0.8).astype(np.float32)
    s = 30000
    K = _kernel_rows(X, 1.0)
    src, dst, w, deg, _ = oracle.simgraph_tree(X, 1.0, s, 32, 96, 11)
    for i in [64, 70, 95]:
        got = np.bincount(dst[i * s:(i + 1) * s], minlength=96).astype(np.float64)
        p = K[i] / K[i].sum()
        # rows 0..63 are equally likely: two pooled bins, then rows 64.. apart from i
        g = np.concatenate([[got[:32].sum(), got[32:64].sum()], np.delete(got[64:], i - 64)])
        e = np.concatenate([[p[:32].sum(), p[32:64].sum()], np.delete(p[64:], i - 64)]) * s
        res = chisquare(g, e)
        assert res.pvalue > 1e-4, (i, res)


def test_degree_estimator_unbiased():
    # rest_i from t_deg = 10 uniform samples of the 200 rows (own row counted
    # as 0), scaled by n / t_deg: its mean over seeds is sum_{j != i} k_ij
    rng = np.random.default_rng(2)
    X = rng.normal(size=(200, 3)).astype(np.float32)
    K = _kernel_rows(X, 0.4)
    exact = K.sum(1)
    est = np.array([oracle.simgraph_tree(X, 0.4, 1, 8, 10, seed)[3] - 1.0 for seed in range(1500)])
    mean, se = est.mean(0), est.std(0) / math.sqrt(len(est))
    z = np.abs(mean - exact) / se
    assert np.all(z < 5.0), z.max()
    # and t_deg >= n gives the exact sum
    _, _, _, deg, _ = oracle.simgraph_tree(X, 0.4, 1, 8, 200, 0)
    np.testing.assert_allclose(deg - 1.0, exact, rtol=1e-13)


def test_weights_with_exact_degrees():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(150, 4)).astype(np.float32)
    s = 8
    K = _kernel_rows(X, 0.3)
    rest = K.sum(1)
    src, dst, w, deg, _ = oracle.simgraph_tree(X, 0.3, s, 4, 150, 21)
    want = 1.0 / (s * (1.0 / rest[src] + 1.0 / rest[dst]))
    np.testing.assert_allclose(w, want, rtol=1e-13)


def test_expected_pair_weight_is_kernel_value():
    # exact law (n = 64, t = 32, exact degrees): every pair's expected sampled
    # weight is s (P_i(j) + P_j(i)) w_ij = k_ij; mean over seeds
    rng = np.random.default_rng(8)
    X = rng.normal(size=(64, 2)).astype(np.float32)
    K = _kernel_rows(X, 0.5)
    s, seeds = 6, 600
    acc = np.zeros((64, 64))
    for seed in range(seeds):
        src, dst, w, _, _ = oracle.simgraph_tree(X, 0.5, s, 32, 64, 1000 + seed)
        np.add.at(acc, (np.minimum(src, dst), np.maximum(src, dst)), w)
    iu = np.triu_indices(64, 1)
    mean = acc[iu] / seeds
    big = K[iu] > 0.2  # pairs sampled often enough for a tight mean
    rel = np.abs(mean[big] - K[iu][big]) / K[iu][big]
    assert np.median(rel) < 0.1 and rel.max() < 0.5, (np.median(rel), rel.max())


def test_zero_kernel_rule():
    # points 100 apart with a = 1: every kernel value underflows to 0, so each
    # level goes to the child with more rows other than i (left on a tie) and
    # the leaf takes the floor(u m)-th row other than i, u = U(i, r, h)
    n, s = 75, 5
    X = (np.arange(n, dtype=np.float32)[:, None] * np.float32(100.0)).repeat(2, axis=1)
    src, dst, w, deg, _ = oracle.simgraph_tree(X, 1.0, s, 4, 10, 7)
    assert np.all(w == 0.0) and np.all(deg == 1.0)
    nb = (n + 31) // 32
    h = max(0, math.ceil(math.log2(nb)))
    for i in range(n):
        for r in range(s):
            k = 0
            for lev in range(h):
                span = 32 << (h - lev - 1)
                a_lo, a_hi = min(n, 2 * k * span), min(n, (2 * k + 1) * span)
                b_lo, b_hi = a_hi, min(n, (2 * k + 2) * span)
                m_a = (a_hi - a_lo) - (1 if a_lo <= i < a_hi else 0)
                m_b = (b_hi - b_lo) - (1 if b_lo <= i < b_hi else 0)
                k = 2 * k if m_a >= m_b else 2 * k + 1
            lo, hi = min(n, 32 * k), min(n, 32 * (k + 1))
            rows = [j for j in range(lo, hi) if j != i]
            u = (oracle.counter_bits(7, 0x5452554E, i, r, h) >> 11) * 2.0 ** -53
            assert dst[i * s + r] == rows[int(u * len(rows))]


@pytest.mark.parametrize("n", [2, 33, 97, 1000])
def test_draws_valid(n):
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 3)).astype(np.float32)
    s = 7
    src, dst, w, deg, mg = oracle.simgraph_tree(X, 0.8, s, 5, 20, 4)
    assert np.array_equal(src, np.repeat(np.arange(n), s))
    assert np.all(dst != src) and dst.min() >= 0 and dst.max() < n
    assert np.all(w >= 0.0) and np.all(deg >= 1.0) and np.all((mg >= 0) & (mg <= 1))
