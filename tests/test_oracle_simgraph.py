"""Pins of the oracle's similarity-graph edge sampler (Sec. "The MS Algorithm":
sample edge (i,j) with probability proportional to w/deg(i) + w/deg(j), deg
the kernel degree in the fully connected graph)."""
import math

import numpy as np
from scipy import stats


def _kmat(X, a):
    X = X.astype(np.float64)
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-a * D)


def test_draw_distribution_chi2(orc):
    rng = np.random.default_rng(2)
    n, s, a = 12, 6000, 0.3
    X = rng.normal(size=(n, 3)).astype(np.float32)
    src, dst, w, deg = orc.simgraph_exact(X, a, s, seed=9)
    Kf = _kmat(X, a)
    assert np.allclose(deg, Kf.sum(1), rtol=1e-13)
    assert np.all(src != dst) and np.all(w > 0)
    assert np.all(src == np.repeat(np.arange(n), s))
    for i in range(n):
        pr = Kf[i].copy()
        pr[i] = 0.0
        pr /= pr.sum()
        obs = np.bincount(dst[src == i], minlength=n)
        keep = pr > 0
        chi = stats.chisquare(obs[keep], pr[keep] * s)
        assert chi.pvalue > 1e-4


def test_expected_weights_reproduce_full_graph(orc):
    """E[sum of sampled weights between i and j] = k_ij: the sampled graph is
    an unbiased sparsifier of the fully connected one (self-loops excluded)."""
    rng = np.random.default_rng(3)
    n, s, a = 8, 20000, 0.5
    X = rng.normal(size=(n, 2)).astype(np.float32)
    src, dst, w, deg = orc.simgraph_exact(X, a, s, seed=4)
    Kf = _kmat(X, a)
    tot = np.zeros((n, n))
    np.add.at(tot, (np.minimum(src, dst), np.maximum(src, dst)), w)
    for i in range(n):
        for j in range(i + 1, n):
            # per-draw weight is constant for a pair, so the count is binomial
            pij = s * (Kf[i, j] / (deg[i] - 1) + Kf[i, j] / (deg[j] - 1))
            wpair = 1.0 / (s * (1 / (deg[i] - 1) + 1 / (deg[j] - 1)))
            sd = wpair * math.sqrt(pij)
            assert abs(tot[i, j] - Kf[i, j]) < 5 * sd + 1e-12
    # incident weight of each node is deg(i) - 1 in expectation
    inc = np.bincount(src, weights=w, minlength=n) + np.bincount(dst, weights=w, minlength=n)
    assert np.allclose(inc, deg - 1, rtol=0.1)


def test_uniform_draws(orc):
    u = np.array([orc.draw_uniform(5, i, r) for i in range(200) for r in range(50)])
    assert np.all((u >= 0) & (u < 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-4
