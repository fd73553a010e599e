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


def test_lsh_mode_degenerate_equals_exact_rows(orc):
    """With every point sampled, zero projections and 2^i weights the CKNS
    terms of node i are exactly k_ij for D < T_J, so the LSH-mode degrees equal
    the exact ones (all pairs within T_J here) and the draws follow k_ij."""
    import synth
    rng = np.random.default_rng(8)
    n, d, a, s = 14, 2, 0.2, 64
    X = (0.6 * rng.normal(size=(n, d))).astype(np.float32)
    kw = dict(eps=0.5, k1=1, k2_constant=2, flags=orc.FLAG_LITERAL | orc.FLAG_ALL_SAMPLED)
    sh = orc.lsh_derive(n, a, **kw)
    Kf = _kmat(X, a)
    D = -np.log(Kf) / a
    assert D.max() < sh["T"][-1]
    npj = sh["K1"] * sh["J"] * sh["L"] * sh["K"]
    G0, B = synth.e2lsh_randomness(npj, d, 3)
    src, dst, w, deg, mg = orc.simgraph_lsh(X, a, s, 21, np.zeros_like(G0), B, lsh_seed=4, **kw)
    assert np.allclose(deg, Kf.sum(1), rtol=1e-12)
    _, _, w_ex, deg_ex = orc.simgraph_exact(X, a, s, seed=21)
    assert np.allclose(deg, deg_ex, rtol=1e-12)
    assert np.all(src != dst) and np.all(w > 0)
    # chi-square of all draws pooled over nodes against k_ij / rest_i
    obs = np.zeros((n, n))
    np.add.at(obs, (src, dst), 1)
    exp_ = (Kf - np.eye(n)) / (Kf.sum(1, keepdims=True) - 1) * s
    keep = exp_ > 0
    chi = stats.chisquare(obs[keep], exp_[keep] * obs[keep].sum() / exp_[keep].sum())
    assert chi.pvalue > 1e-4


def test_lsh_mode_weights_and_margins(orc):
    import synth
    X, _, _ = synth.config_points(1, n=300, m=1)
    kw = dict(eps=0.5, k1=2, k2_constant=4)
    sh = orc.lsh_derive(300, 0.05, **kw)
    npj = sh["K1"] * sh["J"] * sh["L"] * sh["K"]
    G0, B = synth.e2lsh_randomness(npj, 10, 9)
    src, dst, w, deg, mg = orc.simgraph_lsh(X, 0.05, 6, 5, G0, B, lsh_seed=6, **kw)
    ok = dst >= 0
    assert ok.mean() > 0.9
    rest = deg - 1
    assert np.allclose(w[ok], 1 / (6 * (1 / rest[src[ok]] + 1 / rest[dst[ok]])), rtol=1e-14)
    assert np.all(mg[ok] >= 0) and np.all(src[ok] != dst[ok])
