"""Pins of the random-sampling KDE oracle (the baseline estimator of Sec.
"Kernel Density Estimation": K(q) from a uniformly random sample of the data)
against what probability fixes: unbiasedness, uniform indices, exact special
cases, and the Chernoff sample size holding in practice."""
import math

import numpy as np
import pytest

import oracle


def test_unbiased_over_seeds():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(40, 3)).astype(np.float32)
    Q = rng.normal(size=(3, 3)).astype(np.float32)
    a = 0.7
    exact = oracle.kde_exact(X, Q, a)
    est = np.array([oracle.kde_random_sample(X, Q, a, 25, seed)[0] for seed in range(3000)])
    mean, sd = est.mean(0), est.std(0)
    assert np.all(np.abs(mean - exact) < 5 * sd / math.sqrt(len(est)))


def test_indices_uniform_and_in_range():
    X = np.zeros((7, 1), dtype=np.float32)
    _, idx = oracle.kde_random_sample(X, X[:1], 1.0, 210_000, 3)
    assert idx.min() >= 0 and idx.max() <= 6
    cnt = np.bincount(idx, minlength=7)
    p = 1 / 7
    assert np.all(np.abs(cnt - 30_000) < 5 * math.sqrt(210_000 * p * (1 - p)))


def test_identical_points_and_single_point():
    x = np.array([[0.5, -1.0, 2.0]], dtype=np.float32)
    q = np.array([[0.0, 0.0, 1.0]], dtype=np.float32)
    k = math.exp(-0.3 * (0.25 + 1.0 + 1.0))
    S, _ = oracle.kde_random_sample(np.repeat(x, 100, axis=0), q, 0.3, 37, 9)
    assert S[0] == pytest.approx(100 * k, rel=1e-14)
    S1, idx = oracle.kde_random_sample(x, q, 0.3, 5, 9)
    assert np.all(idx == 0) and S1[0] == pytest.approx(k, rel=1e-15)


def test_chernoff_sample_size_holds():
    # queries drawn from the data, densities well above mu: with the sample
    # size for (eps, mu, m, delta) no query may miss (1 +- eps), across seeds
    rng = np.random.default_rng(4)
    X = rng.normal(size=(2000, 2)).astype(np.float32)
    Q = X[:50]
    a = 1.0
    exact = oracle.kde_exact(X, Q, a)
    mu = float((exact / len(X)).min())
    eps, delta = 0.2, 0.05
    s = oracle.rs_sample_size(eps, mu, len(Q), delta)
    assert s >= 3 * math.log(2 * len(Q) / delta) / (eps * eps * mu)
    fails = 0
    for seed in range(20):
        est, _ = oracle.kde_random_sample(X, Q, a, s, seed)
        fails += int(np.sum(np.abs(est - exact) > eps * exact))
    # expected failures per seed are at most delta in total; 20 seeds -> <= 1
    assert fails <= 1
    # and a sample 100x smaller does miss
    small = 0
    for seed in range(20):
        est, _ = oracle.kde_random_sample(X, Q, a, max(1, s // 100), seed)
        small += int(np.sum(np.abs(est - exact) > eps * exact))
    assert small > 0
