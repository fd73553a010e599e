"""Pins of the oracle's exact kernel density against facts the paper and the
mathematics fix (Sec. "Kernel Density Estimation": K(q) = (1/n) sum_i k(||q-x_i||)
with the Gaussian kernel k(x) = exp(-a x^2); the oracle returns the sum S = n K).
"""
import math

import numpy as np
import pytest

import synth


def test_hand_values(orc):
    # one point: d=1, x=0, q=1, a=0.5  ->  e^{-1/2}
    S = orc.kde_exact(np.zeros((1, 1)), np.ones((1, 1)), 0.5)
    assert S[0] == pytest.approx(math.exp(-0.5), rel=1e-15)
    # two points at distance 1 and 2 from q in d=2 -> e^{-a} + e^{-4a}
    X = np.array([[1.0, 0.0], [0.0, 2.0]], np.float32)
    S = orc.kde_exact(X, np.zeros((1, 2)), 0.3)
    assert S[0] == pytest.approx(math.exp(-0.3) + math.exp(-1.2), rel=1e-15)
    # the single-pair kernel of the user's guide
    assert orc.gaussian_kernel(1.0, [0, 0, 0], [1, 1, 1]) == pytest.approx(math.exp(-3.0), rel=1e-15)


def test_brute_force_tiny(orc):
    rng = np.random.default_rng(7)
    for n, m, d in [(1, 1, 1), (3, 5, 2), (8, 8, 7), (5, 2, 16)]:
        X = rng.normal(size=(n, d)).astype(np.float32)
        Q = rng.normal(size=(m, d)).astype(np.float32)
        a = float(rng.uniform(0.05, 2.0))
        S = orc.kde_exact(X, Q, a)
        for qi in range(m):
            ref = 0.0
            for i in range(n):
                dd = 0.0
                for j in range(d):
                    t = float(Q[qi, j]) - float(X[i, j])
                    dd += t * t
                ref += math.exp(-a * dd)
            assert S[qi] == pytest.approx(ref, rel=1e-13)


def test_all_points_at_query_gives_n_exactly(orc):
    q = np.array([[0.25, -1.5, 3.0]], np.float32)
    for n in (1, 7, 1000):
        X = np.repeat(q, n, axis=0)
        assert orc.kde_exact(X, q, 0.7)[0] == float(n)


def test_invariants(orc):
    X, Q, _ = synth.config_points(1, n=300, m=40)
    a_vals = [0.01, 0.1, 0.5, 2.0]
    Ss = [orc.kde_exact(X, Q, a) for a in a_vals]
    for S in Ss:
        assert np.all(S >= 0) and np.all(S <= X.shape[0])
    for lo, hi in zip(Ss, Ss[1:]):
        assert np.all(hi <= lo)  # non-increasing in a
    # a -> 0 gives n
    assert np.allclose(orc.kde_exact(X, Q, 1e-12), X.shape[0], rtol=1e-9)
    # permutation of X
    perm = np.random.default_rng(3).permutation(X.shape[0])
    assert np.allclose(orc.kde_exact(X[perm], Q, 0.5), Ss[2], rtol=1e-13)
    # common translation of X and Q; coordinates on a 2^-10 grid so that the
    # shifted fp32 values are exact
    Xg = (np.round(X * 1024) / 1024).astype(np.float32)
    Qg = (np.round(Q * 1024) / 1024).astype(np.float32)
    sh = np.float32(8.0)
    assert np.allclose(orc.kde_exact(Xg + sh, Qg + sh, 0.5), orc.kde_exact(Xg, Qg, 0.5), rtol=1e-12)


def test_against_independent_library_route(orc):
    from scipy.spatial.distance import cdist
    from scipy.special import logsumexp
    X, Q, _ = synth.config_points(2, n=500, m=30)
    a = 0.05
    D = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    ref = np.exp(logsumexp(-a * D, axis=1))
    assert np.allclose(orc.kde_exact(X, Q, a), ref, rtol=1e-11)


def test_gaussian_closed_form(orc):
    # x ~ N(mu, s^2 I_d):  E exp(-a||q-x||^2) = (1+2as^2)^{-d/2} exp(-a||q-mu||^2/(1+2as^2))
    d, s, a, n = 4, 0.8, 0.3, 200_000
    rng = np.random.default_rng(11)
    mu = rng.uniform(-1, 1, size=d)
    X = (mu + s * rng.standard_normal((n, d))).astype(np.float32)
    Q = (mu + rng.uniform(-1.5, 1.5, size=(5, d))).astype(np.float32)
    S = orc.kde_exact(X, Q, a, nthreads=4)
    for qi in range(Q.shape[0]):
        q = Q[qi].astype(np.float64)
        f = 1.0 + 2.0 * a * s * s
        expect = f ** (-d / 2) * math.exp(-a * float(np.sum((q - mu) ** 2)) / f)
        terms = np.exp(-a * np.sum((X.astype(np.float64) - q) ** 2, axis=1))
        se = terms.std() / math.sqrt(n)
        assert abs(S[qi] / n - expect) < 5 * se


def test_underflow_returns_log(orc):
    X = np.zeros((3, 2), np.float32)
    Q = np.array([[100.0, 0.0]], np.float32)
    S, lg = orc.kde_exact(X, Q, 1.0, return_log=True)
    assert S[0] == 0.0
    assert lg[0] == pytest.approx(-1e4 + math.log(3.0), rel=1e-15)
    # mixed magnitudes: log-sum-exp keeps the tiny tail exactly
    X = np.array([[0.0], [30.0]], np.float32)
    S, lg = orc.kde_exact(X, np.zeros((1, 1), np.float32), 1.0, return_log=True)
    assert lg[0] == pytest.approx(math.log1p(math.exp(-900.0)), abs=1e-300)
