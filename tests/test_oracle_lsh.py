"""Pins of the oracle's E2LSH and CKNS estimator.

Sec. "Random Projection": h(x) = floor((<x,g> + b)/4), g ~ N(0, I_d),
b ~ U(0,4), and the collision probability p(c) both as an integral over the
half-normal density and in closed form.  Sec. "Boosting the Probability":
p^K for K concatenated functions, 1-(1-p^K)^L over L tables.  Sec. "The CKNS
Algorithm": levels, 2^-i subsampling, importance weighting, unbiasedness.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synth


def _p_integral(c):
    # p(c) = int_0^4 (1/c) f(t/c) (1 - t/4) dt, f the density of |N(0,1)|
    f = lambda u: math.sqrt(2.0 / math.pi) * math.exp(-u * u / 2.0)
    val, _ = integrate.quad(lambda t: f(t / c) / c * (1.0 - t / 4.0), 0.0, 4.0, epsabs=1e-14, epsrel=1e-13)
    return val


@pytest.mark.parametrize("c", [0.05, 0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 8.0, 20.0])
def test_collision_closed_form_equals_integral(orc, c):
    assert orc.collision_probability(c) == pytest.approx(_p_integral(c), abs=1e-11)


def test_collision_shape(orc):
    cs = np.linspace(1e-3, 30, 400)
    ps = np.array([orc.collision_probability(c) for c in cs])
    assert orc.collision_probability(0.0) == 1.0
    assert ps[0] > 0.999
    assert np.all(np.diff(ps) < 0)
    assert np.all((ps > 0) & (ps <= 1))
    # boosting
    for c in (0.5, 1.0, 2.0, 4.0):
        p = orc.collision_probability(c)
        for K, L in [(1, 1), (8, 16), (6, 50)]:
            assert orc.boosted_probability(c, K, L) == pytest.approx(1 - (1 - p ** K) ** L, rel=1e-12)


@pytest.mark.parametrize("c", [0.5, 1.0, 2.0, 4.0])
def test_hash_collision_rate_matches_p(orc, c):
    """Two points at distance c hashed by many independent (g, b): the fraction
    of equal codes is p(c) within a 4-sigma binomial interval."""
    d, nproj = 6, 200_000
    rng = np.random.default_rng(int(c * 100))
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    x1 = rng.uniform(-3, 3, size=d)
    X = np.stack([x1, x1 + c * u]).astype(np.float32)
    c_eff = float(np.linalg.norm(X[1].astype(np.float64) - X[0].astype(np.float64)))
    G, b = synth.e2lsh_randomness(nproj, d, seed=99 + int(c * 10))
    codes, _ = orc.e2lsh_hash(X, G, b, K=1, L=nproj)
    rate = float(np.mean(codes[0, :, 0] == codes[1, :, 0]))
    p = orc.collision_probability(c_eff)
    assert abs(rate - p) < 4 * math.sqrt(p * (1 - p) / nproj)


def test_key_collision_rate_matches_boosting(orc):
    d, K, L, c = 5, 4, 30_000, 1.0
    X = np.array([[0.0] * d, [c] + [0.0] * (d - 1)], np.float32)
    G, b = synth.e2lsh_randomness(K * L, d, seed=5)
    _, keys = orc.e2lsh_hash(X, G, b, K=K, L=L)
    rate = float(np.mean(keys[0] == keys[1]))
    pk = orc.collision_probability(c) ** K
    assert abs(rate - pk) < 4 * math.sqrt(pk * (1 - pk) / L)


def test_hash_floor_and_definition(orc):
    # floor, not truncation, on negative projections
    X = np.array([[1.0]], np.float32)
    G = np.array([[-1.5]], np.float32)
    codes, _ = orc.e2lsh_hash(X, G, np.array([0.25]), K=1, L=1)
    assert codes[0, 0, 0] == -1
    # the origin lands in bucket 0 for every b in [0,4)
    codes, _ = orc.e2lsh_hash(np.zeros((1, 3), np.float32), np.ones((4, 3), np.float32),
                              np.array([0.0, 1.0, 3.999, 2.5]), K=2, L=2)
    assert np.all(codes == 0)
    # brute force in Python doubles (left-to-right sum of exact products)
    rng = np.random.default_rng(1)
    X = (rng.normal(size=(20, 9)) * 5).astype(np.float32)
    G, b = synth.e2lsh_randomness(12, 9, seed=2)
    codes, _ = orc.e2lsh_hash(X, G, b, K=3, L=4)
    for i in range(20):
        for p in range(12):
            s = 0.0
            for j in range(9):
                s += float(X[i, j]) * float(G[p, j])
            assert codes[i, p // 3, p % 3] == math.floor((s + float(b[p])) / 4.0)


def test_keys_identify_code_tuples(orc):
    rng = np.random.default_rng(4)
    X = rng.normal(size=(400, 3)).astype(np.float32) * 3
    G, b = synth.e2lsh_randomness(2 * 5, 3, seed=8)
    codes, keys = orc.e2lsh_hash(X, G, b, K=2, L=5)
    for l in range(5):
        tup = {}
        for i in range(400):
            t = tuple(codes[i, l])
            tup.setdefault(t, set()).add(int(keys[i, l]))
        assert all(len(v) == 1 for v in tup.values())          # equal codes -> equal key
        assert len({next(iter(v)) for v in tup.values()}) == len(tup)  # distinct codes -> distinct keys
        assert all(orc.bucket_key(l, codes[i, l]) == int(keys[i, l]) for i in range(0, 400, 37))
    # the table index enters the key
    assert orc.bucket_key(0, [1, 2]) != orc.bucket_key(1, [1, 2])


def test_counter_generator(orc):
    # SplitMix64: the c-th output of state s is mix(s + (c+1) gamma); check the
    # finaliser against its definition evaluated in Python integers.
    M = (1 << 64) - 1

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for z in [0, 1, 0xDEADBEEF, M, 0x9E3779B97F4A7C15]:
        assert orc.mix64(z) == mix(z)
    # uniform bits: the kept fraction of a mask is p within 4 sigma, and masks
    # of different (copy, level) are independent
    n = 200_000
    for i, p in [(1, 0.5), (3, 0.125), (6, 1 / 64)]:
        keep = orc.lsh_mask(123, 0, i, n, int(p * 2 ** 53))
        assert abs(keep.mean() - p) < 4 * math.sqrt(p * (1 - p) / n)
    k1 = orc.lsh_mask(123, 0, 1, n, 2 ** 52)
    k2 = orc.lsh_mask(123, 1, 1, n, 2 ** 52)
    both = np.mean(k1 & k2)
    assert abs(both - 0.25) < 4 * math.sqrt(0.25 * 0.75 / n)


def test_parameter_reading(orc):
    sh = orc.lsh_derive(100_000, 0.01, eps=0.5)
    assert (sh["J"], sh["L"], sh["K"], sh["K1"]) == (17, 17, 9, 67)
    assert sh["p"][1] == 0.5 and sh["p"][17] == 2.0 ** -17
    assert sh["T"][3] == pytest.approx(3 * math.log(2) / 0.01, rel=1e-15)
    # K is the largest with recovery >= 1 - eps/4 at unit scaled distance
    K, L = sh["K"], sh["L"]
    assert orc.boosted_probability(1.0, K, L) >= 0.875 > orc.boosted_probability(1.0, K + 1, L)
    # the paper's fine-grained constructor example: min_mu=1e-4, K1=10, K2_constant=5, p_offset=1
    sh = orc.lsh_derive(100_000, 1.0, eps=0.5, min_mu=1e-4, k1=10, k2_constant=5, p_offset=1)
    assert (sh["J"], sh["L"], sh["K1"]) == (14, 5, 10)
    assert sh["p"][1] == pytest.approx(min(1.0, 0.5 / 10.0) / 2)
    with pytest.raises(ValueError):
        orc.lsh_derive(10, 1.0, eps=1.5)


def _lsh_inputs(orc, n, d, a, seed, **kw):
    sh = orc.lsh_derive(n, a, **kw)
    npj = sh["K1"] * sh["J"] * sh["L"] * sh["K"]
    G0, B = synth.e2lsh_randomness(npj, d, seed)
    return sh, G0, B


def _truncated_exact(X, Q, a, TJ):
    D = ((Q.astype(np.float64)[:, None, :] - X.astype(np.float64)[None, :, :]) ** 2).sum(-1)
    return np.where(D < TJ, np.exp(-a * D), 0.0).sum(1)


def test_lsh_degenerate_case_is_truncated_exact(orc):
    """p_i = 1, zero projections, 2^i weights: every point shares q's bucket in
    every table, dedupe keeps the first table, each point lands in exactly one
    level, so every copy equals sum_{D < T_J} exp(-aD)."""
    X, Q, _ = synth.config_points(1, n=200, m=12)
    a = 0.05
    kw = dict(eps=0.5, k1=3, flags=orc.FLAG_LITERAL | orc.FLAG_ALL_SAMPLED)
    sh, G0, B = _lsh_inputs(orc, 200, 10, a, 17, **kw)
    S, st = orc.lsh_kde(X, Q, a, np.zeros_like(G0), B, seed=1, return_stats=True, **kw)
    ref = _truncated_exact(X, Q, a, sh["T"][-1])
    assert np.allclose(S, ref, rtol=1e-12)
    assert np.allclose(st["S_copies"], ref[:, None], rtol=1e-12)
    # every point was examined in every table of every level of every copy
    assert np.all(st["n_cand"] == 200 * sh["J"] * sh["L"] * 3)


def test_lsh_unbiased(orc):
    """Mean over independent copies of the reweighted estimator equals the
    truncated exact sum within 4 standard errors (Sec. "The CKNS Algorithm":
    the estimate is unbiased; here, unbiased over masks and hash draws)."""
    rng = np.random.default_rng(5)
    n, d, a = 40, 3, 0.4
    X = rng.normal(size=(n, d)).astype(np.float32) * 1.5
    Q = rng.normal(size=(4, d)).astype(np.float32)
    kw = dict(eps=0.5, k1=3000, k2_constant=3)
    sh, G0, B = _lsh_inputs(orc, n, d, a, 21, **kw)
    S, st = orc.lsh_kde(X, Q, a, G0, B, seed=77, return_stats=True, **kw)
    ref = _truncated_exact(X, Q, a, sh["T"][-1])
    Sc = st["S_copies"]
    se = Sc.std(axis=1, ddof=1) / math.sqrt(Sc.shape[1])
    assert np.all(np.abs(Sc.mean(axis=1) - ref) < 4 * se + 1e-12)
    # the literal 2^i weighting under-counts whatever the tables miss
    S_lit, st_lit = orc.lsh_kde(X, Q, a, G0, B, seed=77, return_stats=True, flags=orc.FLAG_LITERAL, **kw)
    assert np.all(S_lit <= ref + 4 * st_lit["S_copies"].std(axis=1) / math.sqrt(Sc.shape[1]))


@pytest.mark.slow
def test_lsh_relative_error_rate(orc):
    """With the default parameters, at least 90 % of queries with S >= n mu_min
    are within (1 +- eps) of the exact sum."""
    X, Q, _ = synth.config_points(2, n=3000, m=60)
    a, eps = 0.01, 0.5
    sh, G0, B = _lsh_inputs(orc, 3000, 64, a, 3002, eps=eps)
    S = orc.lsh_kde(X, Q, a, G0, B, seed=3002, eps=eps)
    ex = orc.kde_exact(X, Q, a)
    ok = ex >= 1.0
    rel = np.abs(S[ok] - ex[ok]) / ex[ok]
    assert ok.sum() > 30
    assert np.mean(rel <= eps) >= 0.9
