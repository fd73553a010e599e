"""Pins of the oracle's E2LSH near-neighbour listing (the E2LSH class's
get_near_neighbours; Sec. "Random Projection", "Boosting the Probability")."""
import numpy as np

import synth


def test_matches_bucket_definition_by_brute_force(orc):
    """Tiny case: every listed point shares a key with the query in its
    listed table and in no earlier one; every colliding point is listed."""
    rng = np.random.default_rng(11)
    X = rng.normal(size=(60, 5)).astype(np.float32)
    Q = (X[:7] + 0.3 * rng.normal(size=(7, 5))).astype(np.float32)
    K, L = 2, 5
    G, b = synth.e2lsh_randomness(K * L, 5, 12)
    off, idx = orc.e2lsh_near_neighbours(X, Q, G, b, K, L)
    _, kx = orc.e2lsh_hash(X, G, b, K, L)
    _, kq = orc.e2lsh_hash(Q, G, b, K, L)
    for q in range(Q.shape[0]):
        want = []
        for l in range(L):
            for j in range(X.shape[0]):
                if kx[j, l] == kq[q, l] and not any(kx[j, t] == kq[q, t] for t in range(l)):
                    want.append(j)
        assert list(idx[off[q]:off[q + 1]]) == want


def test_each_point_lists_itself_first_in_table_zero(orc):
    X, _, _ = synth.config_points(1)
    X = X[:300]
    G, b = synth.e2lsh_randomness(8 * 6, 10, 13)
    off, idx = orc.e2lsh_near_neighbours(X, X, G, b, 8, 6)
    _, kx = orc.e2lsh_hash(X, G, b, 8, 6)
    for i in range(X.shape[0]):
        lst = idx[off[i]:off[i + 1]]
        assert i in lst
        assert len(set(lst.tolist())) == len(lst)
        t0 = int(np.sum(kx[:, 0] == kx[i, 0]))  # table-0 bucket comes first
        assert i in lst[:t0]


def test_listing_probability_is_the_boosted_collision_probability(orc):
    """A pair at distance c is listed with probability 1 - (1 - p(c)^K)^L over
    the random projections (Monte Carlo, 4 standard errors)."""
    rng = np.random.default_rng(14)
    d, K, L, trials = 6, 3, 4, 1500
    for c in (0.7, 2.0, 4.0):
        hits = 0
        for t in range(trials):
            x = rng.normal(size=(1, d)).astype(np.float32)
            u = rng.normal(size=d)
            y = (x[0] + c * u / np.linalg.norm(u)).astype(np.float32)[None, :]
            G, b = synth.e2lsh_randomness(K * L, d, 100000 + t)
            off, idx = orc.e2lsh_near_neighbours(x, y, G, b, K, L)
            hits += int(off[1] > 0)
        p = orc.boosted_probability(c, K, L)
        se = np.sqrt(p * (1 - p) / trials)
        assert abs(hits / trials - p) < 4 * se + 2e-3, (c, hits / trials, p)
