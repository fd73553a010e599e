"""Pins of the spectral-clustering oracle (Sec. "Fast Spectral Clustering":
similarity graph, bottom-k Laplacian eigenvectors, k-means), against closed
forms of graph spectra and hand-worked k-means runs."""
import math

import numpy as np
import pytest

import oracle
from oracle import spectral


def _edges_of(pairs, w=None):
    src = np.array([p[0] for p in pairs], dtype=np.int64)
    dst = np.array([p[1] for p in pairs], dtype=np.int64)
    w = np.ones(len(pairs)) if w is None else np.asarray(w, dtype=np.float64)
    return src, dst, w


def _same_partition(a, b):
    # equal up to a relabelling
    a, b = np.asarray(a), np.asarray(b)
    m1, m2 = {}, {}
    for x, y in zip(a.tolist(), b.tolist()):
        if m1.setdefault(x, y) != y or m2.setdefault(y, x) != x:
            return False
    return True


# ---------------------------------------------------------------- k-means

def test_kmeans_hand_worked_run():
    # points 0, 1, 10, 11 from centres (0, 1): assignment {0 | 1, 10, 11},
    # centres (0, 22/3); then {0, 1 | 10, 11}, centres (0.5, 10.5); then stable
    P = np.array([[0.0], [1.0], [10.0], [11.0]])
    labels, C, it, _ = oracle.kmeans(P, 2, seed=0, init=np.array([[0.0], [1.0]]))
    assert labels.tolist() == [0, 0, 1, 1]
    assert C[:, 0].tolist() == [0.5, 10.5]
    assert it == 3


def test_kmeans_tie_goes_to_lowest_centre():
    P = np.array([[0.0], [2.0], [4.0]])
    labels, _, _, _ = oracle.kmeans(P, 2, seed=0, init=np.array([[1.0], [3.0]]), max_iter=1)
    # 2.0 is at distance 1 from both centres
    assert labels.tolist() == [0, 0, 1]


def test_kmeanspp_first_centre_uniform_then_d2_weighted():
    # points 0, 1, 3: the first centre is uniform; from centre 0 the second is
    # point 1 w.p. 1/10 and point 3 w.p. 9/10 (squared distances 0, 1, 9)
    P = np.array([[0.0], [1.0], [3.0]])
    firsts, seconds = [], []
    for seed in range(12000):
        _, _, _, s = oracle.kmeans(P, 2, seed=seed, max_iter=1)
        firsts.append(s[0])
        if s[0] == 0:
            seconds.append(s[1])
    f = np.bincount(firsts, minlength=3) / len(firsts)
    assert np.all(np.abs(f - 1 / 3) < 5 * math.sqrt(2 / 9 / len(firsts)))
    p1 = np.mean(np.array(seconds) == 1)
    assert abs(p1 - 0.1) < 5 * math.sqrt(0.09 / len(seconds))
    assert set(seconds) <= {1, 2}


def test_kmeans_objective_never_increases_and_ends_at_argmin():
    rng = np.random.default_rng(3)
    P = rng.normal(size=(500, 4))
    prev = np.inf
    for it in range(1, 12):
        labels, C, used, _ = oracle.kmeans(P, 6, seed=9, max_iter=it)
        # objective of the labels against the centres they were assigned with
        # is not available after an update; use the converged-or-not centres
        obj = ((P - C[labels]) ** 2).sum()
        assert obj <= prev + 1e-9
        prev = obj
    labels, C, used, _ = oracle.kmeans(P, 6, seed=9, max_iter=300)
    d = ((P[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    assert used < 300
    assert np.array_equal(labels, np.argmin(d, axis=1))


def test_kmeans_separated_blobs_and_k_equals_n():
    rng = np.random.default_rng(4)
    centres = np.array([[0.0, 0.0], [50.0, 0.0], [0.0, 50.0]])
    truth = np.repeat(np.arange(3), 40)
    P = centres[truth] + rng.normal(size=(120, 2))
    labels, _, _, _ = oracle.kmeans(P, 3, seed=1)
    assert _same_partition(labels, truth)
    P2 = rng.normal(size=(7, 3))
    labels2, C2, _, seeds = oracle.kmeans(P2, 7, seed=2)
    assert sorted(seeds.tolist()) == list(range(7))
    assert sorted(labels2.tolist()) == list(range(7))


def test_kmeans_duplicates_use_the_fallback():
    # two distinct points, k = 3: the third seed has total weight 0
    P = np.array([[0.0], [0.0], [5.0], [5.0]])
    labels, C, _, seeds = oracle.kmeans(P, 3, seed=5)
    assert len(set(seeds.tolist())) == 3
    assert _same_partition(labels[[0, 2]], [0, 1])


# ---------------------------------------------------------------- spectra

def test_disjoint_cliques():
    # union of cliques K_5, K_7, K_9: N has eigenvalue 0 once per component
    # (eigenvector D^{1/2} 1 on the component) and s/(s-1) on K_s
    sizes, pairs, base = [5, 7, 9], [], 0
    for s in sizes:
        pairs += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
        base += s
    src, dst, w = _edges_of(pairs)
    n = base
    vals, U = spectral.spectral_embedding(n, src, dst, w, 4)
    np.testing.assert_allclose(vals[:3], 0.0, atol=1e-12)
    assert vals[3] == pytest.approx(9 / 8, rel=1e-12)
    P = U[:, :3] @ U[:, :3].T
    Z = np.zeros((n, 3))
    base = 0
    for c, s in enumerate(sizes):
        Z[base:base + s, c] = 1.0 / math.sqrt(s)  # equal degrees inside a clique
        base += s
    np.testing.assert_allclose(P, Z @ Z.T, atol=1e-12)


@pytest.mark.parametrize("n", [5, 12, 31])
def test_cycle_spectrum(n):
    src, dst, w = _edges_of([(i, (i + 1) % n) for i in range(n)], w=np.full(n, 2.5))
    vals, _ = spectral.spectral_embedding(n, src, dst, w, n)
    want = np.sort(1.0 - np.cos(2 * np.pi * np.arange(n) / n))
    np.testing.assert_allclose(vals, want, atol=1e-12)


def test_complete_graph_spectrum():
    n = 9
    src, dst, w = _edges_of([(i, j) for i in range(n) for j in range(i + 1, n)], w=np.full(36, 0.3))
    vals, _ = spectral.spectral_embedding(n, src, dst, w, n)
    assert abs(vals[0]) < 1e-12
    np.testing.assert_allclose(vals[1:], n / (n - 1), rtol=1e-12)


def test_edge_list_reading():
    # duplicates add up, direction does not matter, dst = -1 is skipped, an
    # isolated vertex has eigenvalue 1
    s1, d1, w1 = _edges_of([(0, 1), (1, 0), (1, 2), (2, 3)], w=[0.5, 0.25, 1.0, 2.0])
    s2, d2, w2 = _edges_of([(0, 1), (2, 1), (3, 2), (3, -1)], w=[0.75, 1.0, 2.0, 9.0])
    np.testing.assert_array_equal(spectral.adjacency_dense(5, s1, d1, w1), spectral.adjacency_dense(5, s2, d2, w2))
    vals, U = spectral.spectral_embedding(5, s1, d1, w1, 5)
    assert np.any(np.abs(vals - 1.0) < 1e-12)
    iso = np.abs(U[4]) > 0.5
    assert iso.sum() == 1


def test_spectral_cluster_recovers_separated_mixture():
    # the full pipeline on the oracle's own sampled graph of three far-apart blobs
    rng = np.random.default_rng(8)
    centres = np.array([[0.0, 0.0, 0.0], [30.0, 0.0, 0.0], [0.0, 30.0, 0.0]])
    truth = np.repeat(np.arange(3), [60, 80, 100])
    X = (centres[truth] + rng.normal(size=(240, 3))).astype(np.float32)
    src, dst, w, _ = oracle.simgraph_exact(X, 0.5, 8, seed=77)  # s = ceil(log2 240)
    labels = spectral.spectral_cluster(240, src, dst, w, 3, seed=5)
    assert _same_partition(labels, truth)


def test_bottom_eigenvector_is_sqrt_degree():
    # connected graph with unequal degrees: N D^{1/2} 1 = 0, so the bottom
    # eigenvector is sqrt(deg) / ||sqrt(deg)||, positive under the sign rule
    # (a random-walk or unnormalised Laplacian would give the constant vector)
    src, dst, w = _edges_of([(0, 1), (1, 2), (2, 3), (0, 2), (3, 4)], w=[1.0, 3.0, 0.5, 2.0, 4.0])
    A = spectral.adjacency_dense(5, src, dst, w)
    deg = A.sum(1)
    assert deg.tolist() == [3.0, 4.0, 5.5, 4.5, 4.0]
    vals, U = spectral.spectral_embedding(5, src, dst, w, 2)
    assert abs(vals[0]) < 1e-12 and vals[1] > 1e-3
    np.testing.assert_allclose(U[:, 0], np.sqrt(deg) / np.linalg.norm(np.sqrt(deg)), rtol=1e-12)
