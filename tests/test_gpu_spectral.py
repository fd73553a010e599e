"""GPU parity of spectral clustering (Sec. "Fast Spectral Clustering") through
the C ABI: the graph build and Laplacian embedding against the dense FP64
oracle (eigenvalues within 1e-9, eigenvectors within 1e-7 where the
eigenvalue is separated from its neighbours by more than 1e-3, the subspace
otherwise), closed-form spectra, and k-means bit-exact against the oracle's
k-means on the same points (labels, centres, rounds and seeds equal)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import spectral as ospec
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def _dev_edges(src, dst, w):
    return to_dev(np.asarray(src, np.int64)), to_dev(np.asarray(dst, np.int64)), to_dev(np.asarray(w, np.float64))


def _embed(stag, n, src, dst, w, k, **kw):
    import torch
    lam, U, it = stag.spectral_embedding(n, *_dev_edges(src, dst, w), k, **kw)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), U.cpu().numpy(), it


def _same_partition(a, b):
    m1, m2 = {}, {}
    for x, y in zip(np.asarray(a).tolist(), np.asarray(b).tolist()):
        if m1.setdefault(x, y) != y or m2.setdefault(y, x) != x:
            return False
    return True


def _check_against_oracle(n, src, dst, w, k, lam, U):
    lo, Uo = ospec.spectral_embedding(n, src, dst, w, k + 1)
    np.testing.assert_allclose(lam, lo[:k], atol=1e-9)
    # subspace of the k vectors (unique when lambda_k < lambda_{k+1})
    if lo[k] - lo[k - 1] > 1e-3:
        cos = np.linalg.svd(Uo[:, :k].T @ U, compute_uv=False)
        assert cos.min() > 1.0 - 1e-10, cos.min()
    for j in range(k):
        sep = min([abs(lo[j] - lo[i]) for i in range(k + 1) if i != j] + [1.0])
        if sep > 1e-3:
            np.testing.assert_allclose(U[:, j], Uo[:, j], atol=1e-7)
    # the sign rule on the GPU output itself
    for j in range(k):
        i = int(np.argmax(np.abs(U[:, j])))
        assert U[i, j] > 0


@pytest.mark.parametrize("cfg,n,k,a", [(1, 1000, 5, 0.5), (2, 3000, 20, 0.01), (2, 3000, 20, 0.05),
                                       (1, 1537, 1, 0.5), (1, 700, 7, 2.0)])
def test_embedding_of_sampled_graph(stag, cfg, n, k, a):
    X, _, _ = synth.config_points(cfg, n=n, m=1)
    s = max(1, int(n - 1).bit_length())
    src, dst, w, _ = oracle.simgraph_exact(X, a, s, seed=5)
    announce(f"spectral embedding cfg={cfg} n={n} k={k} a={a}")
    lam, U, it = _embed(stag, n, src, dst, w, k)
    _check_against_oracle(n, src, dst, w, k, lam, U)
    # unit columns, orthogonal
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)


def test_embedding_is_deterministic(stag):
    X, _, _ = synth.config_points(2, n=2000, m=1)
    src, dst, w, _ = oracle.simgraph_exact(X, 0.01, 11, seed=6)
    announce("spectral embedding determinism")
    l1, U1, i1 = _embed(stag, 2000, src, dst, w, 10, seed=3)
    l2, U2, i2 = _embed(stag, 2000, src, dst, w, 10, seed=3)
    assert np.array_equal(l1, l2) and np.array_equal(U1, U2) and i1 == i2


def test_disjoint_cliques_and_isolated_vertices(stag):
    # cliques K_5, K_7, K_9 with unequal weights, one isolated vertex and a few
    # empty draws: eigenvalue 0 per clique, 1 for the isolated vertex
    pairs, wts, base = [], [], 0
    rng = np.random.default_rng(2)
    for s in (5, 7, 9):
        for i in range(s):
            for j in range(i + 1, s):
                pairs.append((base + i, base + j))
                wts.append(rng.uniform(0.5, 2.0))
        base += s
    n = base + 1
    src = np.array([p[0] for p in pairs] + [0, 3], np.int64)
    dst = np.array([p[1] for p in pairs] + [-1, -1], np.int64)
    w = np.array(wts + [5.0, 7.0])
    announce("spectral cliques + isolated vertex")
    lam, U, _ = _embed(stag, n, src, dst, w, 4)
    lo, Uo = ospec.spectral_embedding(n, src, dst, w, 4)
    np.testing.assert_allclose(lam[:3], 0.0, atol=1e-10)
    np.testing.assert_allclose(lam, lo, atol=1e-9)
    np.testing.assert_allclose(U[:, :3] @ U[:, :3].T, Uo[:, :3] @ Uo[:, :3].T, atol=1e-8)


@pytest.mark.parametrize("n", [40, 257])
def test_cycle_spectrum(stag, n):
    src = np.arange(n, dtype=np.int64)
    dst = (src + 1) % n
    w = np.full(n, 1.5)
    k = 9
    announce(f"spectral cycle n={n}")
    lam, _, _ = _embed(stag, n, src, dst, w, k, tol=1e-10, max_iter=2000)
    want = np.sort(1.0 - np.cos(2 * np.pi * np.arange(n) / n))[:k]
    np.testing.assert_allclose(lam, want, atol=1e-9)


@pytest.mark.parametrize("n,k", [(1, 1), (2, 2), (5, 2), (12, 12)])
def test_tiny_graphs(stag, n, k):
    rng = np.random.default_rng(n + k)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    src = np.array([p[0] for p in pairs], np.int64)
    dst = np.array([p[1] for p in pairs], np.int64)
    w = rng.uniform(0.1, 1.0, len(pairs))
    announce(f"spectral tiny n={n} k={k}")
    lam, U, _ = _embed(stag, n, src, dst, w, k)
    lo, Uo = ospec.spectral_embedding(n, src, dst, w, k)
    np.testing.assert_allclose(lam, lo, atol=1e-9)
    np.testing.assert_allclose(U @ U.T, Uo @ Uo.T, atol=1e-8)


def test_invalid_edges_rejected(stag):
    import paper_2407_07096_amd._lib as L
    announce("spectral invalid edges")
    for src, dst, w in [([0, 1], [1, 5], [1.0, 1.0]), ([0, -1], [1, 2], [1.0, 1.0]), ([0, 1], [1, 2], [1.0, -1.0]),
                        ([0, 1], [1, -2], [1.0, 1.0]), ([0, 1], [1, 2], [1.0, np.inf])]:
        with pytest.raises(L.StagError):
            _embed(stag, 4, np.array(src), np.array(dst), np.array(w), 2)


@pytest.mark.parametrize("n,dim,k,seed", [(5000, 8, 8, 1), (3000, 20, 20, 2), (1024, 3, 5, 3), (1025, 3, 5, 4),
                                          (700, 2, 1, 5), (9, 4, 9, 6), (4097, 16, 12, 7)])
def test_kmeans_bit_exact(stag, n, dim, k, seed):
    import torch
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-10, 10, size=(k, dim))
    P = centres[rng.integers(0, k, n)] + rng.normal(size=(n, dim))
    announce(f"kmeans n={n} dim={dim} k={k}")
    lab, C, it, seeds = stag.kmeans(to_dev(P), k, seed=seed)
    torch.cuda.synchronize()
    lo, Co, ito, so = oracle.kmeans(P, k, seed)
    assert np.array_equal(seeds.cpu().numpy(), so)
    assert it == ito
    assert np.array_equal(lab.cpu().numpy(), lo)
    assert np.array_equal(C.cpu().numpy(), Co)


def test_kmeans_ties_duplicates_and_init(stag):
    import torch
    # integer grid: many exact distance ties; duplicated points force the
    # zero-total seeding fallback
    g = np.array([[x, y] for x in range(6) for y in range(6)], dtype=np.float64)
    P = np.concatenate([g, g, np.zeros((5, 2))])
    announce("kmeans ties / duplicates / init")
    for k, seed in [(4, 1), (7, 2), (36, 3)]:
        lab, C, it, seeds = stag.kmeans(to_dev(P), k, seed=seed)
        torch.cuda.synchronize()
        lo, Co, ito, so = oracle.kmeans(P, k, seed)
        assert np.array_equal(seeds.cpu().numpy(), so) and it == ito
        assert np.array_equal(lab.cpu().numpy(), lo) and np.array_equal(C.cpu().numpy(), Co)
    init = np.array([[0.5, 0.5], [4.5, 4.5], [0.0, 5.0]])
    lab, C, it, seeds = stag.kmeans(to_dev(P), 3, init=to_dev(init), max_iter=4)
    torch.cuda.synchronize()
    lo, Co, ito, _ = oracle.kmeans(P, 3, 0, max_iter=4, init=init)
    assert np.array_equal(lab.cpu().numpy(), lo) and np.array_equal(C.cpu().numpy(), Co) and it == ito
    assert np.all(seeds.cpu().numpy() == -1)


def test_kmeans_on_oracle_embedding(stag):
    import torch
    X, _, _ = synth.config_points(2, n=3000, m=1)
    src, dst, w, _ = oracle.simgraph_exact(X, 0.01, 12, seed=5)
    _, Uo = ospec.spectral_embedding(3000, src, dst, w, 20)
    announce("kmeans on the oracle's embedding")
    lab, C, it, _ = stag.kmeans(to_dev(Uo), 20, seed=11)
    torch.cuda.synchronize()
    lo, Co, ito, _ = oracle.kmeans(Uo, 20, 11)
    assert np.array_equal(lab.cpu().numpy(), lo) and np.array_equal(C.cpu().numpy(), Co) and it == ito


@pytest.mark.parametrize("cfg,n,k,a", [(1, 1000, 5, 0.5), (2, 3000, 20, 0.01)])
def test_spectral_cluster_end_to_end(stag, cfg, n, k, a):
    import torch
    X, _, info = synth.config_points(cfg, n=n, m=1)
    s = max(1, int(n - 1).bit_length())
    src, dst, w, _ = oracle.simgraph_exact(X, a, s, seed=7)
    announce(f"spectral cluster cfg={cfg} n={n} k={k}")
    lab = stag.spectral_cluster(n, *_dev_edges(src, dst, w), k, seed=13)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    ref = ospec.spectral_cluster(n, src, dst, w, k, seed=13)
    assert _same_partition(lab, ref)
    # the clusters follow the mixture's components: purity (the share of
    # points in their component's majority cluster) >= 0.97; the oracle's
    # k-means++ seeding can merge two components and split another, as here
    # for the 20-component case (purity 0.98)
    t = info["labels"]
    purity = sum(np.bincount(lab[t == c]).max() for c in range(k)) / n
    assert purity >= 0.97, purity


def _planted_graph(n, k, deg, seed):
    # seeded synthetic graph: k planted clusters, each node draws `deg`
    # neighbours inside its cluster and one anywhere with probability 0.05;
    # weights U[0.5, 1]
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, k, n)
    members = [np.flatnonzero(lab == c) for c in range(k)]
    src = np.repeat(np.arange(n), deg)
    dst = np.empty(n * deg, dtype=np.int64)
    for c in range(k):
        rows = np.flatnonzero(lab[src] == c)
        dst[rows] = members[c][rng.integers(0, len(members[c]), len(rows))]
    cross = rng.random(n * deg) < 0.05 / deg
    dst[cross] = rng.integers(0, n, int(cross.sum()))
    keep = dst != src
    return src[keep], dst[keep], rng.uniform(0.5, 1.0, int(keep.sum())), lab


def test_full_size_planted_graph(stag):
    """n = 100,000 vertices, ~1.6e6 edges, k = 20: properties that hold at any
    size, checked on the host: residuals ||N u - lambda u|| <= 1e-8,
    orthonormal columns, eigenvalues equal to ARPACK's smallest of N, and the
    planted clusters recovered."""
    import torch
    from scipy.sparse import coo_matrix, identity
    from scipy.sparse.linalg import eigsh
    n, k = 100_000, 20
    src, dst, w, lab = _planted_graph(n, k, 16, 31)
    announce("spectral full size planted n=1e5 k=20")
    lam, U, it = _embed(stag, n, src, dst, w, k)
    A = coo_matrix((np.concatenate([w, w]), (np.concatenate([src, dst]), np.concatenate([dst, src]))),
                   shape=(n, n)).tocsr()
    deg = np.asarray(A.sum(axis=1)).ravel()
    dinv = 1.0 / np.sqrt(deg)
    Mop = A.multiply(dinv[:, None]).multiply(dinv[None, :]).tocsr()
    NU = U - Mop @ U
    assert np.linalg.norm(NU - U * lam[None, :], axis=0).max() <= 1e-8
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-10)
    theta = np.sort(eigsh(Mop, k=k + 1, which="LA", tol=1e-12)[0])[::-1]
    np.testing.assert_allclose(lam, 1.0 - theta[:k], atol=1e-8)
    labels = stag.spectral_cluster(n, *_dev_edges(src, dst, w), k, seed=3)
    torch.cuda.synchronize()
    labels = labels.cpu().numpy()
    purity = sum(np.bincount(labels[lab == c]).max() for c in range(k)) / n
    assert purity >= 0.97, purity
