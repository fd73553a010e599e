"""FP64 oracle of spectral clustering on a weighted edge list -- TEST
INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Fast Spectral Clustering": (1) a similarity graph G on the n points,
(2) the bottom k eigenvectors of G's Laplacian embed the vertices into R^k,
(3) k-means on the embedded points gives the clusters.

Readings (the paper names "the Laplacian matrix" without fixing it):
  * the graph of an edge list (src, dst, w) is the symmetric weighted
    adjacency A with A[i, j] += w and A[j, i] += w for every edge whose dst is
    not negative (dst = -1 marks an empty draw); duplicates add up, a self
    loop (i, i, w) adds 2w to A[i, i];
  * the Laplacian is the normalised N = I - D^{-1/2} A D^{-1/2},
    D = diag(row sums of A), with D^{-1/2} = 0 for an isolated vertex (its
    row and column of N are those of I);
  * the embedding of vertex i is row i of the n x k matrix of N's
    eigenvectors for its k smallest eigenvalues, in ascending order, each
    eigenvector of unit norm with its entry of largest magnitude (the first
    such entry) positive;
  * k-means is ``oracle.kmeans`` (Lloyd with k-means++ seeding).
The eigenvectors come from a dense symmetric eigensolver (numpy.linalg.eigh,
LAPACK), so this oracle is for graphs of a few thousand vertices.
"""
from __future__ import annotations

import numpy as np


def adjacency_dense(n: int, src, dst, w) -> np.ndarray:
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    ok = dst >= 0
    A = np.zeros((n, n), dtype=np.float64)
    np.add.at(A, (src[ok], dst[ok]), w[ok])
    np.add.at(A, (dst[ok], src[ok]), w[ok])
    return A


def normalized_laplacian(A: np.ndarray) -> np.ndarray:
    deg = A.sum(axis=1)
    dinv = np.zeros_like(deg)
    pos = deg > 0
    dinv[pos] = 1.0 / np.sqrt(deg[pos])
    return np.eye(A.shape[0]) - dinv[:, None] * A * dinv[None, :]


def fix_signs(U: np.ndarray) -> np.ndarray:
    U = U.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def spectral_embedding(n: int, src, dst, w, k: int):
    """(eigenvalues [k] ascending, U [n][k]) of the normalised Laplacian."""
    N = normalized_laplacian(adjacency_dense(n, src, dst, w))
    vals, vecs = np.linalg.eigh(N)
    return vals[:k].copy(), fix_signs(vecs[:, :k])


def spectral_cluster(n: int, src, dst, w, k: int, seed: int, max_iter: int = 300):
    """Labels [n] of spectral clustering: embedding, then k-means."""
    import oracle
    _, U = spectral_embedding(n, src, dst, w, k)
    labels, _, _, _ = oracle.kmeans(U, k, seed, max_iter)
    return labels
