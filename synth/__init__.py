"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no part of the method's arithmetic: it only draws numbers.
It produces
  * isotropic Gaussian-mixture point sets (the data and query shapes of the
    paper's KDE benchmark, which draws queries from the data distribution,
    Sec. "Kernel Density Estimation" of the showcase studies);
  * the sparse non-negative stand-in for a 784-dimensional image data set
    (80 % zeros, else U[0,1]);
  * the stored randomness that E2LSH consumes: Gaussian projection vectors
    g ~ N(0, I_d) and offsets b ~ U[0, 4) (Sec. "Random Projection");
  * Poisson request streams with log-uniform batch sizes for the serving loop.

All draws use numpy's PCG64 ``default_rng(seed)``; no dataset items of any
public benchmark are reproduced anywhere.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Mixture:
    """Parameters of an equal-weight isotropic Gaussian mixture in R^d."""

    means: np.ndarray   # [k][d] float64
    sigmas: np.ndarray  # [k] float64

    @property
    def d(self) -> int:
        return int(self.means.shape[1])

    @property
    def k(self) -> int:
        return int(self.means.shape[0])


def mixture(d: int, k: int, seed: int, sigma=1.0, box: float = 5.0) -> Mixture:
    """Component means ~ U[-box, box]^d; sigma is a constant or a (lo, hi)
    range from which each component's standard deviation is drawn uniformly."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-box, box, size=(k, d))
    if isinstance(sigma, (tuple, list)):
        sig = rng.uniform(float(sigma[0]), float(sigma[1]), size=k)
    else:
        sig = np.full(k, float(sigma))
    return Mixture(means=means, sigmas=sig)


def sample(mix: Mixture, count: int, seed: int, return_labels: bool = False):
    """Draw ``count`` points (float32, row-major [count][d]) from the mixture
    with equal component weights."""
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, mix.k, size=count)
    pts = mix.means[lab] + rng.standard_normal((count, mix.d)) * mix.sigmas[lab, None]
    pts = np.ascontiguousarray(pts.astype(np.float32))
    if return_labels:
        return pts, lab
    return pts


def sparse_uniform(n: int, d: int, seed: int, zero_prob: float = 0.8) -> np.ndarray:
    """Each entry independently 0 with probability ``zero_prob``, else U[0,1]."""
    rng = np.random.default_rng(seed)
    vals = rng.uniform(0.0, 1.0, size=(n, d))
    keep = rng.uniform(0.0, 1.0, size=(n, d)) >= zero_prob
    return np.ascontiguousarray((vals * keep).astype(np.float32))


def gaussian_projections(count: int, d: int, seed: int) -> np.ndarray:
    """``count`` projection vectors with i.i.d. N(0,1) entries, stored as
    float32 [count][d] (the stored values are what both sides consume)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((count, d)).astype(np.float32))


def uniform_offsets(count: int, seed: int, width: float = 4.0) -> np.ndarray:
    """``count`` bucket offsets b = width * U[0,1), float64."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(width * rng.random(count))


def e2lsh_randomness(n_proj: int, d: int, seed: int):
    """Projections [n_proj][d] fp32 and offsets [n_proj] f64 from one seed."""
    g = gaussian_projections(n_proj, d, seed)
    b = uniform_offsets(n_proj, seed + 0x5EED)
    return g, b


# --------------------------------------------------------------------------
# Workload configurations (seeds: data 1000+c, queries 2000+c, LSH 3000+c,
# arrivals 4000+c).
# --------------------------------------------------------------------------

def config_points(cfg: int, n: int | None = None, m: int | None = None, queries_from_data: bool = False):
    """Data X and queries Q of one of four synthetic workloads, at optional
    reduced sizes.  Returns (X, Q, info dict).

      1: n = m = 1,000, d = 10, 5-component isotropic Gaussian mixture,
         means U[-5,5]^d, sigma = 1 (correctness size);
      2: n = m = 100,000, d = 64, 20 components, sigma U[0.5,2];
      3: n = 2,000,000, m = 200,000, d = 128, 50 components, sigma U[0.5,2]
         (the precision-form workload);
      4: n = 70,000, d = 784, entries 0 with probability 0.8 else U[0,1]
         (queries are the data; edge sampling).
    Queries are fresh draws from the same mixture (or rows of X); for the
    mixtures info["labels"] holds each data point's component."""
    if cfg == 1:
        d, k, sig, n0, m0 = 10, 5, 1.0, 1000, 1000
    elif cfg == 2:
        d, k, sig, n0, m0 = 64, 20, (0.5, 2.0), 100_000, 100_000
    elif cfg == 3:
        d, k, sig, n0, m0 = 128, 50, (0.5, 2.0), 2_000_000, 200_000
    elif cfg == 4:
        n0 = 70_000 if n is None else n
        X = sparse_uniform(n0, 784, 1000 + cfg)
        return X, X, {"d": 784, "n": n0, "m": n0}
    else:
        raise ValueError(cfg)
    n = n0 if n is None else n
    m = m0 if m is None else m
    mix = mixture(d, k, 1000 + cfg, sigma=sig)
    X, lab = sample(mix, n, 1000 + cfg + 10_000, return_labels=True)
    if queries_from_data:
        rng = np.random.default_rng(2000 + cfg)
        Q = np.ascontiguousarray(X[rng.choice(n, size=m, replace=m > n)])
    else:
        Q = sample(mix, m, 2000 + cfg)
    return X, Q, {"d": d, "n": n, "m": m, "k": k, "labels": lab}


def poisson_requests(count: int, rate_per_s: float, seed: int, max_batch: int = 65536,
                     n_datasets: int = 4):
    """A Poisson arrival stream: (arrival_time_s, batch_size, dataset_index).

    Batch sizes are log-uniform on 1..max_batch: m = min(max_batch,
    floor(exp(U * ln(max_batch + 1)))) with U ~ U[0,1)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    u = rng.random(count)
    sizes = np.minimum(max_batch, np.floor(np.exp(u * math.log(max_batch + 1.0)))).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    ds = rng.integers(0, n_datasets, size=count)
    return t, sizes, ds
