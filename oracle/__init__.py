"""FP64 CPU oracle for the Gaussian-KDE hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library does not depend on it and shares no
code with it.  Every function here is a thin numpy/ctypes shim over
``oracle.cpp``, where the arithmetic lives, each function citing the passage
of the paper it follows; the spectral embedding is plain numpy
(``oracle/spectral.py``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TAG_MASK = 0x4D41534B
TAG_DRAW = 0x44524157
FLAG_LITERAL = 1
FLAG_ALL_SAMPLED = 2


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    f64p = C.POINTER(C.c_double)
    f32p = C.POINTER(C.c_float)
    i32p = C.POINTER(C.c_int32)
    i64p = C.POINTER(C.c_int64)
    u64p = C.POINTER(C.c_uint64)
    u8p = C.POINTER(C.c_uint8)
    lib.orc_mix64.restype = C.c_uint64
    lib.orc_mix64.argtypes = [C.c_uint64]
    lib.orc_counter_bits.restype = C.c_uint64
    lib.orc_counter_bits.argtypes = [C.c_uint64] * 5
    lib.orc_bucket_key.restype = C.c_uint64
    lib.orc_bucket_key.argtypes = [C.c_int32, i32p, C.c_int32]
    lib.orc_collision_probability.restype = C.c_double
    lib.orc_collision_probability.argtypes = [C.c_double]
    lib.orc_boosted_probability.restype = C.c_double
    lib.orc_boosted_probability.argtypes = [C.c_double, C.c_int32, C.c_int32]
    lib.orc_gaussian_kernel.restype = C.c_double
    lib.orc_gaussian_kernel.argtypes = [C.c_double, f32p, f32p, C.c_int32]
    lib.orc_kde_exact.restype = None
    lib.orc_kde_exact.argtypes = [f32p, C.c_int64, f32p, C.c_int64, C.c_int32, C.c_double, f64p, f64p, C.c_int32]
    lib.orc_kde_kernel.restype = C.c_int32
    lib.orc_kde_kernel.argtypes = [f32p, C.c_int64, f32p, C.c_int64, C.c_int32, C.c_int32, C.c_double, f64p, C.c_int32]
    lib.orc_kernel_value.restype = C.c_double
    lib.orc_kernel_value.argtypes = [C.c_int32, C.c_double, C.c_double]
    lib.orc_kmeans.restype = C.c_int32
    lib.orc_kmeans.argtypes = [f64p, C.c_int64, C.c_int32, C.c_int32, C.c_uint64, C.c_int32, f64p, i32p, f64p,
                               C.POINTER(C.c_int32), i64p]
    lib.orc_kde_random_sample.restype = None
    lib.orc_kde_random_sample.argtypes = [f32p, C.c_int64, f32p, C.c_int64, C.c_int32, C.c_double, C.c_int64,
                                          C.c_uint64, f64p, i64p, C.c_int32]
    lib.orc_rs_sample_size.restype = C.c_int64
    lib.orc_rs_sample_size.argtypes = [C.c_double, C.c_double, C.c_int64, C.c_double]
    lib.orc_kernel_row.restype = None
    lib.orc_kernel_row.argtypes = [f32p, C.c_int64, C.c_int32, C.c_double, C.c_int64, f64p]
    lib.orc_e2lsh_hash.restype = None
    lib.orc_e2lsh_hash.argtypes = [f32p, C.c_int64, C.c_int32, f32p, f64p, C.c_int32, C.c_int32, i32p, u64p, C.c_int32]
    lib.orc_e2lsh_near_neighbours.restype = None
    lib.orc_e2lsh_near_neighbours.argtypes = [f32p, C.c_int64, f32p, C.c_int64, C.c_int32, f32p, f64p, C.c_int32,
                                              C.c_int32, C.POINTER(C.c_int64), i32p, C.c_int32]
    lib.orc_lsh_derive.restype = C.c_int32
    lib.orc_lsh_derive.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                   C.c_uint32, i32p, f64p, f64p, u64p, f64p, f64p]
    lib.orc_lsh_mask.restype = None
    lib.orc_lsh_mask.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int64, C.c_uint64, u8p]
    lib.orc_lsh_kde.restype = C.c_int32
    lib.orc_lsh_kde.argtypes = [f32p, C.c_int64, C.c_int32, f32p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                C.c_int32, C.c_double, C.c_int32, C.c_uint64, C.c_uint32, f32p, f64p, f64p, i64p, i64p,
                                f64p, C.c_int32]
    lib.orc_draw_uniform.restype = C.c_double
    lib.orc_draw_uniform.argtypes = [C.c_uint64, C.c_int64, C.c_int32]
    lib.orc_simgraph_exact.restype = None
    lib.orc_simgraph_tree.argtypes = [f32p, C.c_int64, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int64,
                                      C.c_uint64, C.c_int64, C.c_int64, i64p, i64p, f64p, f64p, f64p, C.c_int32]
    lib.orc_simgraph_tree.restype = None
    lib.orc_simgraph_exact.argtypes = [f32p, C.c_int64, C.c_int32, C.c_double, C.c_int32, C.c_uint64, i64p, i64p, f64p,
                                       f64p, f64p, C.c_int32]
    lib.orc_simgraph_lsh.restype = C.c_int32
    lib.orc_simgraph_lsh.argtypes = [f32p, C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32,
                                     C.c_double, C.c_int32, C.c_uint64, C.c_uint32, f32p, f64p, C.c_int32, C.c_uint64,
                                     i64p, i64p, f64p, f64p, f64p, C.c_int32]
    _lib = lib
    return lib


def _p(arr, ctype):
    if arr is None:
        return None
    return arr.ctypes.data_as(C.POINTER(ctype))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def mix64(z: int) -> int:
    return int(_load().orc_mix64(C.c_uint64(z & 0xFFFFFFFFFFFFFFFF)))


def counter_bits(seed, tag, a, b, c) -> int:
    m = 0xFFFFFFFFFFFFFFFF
    return int(_load().orc_counter_bits(seed & m, tag & m, a & m, b & m, c & m))


def bucket_key(l: int, codes) -> int:
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    return int(_load().orc_bucket_key(l, _p(codes, C.c_int32), len(codes)))


def collision_probability(c: float) -> float:
    return float(_load().orc_collision_probability(float(c)))


def boosted_probability(c: float, K: int, L: int) -> float:
    return float(_load().orc_boosted_probability(float(c), int(K), int(L)))


def gaussian_kernel(a: float, p1, p2) -> float:
    p1, p2 = _f32(p1), _f32(p2)
    return float(_load().orc_gaussian_kernel(float(a), _p(p1, C.c_float), _p(p2, C.c_float), p1.shape[-1]))


def kde_exact(X, Q, a: float, nthreads: int = 0, return_log: bool = False):
    """S(q) = sum_i exp(-a ||q - x_i||^2) for each row of Q (float64)."""
    X, Q = _f32(X), _f32(Q)
    n, d = X.shape
    m = Q.shape[0]
    S = np.empty(m, dtype=np.float64)
    lg = np.empty(m, dtype=np.float64)
    _load().orc_kde_exact(_p(X, C.c_float), n, _p(Q, C.c_float), m, d, float(a), _p(S, C.c_double),
                          _p(lg, C.c_double), int(nthreads))
    return (S, lg) if return_log else S


KERNELS = {"gaussian": 0, "exponential": 1, "logistic": 2}


def kde_kernel(X, Q, a: float, kernel: str = "gaussian", nthreads: int = 0):
    """S(q) = sum_i k(||q - x_i||) for each row of Q (float64); kernel is
    "gaussian" exp(-a r^2), "exponential" exp(-a r) or "logistic"
    4/(2 + e^{ar} + e^{-ar})."""
    X, Q = _f32(X), _f32(Q)
    n, d = X.shape
    m = Q.shape[0]
    S = np.empty(m, dtype=np.float64)
    rc = _load().orc_kde_kernel(_p(X, C.c_float), n, _p(Q, C.c_float), m, d, KERNELS[kernel], float(a),
                                _p(S, C.c_double), int(nthreads))
    assert rc == 0
    return S


def kernel_value(kernel: str, a: float, r: float) -> float:
    return float(_load().orc_kernel_value(KERNELS[kernel], float(a), float(r)))


def kmeans(P, k: int, seed: int, max_iter: int = 300, init=None):
    """k-means (Lloyd, k-means++ seeding) as stated in oracle.cpp; returns
    (labels int32 [n], centres float64 [k][dim], iterations, seed indices)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    n, dim = P.shape
    labels = np.empty(n, dtype=np.int32)
    Cm = np.empty((k, dim), dtype=np.float64)
    seeds = np.empty(k, dtype=np.int64)
    it = C.c_int32(0)
    ini = None
    if init is not None:
        ini = np.ascontiguousarray(init, dtype=np.float64)
        assert ini.shape == (k, dim)
    rc = _load().orc_kmeans(_p(P, C.c_double), n, dim, int(k), C.c_uint64(int(seed) & (2**64 - 1)), int(max_iter),
                            None if ini is None else _p(ini, C.c_double), _p(labels, C.c_int32), _p(Cm, C.c_double),
                            C.byref(it), _p(seeds, C.c_int64))
    assert rc == 0
    return labels, Cm, int(it.value), seeds


def kde_random_sample(X, Q, a: float, s: int, seed: int, nthreads: int = 0):
    """(estimates float64 [m], sample indices int64 [s]) of the random-sampling
    estimator (n/s) sum_r exp(-a ||q - x_{j_r}||^2)."""
    X, Q = _f32(X), _f32(Q)
    n, d = X.shape
    m = Q.shape[0]
    S = np.empty(m, dtype=np.float64)
    idx = np.empty(int(s), dtype=np.int64)
    _load().orc_kde_random_sample(_p(X, C.c_float), n, _p(Q, C.c_float), m, d, float(a), int(s),
                                  C.c_uint64(int(seed) & (2**64 - 1)), _p(S, C.c_double), _p(idx, C.c_int64),
                                  int(nthreads))
    return S, idx


def rs_sample_size(eps: float, mu: float, m: int, delta: float) -> int:
    return int(_load().orc_rs_sample_size(float(eps), float(mu), int(m), float(delta)))


def kernel_row(X, a: float, i: int):
    X = _f32(X)
    n, d = X.shape
    out = np.empty(n, dtype=np.float64)
    _load().orc_kernel_row(_p(X, C.c_float), n, d, float(a), int(i), _p(out, C.c_double))
    return out


def e2lsh_hash(X, G, b, K: int, L: int, nthreads: int = 0):
    """codes [n][L][K] int32 and keys [n][L] uint64."""
    X, G = _f32(X), _f32(G)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n, d = X.shape
    assert G.shape == (L * K, d) and b.shape == (L * K,)
    codes = np.empty((n, L, K), dtype=np.int32)
    keys = np.empty((n, L), dtype=np.uint64)
    _load().orc_e2lsh_hash(_p(X, C.c_float), n, d, _p(G, C.c_float), _p(b, C.c_double), K, L,
                           _p(codes, C.c_int32), _p(keys, C.c_uint64), int(nthreads))
    return codes, keys


def e2lsh_near_neighbours(X, Q, G, b, K: int, L: int, nthreads: int = 0):
    """(offsets [m+1] int64, idx int32): the points colliding with each query
    in some table, table by table, ascending within a table, each once."""
    X, Q, G = _f32(X), _f32(Q), _f32(G)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n, d = X.shape
    m = Q.shape[0]
    assert Q.shape[1] == d and G.shape == (L * K, d) and b.shape == (L * K,)
    counts = np.empty(m, dtype=np.int64)
    lib = _load()
    lib.orc_e2lsh_near_neighbours(_p(X, C.c_float), n, _p(Q, C.c_float), m, d, _p(G, C.c_float),
                                  _p(b, C.c_double), K, L, _p(counts, C.c_int64), None, int(nthreads))
    off = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    idx = np.empty(int(off[-1]), dtype=np.int32)
    lib.orc_e2lsh_near_neighbours(_p(X, C.c_float), n, _p(Q, C.c_float), m, d, _p(G, C.c_float),
                                  _p(b, C.c_double), K, L, _p(counts, C.c_int64), _p(idx, C.c_int32),
                                  int(nthreads))
    return off, idx


def lsh_derive(n, a, eps=0.5, min_mu=0.0, k1=0, k2_constant=0.0, p_offset=0, flags=0):
    """Derived CKNS parameters: dict(J, L, K, K1, mu_min, p, thr, T, r)."""
    shape = np.zeros(4, dtype=np.int32)
    mu = np.zeros(1, dtype=np.float64)
    p = np.zeros(65, dtype=np.float64)
    thr = np.zeros(65, dtype=np.uint64)
    T = np.zeros(65, dtype=np.float64)
    r = np.zeros(65, dtype=np.float64)
    rc = _load().orc_lsh_derive(int(n), float(a), float(eps), float(min_mu), int(k1), float(k2_constant),
                                int(p_offset), int(flags), _p(shape, C.c_int32), _p(mu, C.c_double),
                                _p(p, C.c_double), _p(thr, C.c_uint64), _p(T, C.c_double), _p(r, C.c_double))
    if rc:
        raise ValueError(f"invalid CKNS parameters (code {rc})")
    J = int(shape[0])
    return dict(J=J, L=int(shape[1]), K=int(shape[2]), K1=int(shape[3]), mu_min=float(mu[0]),
                p=p[:J + 1].copy(), thr=thr[:J + 1].copy(), T=T[:J + 1].copy(), r=r[:J + 1].copy())


def lsh_mask(seed, t, i, n, thr):
    keep = np.empty(n, dtype=np.uint8)
    _load().orc_lsh_mask(seed & 0xFFFFFFFFFFFFFFFF, int(t), int(i), int(n), int(thr), _p(keep, C.c_uint8))
    return keep.astype(bool)


def lsh_kde(X, Q, a, G0, B, seed, eps=0.5, min_mu=0.0, k1=0, k2_constant=0.0, p_offset=0, flags=0,
            nthreads: int = 0, return_stats: bool = False):
    """CKNS estimate for each row of Q.  G0 is [K1][J][L][K][d] N(0,1) fp32,
    B is [K1][J][L][K] in [0,4) (both as produced by the seeded generator)."""
    X, Q = _f32(X), _f32(Q)
    n, d = X.shape
    m = Q.shape[0]
    sh = lsh_derive(n, a, eps, min_mu, k1, k2_constant, p_offset, flags)
    G0 = _f32(G0).reshape(-1)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1)
    npj = sh["K1"] * sh["J"] * sh["L"] * sh["K"]
    assert G0.size == npj * d and B.size == npj, (G0.size, B.size, npj, d)
    S = np.empty(m, dtype=np.float64)
    nc = np.empty(m, dtype=np.int64)
    na = np.empty(m, dtype=np.int64)
    Sc = np.empty((m, sh["K1"]), dtype=np.float64)
    rc = _load().orc_lsh_kde(_p(X, C.c_float), n, d, _p(Q, C.c_float), m, float(a), float(eps), float(min_mu),
                             int(k1), float(k2_constant), int(p_offset), seed & 0xFFFFFFFFFFFFFFFF, int(flags),
                             _p(G0, C.c_float), _p(B, C.c_double), _p(S, C.c_double), _p(nc, C.c_int64),
                             _p(na, C.c_int64), _p(Sc, C.c_double), int(nthreads))
    if rc:
        raise ValueError(f"orc_lsh_kde failed ({rc})")
    if return_stats:
        return S, dict(n_cand=nc, n_acc=na, S_copies=Sc, shape=sh)
    return S


def draw_uniform(seed, i, r) -> float:
    return float(_load().orc_draw_uniform(seed & 0xFFFFFFFFFFFFFFFF, int(i), int(r)))


def simgraph_exact(X, a, s, seed, nthreads: int = 0, return_margin: bool = False):
    """(src, dst, w, deg) of the exact-kernel edge sampler (+ margin)."""
    X = _f32(X)
    n, d = X.shape
    e = n * s
    src = np.empty(e, dtype=np.int64)
    dst = np.empty(e, dtype=np.int64)
    w = np.empty(e, dtype=np.float64)
    deg = np.empty(n, dtype=np.float64)
    mg = np.empty(e, dtype=np.float64)
    _load().orc_simgraph_exact(_p(X, C.c_float), n, d, float(a), int(s), seed & 0xFFFFFFFFFFFFFFFF,
                               _p(src, C.c_int64), _p(dst, C.c_int64), _p(w, C.c_double), _p(deg, C.c_double),
                               _p(mg, C.c_double), int(nthreads))
    return (src, dst, w, deg, mg) if return_margin else (src, dst, w, deg)


def simgraph_tree(X, a, s, t, t_deg, seed, nthreads: int = 0, rows=None):
    """(src, dst, w, deg, margin) of the KDE-tree edge sampler: descent by
    random-sampling node estimates with t samples, degrees with t_deg.
    rows = (lo, hi) limits the draws to those rows (degrees cover all)."""
    X = _f32(X)
    n, d = X.shape
    lo, hi = (0, n) if rows is None else (int(rows[0]), int(rows[1]))
    e = (hi - lo) * s
    src = np.empty(e, dtype=np.int64)
    dst = np.empty(e, dtype=np.int64)
    w = np.empty(e, dtype=np.float64)
    deg = np.empty(n, dtype=np.float64)
    mg = np.empty(e, dtype=np.float64)
    _load().orc_simgraph_tree(_p(X, C.c_float), n, d, float(a), int(s), int(t), int(t_deg),
                              seed & 0xFFFFFFFFFFFFFFFF, lo, hi, _p(src, C.c_int64), _p(dst, C.c_int64), _p(w, C.c_double),
                              _p(deg, C.c_double), _p(mg, C.c_double), int(nthreads))
    return src, dst, w, deg, mg


def simgraph_lsh(X, a, s, draw_seed, G0, B, lsh_seed, eps=0.5, min_mu=0.0, k1=0, k2_constant=0.0, p_offset=0,
                 flags=0, nthreads: int = 0):
    """(src, dst, w, deg, margin) of the CKNS-based edge sampler."""
    X = _f32(X)
    n, d = X.shape
    e = n * s
    src = np.empty(e, dtype=np.int64)
    dst = np.empty(e, dtype=np.int64)
    w = np.empty(e, dtype=np.float64)
    deg = np.empty(n, dtype=np.float64)
    mg = np.empty(e, dtype=np.float64)
    G0 = _f32(G0).reshape(-1)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1)
    rc = _load().orc_simgraph_lsh(_p(X, C.c_float), n, d, float(a), float(eps), float(min_mu), int(k1),
                                  float(k2_constant), int(p_offset), lsh_seed & 0xFFFFFFFFFFFFFFFF, int(flags),
                                  _p(G0, C.c_float), _p(B, C.c_double), int(s), draw_seed & 0xFFFFFFFFFFFFFFFF,
                                  _p(src, C.c_int64), _p(dst, C.c_int64), _p(w, C.c_double), _p(deg, C.c_double),
                                  _p(mg, C.c_double), int(nthreads))
    if rc:
        raise ValueError(f"orc_simgraph_lsh failed ({rc})")
    return src, dst, w, deg, mg
