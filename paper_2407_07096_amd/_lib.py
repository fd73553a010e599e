"""ctypes binding of libstagkde.so (argument marshalling only).

Every function takes device tensors (torch, on the current HIP device), checks
dtype/shape/contiguity, allocates outputs with torch and calls the C ABI on
the tensor's current stream.  All arithmetic happens in the HIP library; if
the library is missing the binding raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstagkde.so")
HEADER = os.path.join(HERE, "..", "include", "stag_kde.h")

STAG_OK, STAG_E_INVAL, STAG_E_NOMEM, STAG_E_DEVICE, STAG_E_UNSUPPORTED, STAG_E_BUSY = range(6)
FORMS = {"fp32": 0, "bf16_split": 1, "fp16_split": 2, "bf16_split3": 3, "auto": 4, "fp16_centred": 5,
         "fp16_adaptive": 6}
KERNELS = {"gaussian": 0, "exponential": 1, "logistic": 2}
NORMALIZE = 1
CHECK_FINITE = 2

LSH_LITERAL = 1
LSH_ALL_SAMPLED = 2

_lib = None


class LshParams(C.Structure):
    _fields_ = [("min_mu", C.c_double), ("k1", C.c_int32), ("k2_constant", C.c_double), ("p_offset", C.c_int32),
                ("seed", C.c_uint64), ("flags", C.c_uint32), ("G0", C.c_void_p), ("b", C.c_void_p)]


class LshShape(C.Structure):
    _fields_ = [("J", C.c_int32), ("L", C.c_int32), ("K", C.c_int32), ("K1", C.c_int32), ("mu_min", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("rejected", C.c_uint64), ("batches", C.c_uint64), ("queries", C.c_uint64), ("p50_s", C.c_double),
                ("p99_s", C.c_double), ("mean_s", C.c_double), ("max_s", C.c_double),
                ("inflight_bytes", C.c_uint64), ("peak_inflight_bytes", C.c_uint64)]


class StagError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"stag status {status}: {msg}")
        self.status = status


def library_path() -> str:
    return LIB_PATH


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2407_07096_amd/build.py; "
                           "there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, u32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_double
    u64 = C.c_uint64
    lib.stag_last_error.restype = C.c_char_p
    lib.stag_last_error.argtypes = []
    lib.stag_version.restype = C.c_char_p
    lib.stag_version.argtypes = []
    lib.stag_e2lsh_collision_probability.restype = f64
    lib.stag_e2lsh_collision_probability.argtypes = [f64, i32, i32]
    lib.stag_kde_exact.restype = C.c_int
    lib.stag_kde_exact.argtypes = [vp, i64, vp, i64, i32, f64, f64, i32, u32, vp, vp, vp]
    lib.stag_kde_exact_noalloc.restype = C.c_int
    lib.stag_kde_exact_noalloc.argtypes = [vp, i64, vp, i64, i32, f64, i32, u32, vp, vp, vp]
    lib.stag_simgraph_draws_per_node.restype = i32
    lib.stag_simgraph_draws_per_node.argtypes = [i64, i32]
    lib.stag_kde_exact_kernel.restype = C.c_int
    lib.stag_kde_exact_kernel.argtypes = [vp, i64, vp, i64, i32, i32, f64, f64, i32, u32, vp, vp, vp]
    lib.stag_kde_random_sample.restype = C.c_int
    lib.stag_kde_random_sample.argtypes = [vp, i64, vp, i64, i32, f64, i64, u64, i32, vp, vp, vp, vp]
    lib.stag_rs_sample_size.restype = i64
    lib.stag_rs_sample_size.argtypes = [f64, f64, i64, f64]
    lib.stag_spectral_embedding.restype = C.c_int
    lib.stag_spectral_embedding.argtypes = [i64, vp, vp, vp, i64, i32, f64, i32, u64, vp, vp, C.POINTER(C.c_int32), vp]
    lib.stag_kmeans.restype = C.c_int
    lib.stag_kmeans.argtypes = [vp, i64, i32, i32, u64, i32, vp, vp, vp, vp, C.POINTER(C.c_int32), vp]
    lib.stag_spectral_cluster.restype = C.c_int
    lib.stag_spectral_cluster.argtypes = [i64, vp, vp, vp, i64, i32, u64, vp, vp]
    lib.stag_e2lsh_hash.restype = C.c_int
    lib.stag_e2lsh_hash.argtypes = [vp, i64, i32, vp, vp, i32, i32, vp, vp, vp]
    pp = C.POINTER(LshParams)
    lib.stag_lsh_derive.restype = C.c_int
    lib.stag_lsh_derive.argtypes = [i64, f64, f64, pp, C.POINTER(LshShape)]
    lib.stag_lsh_index_create.restype = C.c_int
    lib.stag_lsh_index_create.argtypes = [vp, i64, i32, f64, f64, pp, C.POINTER(vp), vp]
    lib.stag_lsh_index_query.restype = C.c_int
    lib.stag_lsh_index_query.argtypes = [vp, vp, i64, vp, vp]
    lib.stag_lsh_index_query_ex.restype = C.c_int
    lib.stag_lsh_index_query_ex.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.stag_lsh_index_shape.restype = C.c_int
    lib.stag_lsh_index_shape.argtypes = [vp, C.POINTER(LshShape)]
    lib.stag_lsh_index_segment.restype = C.c_int
    lib.stag_lsh_index_segment.argtypes = [vp, i32, i32, C.POINTER(C.c_int64), vp, vp, vp]
    lib.stag_lsh_index_destroy.restype = None
    lib.stag_lsh_index_destroy.argtypes = [vp]
    lib.stag_simgraph_sample_tree.restype = C.c_int
    lib.stag_simgraph_sample_tree.argtypes = [vp, i64, i32, f64, i32, i32, i64, C.c_uint64, vp, vp, vp, vp, vp]
    lib.stag_simgraph_sample.restype = C.c_int
    lib.stag_simgraph_sample.argtypes = [vp, i64, i32, f64, i32, i32, i32, f64, pp, C.c_uint64, vp, vp, vp, vp, vp]
    lib.stag_server_create.restype = C.c_int
    lib.stag_server_create.argtypes = [C.c_size_t, i32, i64, i64, C.POINTER(vp)]
    lib.stag_server_add_dataset.restype = C.c_int
    lib.stag_server_add_dataset.argtypes = [vp, vp, i64, i32, f64, i32, C.POINTER(C.c_int32)]
    lib.stag_server_add_dataset_ex.restype = C.c_int
    lib.stag_server_add_dataset_ex.argtypes = [vp, vp, i64, i32, f64, u32, f64, pp, C.POINTER(C.c_int32)]
    lib.stag_server_submit.restype = C.c_int
    lib.stag_server_submit.argtypes = [vp, i32, vp, i64, vp, C.POINTER(C.c_uint64)]
    lib.stag_server_submit_ex.restype = C.c_int
    lib.stag_server_submit_ex.argtypes = [vp, i32, vp, i64, i32, i32, f64, vp, vp, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_uint64)]
    lib.stag_server_wait.restype = C.c_int
    lib.stag_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(f64)]
    lib.stag_server_poll.restype = C.c_int
    lib.stag_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_int), C.POINTER(f64)]
    lib.stag_server_stats.restype = C.c_int
    lib.stag_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.stag_server_destroy.restype = None
    lib.stag_server_destroy.argtypes = [vp]
    lib.stag_kde_lsh.restype = C.c_int
    lib.stag_kde_lsh.argtypes = [vp, i64, vp, i64, i32, f64, f64, pp, vp, vp]
    lib.stag_e2lsh_table_create.restype = C.c_int
    lib.stag_e2lsh_table_create.argtypes = [vp, i64, i32, vp, vp, i32, i32, C.POINTER(vp), vp]
    lib.stag_e2lsh_table_count.restype = C.c_int
    lib.stag_e2lsh_table_count.argtypes = [vp, vp, i64, vp, vp]
    lib.stag_e2lsh_table_neighbours.restype = C.c_int
    lib.stag_e2lsh_table_neighbours.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.stag_e2lsh_table_destroy.restype = None
    lib.stag_e2lsh_table_destroy.argtypes = [vp]
    _lib = lib
    return lib


def declared_symbols() -> list[str]:
    """Function names declared in include/stag_kde.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stag_[a-z0-9_]+)\s*\(", txt)))


def check(status: int, what: str = ""):
    if status != STAG_OK:
        msg = load().stag_last_error().decode(errors="replace")
        raise StagError(status, f"{what}: {msg}" if what else msg)


def last_error() -> str:
    return load().stag_last_error().decode(errors="replace")


def _torch():
    import torch
    return torch


def _stream_handle(dev):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _need(t, dtype, ndim, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dims, got {tuple(t.shape)}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def collision_probability(c: float, K: int = 1, L: int = 1) -> float:
    return float(load().stag_e2lsh_collision_probability(float(c), int(K), int(L)))


def kde_exact(X, Q, a: float, form: str = "fp32", normalize: bool = False, return_bound: bool = False,
              S_out=None, bound_out=None, kernel: str = "gaussian", eps: float = 0.0, check_finite: bool = False):
    """S(q) = sum_i k(||q - x_i||) for every row q of Q (float64 [m]); kernel
    "gaussian" exp(-a r^2) (default), "exponential" exp(-a r) or "logistic"
    4/(2 + e^{ar} + e^{-ar}).  form "auto" takes the cheapest arithmetic form
    whose a-priori bound is <= eps.  check_finite rejects NaN/Inf inputs.
    With return_bound also the per-result relative error bound."""
    torch = _torch()
    _need(X, torch.float32, 2, "X")
    _need(Q, torch.float32, 2, "Q")
    if X.shape[1] != Q.shape[1]:
        raise ValueError("X and Q must have the same number of columns")
    if kernel not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}")
    n, d = X.shape
    m = Q.shape[0]
    S = S_out if S_out is not None else torch.empty(m, dtype=torch.float64, device=X.device)
    B = None
    if return_bound:
        B = bound_out if bound_out is not None else torch.empty(m, dtype=torch.float64, device=X.device)
    flags = (NORMALIZE if normalize else 0) | (CHECK_FINITE if check_finite else 0)
    if kernel == "gaussian":
        st = load().stag_kde_exact(_ptr(X), n, _ptr(Q), m, d, float(a), float(eps), FORMS[form], flags, _ptr(S),
                                   _ptr(B), _stream_handle(X.device))
        check(st, "stag_kde_exact")
    else:
        st = load().stag_kde_exact_kernel(_ptr(X), n, _ptr(Q), m, d, KERNELS[kernel], float(a), float(eps),
                                          FORMS[form], flags, _ptr(S), _ptr(B), _stream_handle(X.device))
        check(st, "stag_kde_exact_kernel")
    return (S, B) if return_bound else S


def kde_random_sample(X, Q, a: float, samples: int, seed: int = 0, form: str = "fp32", return_bound: bool = False,
                      return_indices: bool = False):
    """Random-sampling estimate (n/s) sum_r exp(-a ||q - x_{j_r}||^2) of S(q)
    for every row of Q (float64 [m]); optionally the per-result bound and the
    sampled indices (int64 [samples])."""
    torch = _torch()
    _need(X, torch.float32, 2, "X")
    _need(Q, torch.float32, 2, "Q")
    if X.shape[1] != Q.shape[1]:
        raise ValueError("X and Q must have the same number of columns")
    n, d = X.shape
    m = Q.shape[0]
    S = torch.empty(m, dtype=torch.float64, device=X.device)
    B = torch.empty(m, dtype=torch.float64, device=X.device) if return_bound else None
    I = torch.empty(int(samples), dtype=torch.int64, device=X.device) if return_indices else None
    st = load().stag_kde_random_sample(_ptr(X), n, _ptr(Q), m, d, float(a), int(samples),
                                       int(seed) & 0xFFFFFFFFFFFFFFFF, FORMS[form], _ptr(S), _ptr(B), _ptr(I),
                                       _stream_handle(X.device))
    check(st, "stag_kde_random_sample")
    out = (S,)
    if return_bound:
        out += (B,)
    if return_indices:
        out += (I,)
    return out if len(out) > 1 else S


def rs_sample_size(eps: float, mu: float, m: int, delta: float) -> int:
    return int(load().stag_rs_sample_size(float(eps), float(mu), int(m), float(delta)))


def e2lsh_hash(X, G, b, K: int, L: int, want_codes: bool = True, want_keys: bool = True):
    """codes [n][L][K] int32 and keys [n][L] (int64 tensor holding the uint64 bits)."""
    torch = _torch()
    _need(X, torch.float32, 2, "X")
    _need(G, torch.float32, 2, "G")
    _need(b, torch.float64, 1, "b")
    n, d = X.shape
    if G.shape != (L * K, d) or b.shape[0] != L * K:
        raise ValueError("G must be [L*K][d] and b [L*K]")
    codes = torch.empty((n, L, K), dtype=torch.int32, device=X.device) if want_codes else None
    keys = torch.empty((n, L), dtype=torch.int64, device=X.device) if want_keys else None
    st = load().stag_e2lsh_hash(_ptr(X), n, d, _ptr(G), _ptr(b), K, L, _ptr(codes), _ptr(keys),
                                _stream_handle(X.device))
    check(st, "stag_e2lsh_hash")
    return codes, keys


def _lsh_params(min_mu=0.0, k1=0, k2_constant=0.0, p_offset=0, seed=0, flags=0, G0=None, b=None):
    return LshParams(float(min_mu), int(k1), float(k2_constant), int(p_offset), int(seed) & 0xFFFFFFFFFFFFFFFF,
                     int(flags), None if G0 is None else G0.data_ptr(), None if b is None else b.data_ptr())


def lsh_derive(n: int, a: float, eps: float = 0.5, **kw) -> dict:
    """Derived CKNS shape (host only): dict(J, L, K, K1, mu_min)."""
    prm = _lsh_params(**kw)
    sh = LshShape()
    check(load().stag_lsh_derive(int(n), float(a), float(eps), C.byref(prm), C.byref(sh)), "stag_lsh_derive")
    return dict(J=sh.J, L=sh.L, K=sh.K, K1=sh.K1, mu_min=sh.mu_min)


class LshIndex:
    """CKNS index over device data X (fp32 [n][d]); see include/stag_kde.h."""

    def __init__(self, X, a: float, eps: float = 0.5, G0=None, b=None, **kw):
        torch = _torch()
        _need(X, torch.float32, 2, "X")
        if G0 is not None:
            _need(G0, torch.float32, G0.dim(), "G0")
            _need(b, torch.float64, b.dim(), "b")
        self._keep = (G0, b)
        prm = _lsh_params(G0=G0, b=b, **kw)
        h = C.c_void_p()
        self.device = X.device
        st = load().stag_lsh_index_create(_ptr(X), X.shape[0], X.shape[1], float(a), float(eps), C.byref(prm),
                                          C.byref(h), _stream_handle(X.device))
        check(st, "stag_lsh_index_create")
        self._h = h
        self.d = X.shape[1]
        sh = LshShape()
        check(load().stag_lsh_index_shape(self._h, C.byref(sh)))
        self.shape = dict(J=sh.J, L=sh.L, K=sh.K, K1=sh.K1, mu_min=sh.mu_min)

    def query(self, Q, stats: bool = False):
        torch = _torch()
        _need(Q, torch.float32, 2, "Q")
        if Q.shape[1] != self.d:
            raise ValueError("Q has the wrong number of columns")
        m = Q.shape[0]
        S = torch.empty(m, dtype=torch.float64, device=Q.device)
        if not stats:
            check(load().stag_lsh_index_query(self._h, _ptr(Q), m, _ptr(S), _stream_handle(Q.device)),
                  "stag_lsh_index_query")
            return S
        K1 = self.shape["K1"]
        cp = torch.empty((m, K1), dtype=torch.float64, device=Q.device)
        nc = torch.empty(m, dtype=torch.int64, device=Q.device)
        na = torch.empty(m, dtype=torch.int64, device=Q.device)
        check(load().stag_lsh_index_query_ex(self._h, _ptr(Q), m, _ptr(S), _ptr(cp), _ptr(nc), _ptr(na),
                                             _stream_handle(Q.device)), "stag_lsh_index_query_ex")
        return S, dict(S_copies=cp, n_cand=nc, n_acc=na)

    def segment(self, t: int, i: int):
        """(members, keys) of copy t, level i as numpy arrays (host)."""
        import numpy as np
        cnt = C.c_int64()
        check(load().stag_lsh_index_segment(self._h, t, i, C.byref(cnt), None, None, _stream_handle(self.device)))
        mem = np.empty(cnt.value, dtype=np.int32)
        keys = np.empty((cnt.value, self.shape["L"]), dtype=np.uint64)
        check(load().stag_lsh_index_segment(self._h, t, i, C.byref(cnt), mem.ctypes.data_as(C.c_void_p),
                                            keys.ctypes.data_as(C.c_void_p), _stream_handle(self.device)))
        return mem, keys

    def close(self):
        if getattr(self, "_h", None):
            load().stag_lsh_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class E2LSHTable:
    """E2LSH hash table over device points X (fp32 [n][d]) with projections
    G (fp32 [L*K][d]) and offsets b (f64 [L*K]); see include/stag_kde.h."""

    def __init__(self, X, G, b, K: int, L: int):
        torch = _torch()
        _need(X, torch.float32, 2, "X")
        _need(G, torch.float32, 2, "G")
        _need(b, torch.float64, 1, "b")
        if G.shape != (L * K, X.shape[1]) or b.shape[0] != L * K:
            raise ValueError("G must be [L*K][d] and b [L*K]")
        h = C.c_void_p()
        self.device = X.device
        check(load().stag_e2lsh_table_create(_ptr(X), X.shape[0], X.shape[1], _ptr(G), _ptr(b), int(K), int(L),
                                             C.byref(h), _stream_handle(X.device)), "stag_e2lsh_table_create")
        self._h = h
        self.d = X.shape[1]

    def near_neighbours(self, Q):
        """(offsets int64 [m+1], idx int32 [offsets[m]]): query q's neighbours
        are idx[offsets[q]:offsets[q+1]]."""
        torch = _torch()
        _need(Q, torch.float32, 2, "Q")
        if Q.shape[1] != self.d:
            raise ValueError("Q has the wrong number of columns")
        m = Q.shape[0]
        off = torch.empty(m + 1, dtype=torch.int64, device=Q.device)
        check(load().stag_e2lsh_table_count(self._h, _ptr(Q), m, _ptr(off), _stream_handle(Q.device)),
              "stag_e2lsh_table_count")
        total = int(off[m].item())
        idx = torch.empty(max(total, 1), dtype=torch.int32, device=Q.device)
        if total > 0:
            check(load().stag_e2lsh_table_neighbours(self._h, _ptr(Q), m, _ptr(off), _ptr(idx),
                                                     _stream_handle(Q.device)), "stag_e2lsh_table_neighbours")
        return off, idx[:total]

    def close(self):
        if getattr(self, "_h", None):
            load().stag_e2lsh_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kde_lsh(X, Q, a: float, eps: float = 0.5, G0=None, b=None, **kw):
    """One-shot CKNS estimate (index create + query + destroy)."""
    torch = _torch()
    _need(X, torch.float32, 2, "X")
    _need(Q, torch.float32, 2, "Q")
    prm = _lsh_params(G0=G0, b=b, **kw)
    S = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
    check(load().stag_kde_lsh(_ptr(X), X.shape[0], _ptr(Q), Q.shape[0], X.shape[1], float(a), float(eps),
                              C.byref(prm), _ptr(S), _stream_handle(X.device)), "stag_kde_lsh")
    return S


def draws_per_node(n: int, samples_per_node: int = 0) -> int:
    """Draws per node the edge samplers take (the library's rule: 0 means
    ceil(log2 n)); raises for arguments the samplers reject."""
    s = load().stag_simgraph_draws_per_node(int(n), int(samples_per_node))
    if s < 1:
        raise StagError(STAG_E_INVAL, f"samples_per_node = {samples_per_node} outside [0, 64] or n < 1")
    return s


def simgraph_sample(X, a: float, samples_per_node: int = 0, mode: str = "exact", form: str = "fp32",
                    eps: float = 0.5, seed: int = 0, G0=None, b=None, lsh_seed: int = 0, **lsh_kw):
    """Edge sample of the kernel similarity graph: (src, dst, w, deg) tensors.
    seed drives the draws; lsh_seed and lsh_kw (k1, k2_constant, p_offset,
    min_mu, flags) the CKNS index of the "lsh" mode."""
    torch = _torch()
    _need(X, torch.float32, 2, "X")
    n, d = X.shape
    s = draws_per_node(n, samples_per_node)
    src = torch.empty(n * s, dtype=torch.int64, device=X.device)
    dst = torch.empty(n * s, dtype=torch.int64, device=X.device)
    w = torch.empty(n * s, dtype=torch.float64, device=X.device)
    deg = torch.empty(n, dtype=torch.float64, device=X.device)
    prm = _lsh_params(G0=G0, b=b, seed=lsh_seed, **lsh_kw)
    st = load().stag_simgraph_sample(_ptr(X), n, d, float(a), s, {"exact": 0, "lsh": 1}[mode], FORMS[form],
                                     float(eps), C.byref(prm), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(src), _ptr(dst),
                                     _ptr(w), _ptr(deg), _stream_handle(X.device))
    check(st, "stag_simgraph_sample")
    return src, dst, w, deg


def simgraph_sample_tree(X, a: float, samples_per_node: int = 0, est_samples: int = 32, degree_samples: int = 1024,
                         seed: int = 0):
    """Edge sample through the KDE tree with random-sampling node estimates:
    (src, dst, w, deg) tensors."""
    torch = _torch()
    _need(X, torch.float32, 2, "X")
    n, d = X.shape
    s = draws_per_node(n, samples_per_node)
    src = torch.empty(n * s, dtype=torch.int64, device=X.device)
    dst = torch.empty(n * s, dtype=torch.int64, device=X.device)
    w = torch.empty(n * s, dtype=torch.float64, device=X.device)
    deg = torch.empty(n, dtype=torch.float64, device=X.device)
    st = load().stag_simgraph_sample_tree(_ptr(X), n, d, float(a), s, int(est_samples), int(degree_samples),
                                          int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(src), _ptr(dst), _ptr(w), _ptr(deg),
                                          _stream_handle(X.device))
    check(st, "stag_simgraph_sample_tree")
    return src, dst, w, deg


def _edges(src, dst, w):
    torch = _torch()
    _need(src, torch.int64, 1, "src")
    _need(dst, torch.int64, 1, "dst")
    _need(w, torch.float64, 1, "w")
    if not (src.shape == dst.shape == w.shape):
        raise ValueError("src, dst and w must have the same length")
    return src.shape[0]


def spectral_embedding(n: int, src, dst, w, k: int, tol: float = 1e-8, max_iter: int = 300, seed: int = 0):
    """Bottom-k eigenpairs of the normalised Laplacian of the edge-list graph:
    (eigenvalues float64 [k] ascending, U float64 [n][k], filter steps)."""
    torch = _torch()
    E = _edges(src, dst, w)
    lam = torch.empty(k, dtype=torch.float64, device=src.device)
    U = torch.empty((n, k), dtype=torch.float64, device=src.device)
    it = C.c_int32(0)
    st = load().stag_spectral_embedding(int(n), _ptr(src), _ptr(dst), _ptr(w), E, int(k), float(tol), int(max_iter),
                                        int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(lam), _ptr(U), C.byref(it),
                                        _stream_handle(src.device))
    check(st, "stag_spectral_embedding")
    return lam, U, int(it.value)


def kmeans(P, k: int, seed: int = 0, max_iter: int = 300, init=None):
    """k-means of the rows of P (float64 [n][dim]): (labels int32 [n],
    centroids float64 [k][dim], rounds, seed indices int64 [k])."""
    torch = _torch()
    _need(P, torch.float64, 2, "P")
    n, dim = P.shape
    if init is not None:
        _need(init, torch.float64, 2, "init")
        if tuple(init.shape) != (k, dim):
            raise ValueError("init must be [k][dim]")
    labels = torch.empty(n, dtype=torch.int32, device=P.device)
    Cm = torch.empty((k, dim), dtype=torch.float64, device=P.device)
    seeds = torch.empty(k, dtype=torch.int64, device=P.device)
    it = C.c_int32(0)
    st = load().stag_kmeans(_ptr(P), n, dim, int(k), int(seed) & 0xFFFFFFFFFFFFFFFF, int(max_iter), _ptr(init),
                            _ptr(labels), _ptr(Cm), _ptr(seeds), C.byref(it), _stream_handle(P.device))
    check(st, "stag_kmeans")
    return labels, Cm, int(it.value), seeds


def spectral_cluster(n: int, src, dst, w, k: int, seed: int = 0):
    """Cluster labels (int32 [n]) of the edge-list graph: embedding + k-means."""
    torch = _torch()
    E = _edges(src, dst, w)
    labels = torch.empty(n, dtype=torch.int32, device=src.device)
    st = load().stag_spectral_cluster(int(n), _ptr(src), _ptr(dst), _ptr(w), E, int(k),
                                      int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(labels), _stream_handle(src.device))
    check(st, "stag_spectral_cluster")
    return labels


class Server:
    """Continuous-batching KDE server over resident data sets and CKNS
    indexes (see include/stag_kde.h).

    submit() returns a ticket; wait(ticket) returns (S, status, latency_s)
    and, for requests submitted with bound=True, bound_of(ticket) the
    per-result bounds afterwards."""

    def __init__(self, budget_bytes: int = 0, n_streams: int = 0, max_batch_queries: int = 0,
                 chunk_queries: int = 0):
        h = C.c_void_p()
        check(load().stag_server_create(int(budget_bytes), int(n_streams), int(max_batch_queries),
                                        int(chunk_queries), C.byref(h)), "stag_server_create")
        self._h = h
        self._live = {}
        self._bounds = {}

    def add_dataset(self, X, a: float, form="fp32", lsh: dict | None = None) -> int:
        """form: one form name or a list of names to keep resident (may be
        empty with an index); lsh: None, or dict(eps=..., plus stag_lsh_params
        fields k1, k2_constant, p_offset, min_mu, seed, flags) for a resident
        CKNS index."""
        torch = _torch()
        _need(X, torch.float32, 2, "X")
        forms = [form] if isinstance(form, str) else list(form)
        mask = 0
        for f in forms:
            mask |= 1 << FORMS[f]
        torch.cuda.current_stream(X.device).synchronize()  # X must be complete before the server reads it
        i = C.c_int32()
        if lsh is None:
            prm, eps = None, 0.0
        else:
            kw = dict(lsh)
            eps = float(kw.pop("eps", 0.5))
            prm = C.byref(_lsh_params(**kw))
        check(load().stag_server_add_dataset_ex(self._h, _ptr(X), X.shape[0], X.shape[1], float(a), mask, eps, prm,
                                                C.byref(i)), "stag_server_add_dataset_ex")
        return int(i.value)

    def submit(self, dataset: int, Q, S_out=None, form: str | None = None, eps: float = 0.0, lsh: bool = False,
               bound: bool = False) -> int:
        """Exact request in `form` (None: the data set's first resident form;
        "auto": chosen from eps), or an LSH request (lsh=True)."""
        torch = _torch()
        _need(Q, torch.float32, 2, "Q")
        S = S_out if S_out is not None else torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
        B = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device) if bound else None
        torch.cuda.current_stream(Q.device).synchronize()  # Q must be complete before the server reads it
        t = C.c_uint64()
        if form is None and not lsh and not bound:
            check(load().stag_server_submit(self._h, int(dataset), _ptr(Q), Q.shape[0], _ptr(S), C.byref(t)),
                  "stag_server_submit")
            self._live[t.value] = (Q, S, None, None)
            return int(t.value)
        chosen = C.c_int32(-1)
        kind = 1 if lsh else 0
        fcode = FORMS["fp32" if form is None else form] if not lsh else 0
        check(load().stag_server_submit_ex(self._h, int(dataset), _ptr(Q), Q.shape[0], kind, fcode, float(eps),
                                           _ptr(S), _ptr(B), C.byref(chosen), C.byref(t)), "stag_server_submit_ex")
        name = None if chosen.value < 0 else next(k for k, v in FORMS.items() if v == chosen.value)
        self._live[t.value] = (Q, S, B, name)
        return int(t.value)

    def form_of(self, ticket: int):
        """The form a pending request runs in (None for LSH or the plain
        submit)."""
        return self._live[ticket][3]

    def bound_of(self, ticket: int):
        return self._bounds.pop(ticket, None)

    def wait(self, ticket: int):
        st, lat = C.c_int(), C.c_double()
        check(load().stag_server_wait(self._h, ticket, C.byref(st), C.byref(lat)), "stag_server_wait")
        Q, S, B, _ = self._live.pop(ticket)
        if B is not None:
            self._bounds[ticket] = B
        return S, int(st.value), float(lat.value)

    def poll(self, ticket: int):
        done, st, lat = C.c_int32(), C.c_int(), C.c_double()
        check(load().stag_server_poll(self._h, ticket, C.byref(done), C.byref(st), C.byref(lat)), "stag_server_poll")
        return bool(done.value), int(st.value), float(lat.value)

    def stats(self) -> dict:
        s = ServerStats()
        check(load().stag_server_stats(self._h, C.byref(s)), "stag_server_stats")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().stag_server_destroy(self._h)
            self._h = None
            self._live.clear()
            self._bounds.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
