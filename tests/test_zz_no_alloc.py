"""stag_kde_exact_noalloc, the exact Gaussian density without device
allocation, against stag_kde_exact on the same inputs, through the C ABI.

Both entry points share their kernels, so results must agree bit for bit
(S and the per-result bound).  Two calls follow each other with the second on
a smaller input (the scratch keeps the first call's contents), one call
takes the underflow rescue, and the default stream-ordered memory pool shows
no allocation made during the calls."""
import ctypes as C

import numpy as np
import pytest

import synth
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu

HIP_POOL_USED_HIGH = 8  # hipMemPoolAttrUsedMemHigh
HIP_POOL_USED_CURRENT = 7  # hipMemPoolAttrUsedMemCurrent


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    return s.load()


def _hip():
    hip = C.CDLL("libamdhip64.so.7")  # the runtime already loaded in this process
    pool = C.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(C.byref(pool), 0) == 0
    return hip, pool


def _pool_attr(hip, pool, attr):
    v = C.c_uint64(0)
    assert hip.hipMemPoolGetAttribute(pool, attr, C.byref(v)) == 0
    return v.value


def _both(lib, X, Q, a, form, normalize=False):
    import torch
    from paper_2407_07096_amd import _lib as L
    Xd, Qd = to_dev(X), to_dev(Q)
    n, d = X.shape
    m = Q.shape[0]
    flags = L.NORMALIZE if normalize else 0
    stream = torch.cuda.current_stream().cuda_stream
    S0 = torch.empty(m, dtype=torch.float64, device=Xd.device)
    B0 = torch.empty_like(S0)
    S1 = torch.full_like(S0, -1.0)
    B1 = torch.full_like(S0, -1.0)
    st = lib.stag_kde_exact(Xd.data_ptr(), n, Qd.data_ptr(), m, d, a, 0.0, L.FORMS[form], flags, S0.data_ptr(),
                            B0.data_ptr(), C.c_void_p(stream))
    assert st == 0, lib.stag_last_error()
    torch.cuda.synchronize()
    hip, pool = _hip()
    used0 = _pool_attr(hip, pool, HIP_POOL_USED_CURRENT)
    zero = C.c_uint64(0)
    assert hip.hipMemPoolSetAttribute(pool, HIP_POOL_USED_HIGH, C.byref(zero)) == 0  # reset to the current use
    st = lib.stag_kde_exact_noalloc(Xd.data_ptr(), n, Qd.data_ptr(), m, d, a, L.FORMS[form], flags, S1.data_ptr(),
                                    B1.data_ptr(), C.c_void_p(stream))
    assert st == 0, lib.stag_last_error()
    torch.cuda.synchronize()
    high = _pool_attr(hip, pool, HIP_POOL_USED_HIGH)
    assert high <= used0, (high, used0)  # nothing was taken from the stream-ordered pool
    return S0.cpu().numpy(), B0.cpu().numpy(), S1.cpu().numpy(), B1.cpu().numpy()


@pytest.mark.parametrize("form", ["fp16_split", "fp32", "bf16_split3", "fp16_centred", "fp16_adaptive"])
def test_noalloc_matches_allocating_call_twice(lib, orc, form):
    # first call: larger input; second: smaller and ragged (d not a multiple of 16)
    X, Q, _ = synth.config_points(2, n=20000, m=3000)
    announce(f"noalloc first call n=20000 m=3000 d=64 form={form}")
    S0, B0, S1, B1 = _both(lib, X, Q, 0.05, form)
    assert np.array_equal(S0, S1) and np.array_equal(B0, B1)
    rng = np.random.default_rng(5)
    X2 = rng.normal(size=(4099, 40)).astype(np.float32)
    Q2 = (X2[rng.integers(0, 4099, size=301)] + 0.2 * rng.normal(size=(301, 40))).astype(np.float32)
    announce(f"noalloc second call n=4099 m=301 d=40 form={form}")
    S0, B0, S1, B1 = _both(lib, X2, Q2, 0.02, form, normalize=True)
    assert np.array_equal(S0, S1) and np.array_equal(B0, B1)
    ref = orc.kde_exact(X2, Q2, 0.02) / 4099.0
    err = np.abs(S1 - ref) / ref
    assert np.all(err <= B1)


@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_noalloc_wide_rows(lib, orc, form):
    # d = 784: the wide tiles (queries staged in LDS, data rows streamed)
    X = synth.sparse_uniform(3000, 784, 1004)
    Q = np.ascontiguousarray(X[::30])
    announce(f"noalloc wide n=3000 m={Q.shape[0]} d=784 form={form}")
    S0, B0, S1, B1 = _both(lib, X, Q, 1e-3, form)
    assert np.array_equal(S0, S1) and np.array_equal(B0, B1)
    ref = orc.kde_exact(X, Q, 1e-3)
    assert np.all(np.abs(S1 - ref) / ref <= B1)


def test_noalloc_underflow_rescue(lib, orc):
    # queries far from the data take the rescue passes (max pass, shifted
    # offsets), whose buffers also live in the scratch
    rng = np.random.default_rng(31)
    d = 32
    X = rng.normal(size=(5000, d)).astype(np.float32)
    far = (X[:64] + 4.0 * rng.normal(size=(64, d)).astype(np.float32)).astype(np.float32)
    Q = np.concatenate([X[100:164], far]).astype(np.float32)
    announce("noalloc rescue m=128 d=32 a=1")
    S0, B0, S1, B1 = _both(lib, X, Q, 1.0, "fp16_split")
    assert np.array_equal(S0, S1) and np.array_equal(B0, B1)
    ref = orc.kde_exact(X, Q, 1.0)
    assert np.sum(ref < 2.0 ** -60) > 10
    ok = ref > 1e-300
    assert np.all(np.abs(S1[ok] - ref[ok]) / ref[ok] <= B1[ok])


def test_noalloc_rejects_before_launch(lib):
    from paper_2407_07096_amd import _lib as L
    fake = C.c_void_p(0x1000)  # never dereferenced: every check fails first
    null = C.c_void_p(0)
    st = lib.stag_kde_exact_noalloc(fake, 3_000_000, fake, 300_000, 64, 0.1, 2, 0, fake, null, null)
    assert st == L.STAG_E_INVAL and b"scratch" in lib.stag_last_error()
    st = lib.stag_kde_exact_noalloc(fake, 100, fake, 100, 8, 0.1, L.FORMS["auto"], 0, fake, null, null)
    assert st == L.STAG_E_UNSUPPORTED
    st = lib.stag_kde_exact_noalloc(fake, 100, fake, 100, 8, 0.1, 0, L.CHECK_FINITE, fake, null, null)
    assert st == L.STAG_E_UNSUPPORTED
