"""GPU parity of the fp16 centred form of the exact Gaussian density
(Sec. "Kernel Density Estimation": the all-pairs sum, here with the data
grouped around centres and one fp16 matrix-core product per pair) against
the FP64 oracle, through the C ABI.

The form's per-result bound is the worst case of its two fp16 roundings per
product (relative 2^-11 each, all aligned), so every result must lie within
it; the measured errors are far smaller where many terms make up a sum, and
the tests print them.  At the n = 2,000,000, m = 200,000, d = 128 workload
the form measures 5.4e-5 at most and 1.1e-6 at the median over 1,000
sampled queries: it does not meet 1e-5 on every query there, and the tests
hold it to twice and ten times those figures as regression guards.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, rel_err, to_dev

pytestmark = pytest.mark.gpu

FORM = "fp16_centred"


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def _run(stag, X, Q, a, **kw):
    import torch
    S, B = stag.kde_exact(to_dev(X), to_dev(Q), a, form=FORM, return_bound=True, **kw)
    torch.cuda.synchronize()
    return S.cpu().numpy(), B.cpu().numpy()


def test_config1_full(stag, orc):
    X, Q, _ = synth.config_points(1)
    announce("fp16 centred config1 n=m=1000 d=10 a=0.5")
    ref = orc.kde_exact(X, Q, 0.5)
    S, B = _run(stag, X, Q, 0.5)
    err = rel_err(S, ref)
    print(f"[measured] fp16 centred config1: max rel err {err.max():.3e}, median {np.median(err):.3e}, "
          f"max bound {B.max():.3e}", flush=True)
    assert np.all(err <= B), (err.max(), B.min())
    Sx, Bx = _run(stag, X, X, 0.5)
    assert np.all(rel_err(Sx, orc.kde_exact(X, X, 0.5)) <= Bx)


@pytest.mark.parametrize("a", [0.01, 0.1, 0.3, 1.0])
def test_config2_reduced(stag, orc, a):
    X, Q, _ = synth.config_points(2, n=9000, m=300)
    announce(f"fp16 centred config2-reduced n=9000 m=300 d=64 a={a}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a)
    err = rel_err(S, ref)
    print(f"[measured] fp16 centred config2 a={a}: max rel err {err.max():.3e}, max bound {B.max():.3e}",
          flush=True)
    assert np.all(err <= B), (err.max(), B.min())
    assert np.all(np.isfinite(S))


@pytest.mark.parametrize("shift", [0.0, 100.0, 3000.0])
def test_translation(stag, orc, shift):
    """The products see q - c_g and x - c_g only, so a common translation of
    X and Q (up to 3000 per coordinate) leaves the bound and the error where
    they were."""
    X, Q, _ = synth.config_points(1)
    X = (X.astype(np.float64) + shift).astype(np.float32)
    Q = (Q.astype(np.float64) + shift).astype(np.float32)
    announce(f"fp16 centred translation shift={shift}")
    ref = orc.kde_exact(X, Q, 0.05)
    S, B = _run(stag, X, Q, 0.05)
    err = rel_err(S, ref)
    print(f"[measured] fp16 centred shift {shift}: max rel err {err.max():.3e}, max bound {B.max():.3e}",
          flush=True)
    assert np.all(err <= B)
    assert B.max() < 2e-2


@pytest.mark.parametrize("n,m,d", [(1, 1, 1), (2, 3, 3), (31, 129, 5), (33, 130, 16), (100, 257, 100),
                                   (4097, 64, 7), (5000, 300, 128), (3000, 200, 160), (5000, 130, 256),
                                   (20000, 512, 40)])
def test_shapes(stag, orc, n, m, d):
    """Ragged sizes (single rows, groups smaller than a tile, several chunks,
    one and two query blocks per wave, the largest tiled dimension), clustered
    data far from the origin; deterministic and independent of the other
    queries."""
    rng = np.random.default_rng(n + 13 * d + m)
    means = rng.uniform(-20, 20, size=(4, d))
    X = (means[rng.integers(0, 4, size=n)] + rng.normal(size=(n, d))).astype(np.float32)
    Q = (X[rng.integers(0, n, size=m)] + 0.5 * rng.normal(size=(m, d))).astype(np.float32)
    a = 0.3 / d
    announce(f"fp16 centred n={n} m={m} d={d}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a)
    err = rel_err(S, ref)
    assert np.all(err <= B), (err.max(), B.max())
    S2, _ = _run(stag, X, Q, a)
    assert np.array_equal(S, S2)
    j = min(5, m - 1)
    S3, _ = _run(stag, X, Q[j:j + 1], a)
    assert S3[0] == S[j]


def test_underflow_rescue(stag, orc):
    """Queries far from the data (sums down to ~1e-270) go through the max
    pass and the shifted second pass; the near ones are untouched (the same
    bits as in a batch without the far ones)."""
    rng = np.random.default_rng(31)
    d = 32
    X = rng.normal(size=(5000, d)).astype(np.float32)
    near = (X[:200] + 0.1 * rng.normal(size=(200, d))).astype(np.float32)
    far = (X[200:328] + rng.uniform(3.0, 6.0, size=(128, 1)).astype(np.float32)
           * rng.normal(size=(128, d)).astype(np.float32) / np.sqrt(d) * 4.0).astype(np.float32)
    Q = np.concatenate([near, far]).astype(np.float32)
    a = 1.0
    announce(f"fp16 centred underflow rescue m={len(Q)} d={d} a={a}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a)
    ok = ref > 1e-300
    err = rel_err(S[ok], ref[ok])
    print(f"[measured] fp16 centred rescue: queries below 2^-60: {int(np.sum(ref < 2.0 ** -60))}, "
          f"max rel err {err.max():.3e}", flush=True)
    assert np.sum(ref < 1e-38) > 20
    assert np.all(err <= B[ok]), (err.max(), B[ok].min())
    Sn, _ = _run(stag, X, near, a)
    assert np.array_equal(Sn, S[:200])
    j = 200 + int(np.argmin(ref[200:]))
    S1, _ = _run(stag, X, Q[j:j + 1], a)
    assert S1[0] == S[j]


def test_fp16_range(stag, orc):
    """Outside fp16's range the results are NaN: a query whose operand
    2 a log2(e) (q - c) reaches 65520 (that query only), or a data row with
    |x_j - c_j| >= 65520 (every result)."""
    rng = np.random.default_rng(5)
    d = 8
    X = rng.normal(size=(300, d)).astype(np.float32)
    Q = rng.normal(size=(40, d)).astype(np.float32)
    Q[7, 3] = 1.0e7  # 2 a log2(e) 1e7 ~ 2.9e6 at a = 0.1
    S, B = _run(stag, X, Q, 0.1)
    ref = orc.kde_exact(X, Q, 0.1)
    assert np.isnan(S[7])
    keep = np.arange(40) != 7
    assert np.all(rel_err(S[keep], ref[keep]) <= B[keep])
    X2 = X.copy()
    X2[11, 0] = 1.0e6
    S2, _ = _run(stag, X2, Q[:5], 0.1)
    assert np.all(np.isnan(S2))


def test_config3_full_size_sampled(stag, orc):
    """n = 2,000,000, m = 200,000, d = 128, a = 0.01: full launch, oracle on
    the same 1,000 sampled queries as the other forms; every result within its
    bound, the largest error below 1e-4 and the median below 1e-5."""
    import torch
    X, Q, _ = synth.config_points(3)
    rng = np.random.default_rng(2003)
    idx = np.sort(rng.choice(Q.shape[0], size=1000, replace=False))
    ref = orc.kde_exact(X, Q[idx], 0.01)
    announce("fp16 centred config3 full n=2e6 m=2e5 d=128 a=0.01")
    S, B = stag.kde_exact(to_dev(X), to_dev(Q), 0.01, form=FORM, return_bound=True)
    torch.cuda.synchronize()
    S, B = S.cpu().numpy(), B.cpu().numpy()
    err = rel_err(S[idx], ref)
    print(f"[measured] fp16 centred config3: max rel err {err.max():.3e}, median {np.median(err):.3e}, "
          f"max bound {B[idx].max():.3e}", flush=True)
    assert np.all(np.isfinite(S))
    assert np.all(err <= B[idx]), err.max()
    assert err.max() <= 1e-4 and np.median(err) <= 1e-5, (err.max(), np.median(err))


def test_config2_full_size_sampled(stag, orc):
    """n = m = 100,000, d = 64: full launch, oracle on 200 sampled queries,
    within the bound (the measured error is printed)."""
    X, Q, _ = synth.config_points(2)
    rng = np.random.default_rng(2002)
    idx = np.sort(rng.choice(Q.shape[0], size=200, replace=False))
    for a in (0.01, 0.1):
        ref = orc.kde_exact(X, Q[idx], a)
        announce(f"fp16 centred config2 full n=m=1e5 a={a}")
        S, B = _run(stag, X, Q, a)
        err = rel_err(S[idx], ref)
        print(f"[measured] fp16 centred config2 full a={a}: max rel err {err.max():.3e}", flush=True)
        assert np.all(err <= B[idx]), (a, err.max())
