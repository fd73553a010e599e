"""GPU parity of the exact kernel density (Sec. "Kernel Density Estimation")
against the FP64 oracle, through the C ABI.

Tolerance: the fp32 form must be within 1e-5 relative wherever the
exponent magnitudes allow it (a small enough that a(||q||^2+||x||^2) stays
moderate); every form must be within its own per-result bound on every query.
"""
import math

import numpy as np
import pytest

import synth
from tests.gpu_util import announce, rel_err, to_dev

pytestmark = pytest.mark.gpu

FORMS = ["fp32", "fp16_split", "bf16_split", "bf16_split3"]


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def _run(stag, X, Q, a, form, **kw):
    import torch
    S, B = stag.kde_exact(to_dev(X), to_dev(Q), a, form=form, return_bound=True, **kw)
    torch.cuda.synchronize()
    return S.cpu().numpy(), B.cpu().numpy()


@pytest.mark.parametrize("form", FORMS)
def test_config1_full(stag, orc, form):
    X, Q, _ = synth.config_points(1)
    announce(f"config1 n=m=1000 d=10 a=0.5 form={form}")
    ref = orc.kde_exact(X, Q, 0.5)
    S, B = _run(stag, X, Q, 0.5, form)
    err = rel_err(S, ref)
    print(f"[measured] config1 {form}: max rel err {err.max():.3e}", flush=True)
    assert np.all(err <= B), (err.max(), B.min())
    # the fp32 form centres every data tile, so its exponents carry a(||q - c||^2
    # + ||x - c||^2) instead of a(||q||^2 + ||x||^2) ~ 90 and it meets 1e-5;
    # the split forms keep the origin expansion (~1e-5 at this a)
    if form == "fp32":
        assert err.max() <= 1e-5
    else:
        assert err.max() <= 5e-5 if form != "bf16_split" else err.max() <= 5e-3
    # queries drawn from the data (self term present)
    Sx, Bx = _run(stag, X, X, 0.5, form)
    errx = rel_err(Sx, orc.kde_exact(X, X, 0.5))
    assert np.all(errx <= Bx)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("a", [0.01, 0.1, 0.3, 1.0])
def test_config2_reduced(stag, orc, form, a):
    X, Q, _ = synth.config_points(2, n=9000, m=300)
    announce(f"config2-reduced n=9000 m=300 d=64 a={a} form={form}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a, form)
    err = rel_err(S, ref)
    print(f"[measured] config2 a={a} {form}: max rel err {err.max():.3e}, min S {ref.min():.3e}", flush=True)
    assert np.all(err <= B), (err.max(), B.min())
    if a == 0.01 and form in ("fp32", "fp16_split", "bf16_split3"):
        assert err.max() <= 1e-5, err.max()


@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_underflow_rescue(stag, orc, form):
    # queries far from the data: their sums (down to ~1e-270) lie far below the
    # fp32 range of the tile's terms and are recomputed with shifted exponents;
    # near queries in the same batch are untouched (bit-identical to a batch
    # without the far ones), and a far query alone gives the same bits
    import torch
    rng = np.random.default_rng(31)
    d = 32
    X = rng.normal(size=(5000, d)).astype(np.float32)
    near = (X[:200] + 0.1 * rng.normal(size=(200, d))).astype(np.float32)
    far = (X[200:328] + rng.uniform(3.0, 6.0, size=(128, 1)).astype(np.float32)
           * rng.normal(size=(128, d)).astype(np.float32) / np.sqrt(d) * 4.0).astype(np.float32)
    Q = np.concatenate([near, far]).astype(np.float32)
    a = 1.0
    announce(f"underflow rescue m={len(Q)} d={d} a={a} form={form}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a, form)
    ok = ref > 1e-300
    err = rel_err(S[ok], ref[ok])
    print(f"[measured] rescue {form}: min S {ref.min():.3e}, queries below 2^-60: "
          f"{int(np.sum(ref < 2.0 ** -60))}, max rel err {err.max():.3e}", flush=True)
    assert np.sum(ref < 1e-38) > 20  # the case is exercised
    assert np.all(err <= B[ok]), (err.max(), B[ok].min())
    # near queries to 1e-4 (about four times what they measure at a = 1);
    # far ones (exponents near -900 in fp32 accumulators) to their bound only
    assert rel_err(S[:200], ref[:200]).max() <= 1e-4
    Sn, _ = _run(stag, X, near, a, form)
    assert np.array_equal(Sn, S[:200])
    j = 200 + int(np.argmin(ref[200:]))
    S1, _ = _run(stag, X, Q[j:j + 1], a, form)
    assert S1[0] == S[j]


@pytest.mark.parametrize("shift", [0.0, 100.0, 3000.0])
def test_centred_fp32_translation(stag, orc, shift):
    """The centred fp32 form expands each tile around its own centre, so a
    common translation of X and Q (here up to 3000 per coordinate, where
    a(||q||^2 + ||x||^2) ~ 5e7) leaves its accuracy unchanged: 1e-5 at
    config 1 for every shift, every result within its bound."""
    X, Q, _ = synth.config_points(1)
    X = (X.astype(np.float64) + shift).astype(np.float32)
    Q = (Q.astype(np.float64) + shift).astype(np.float32)
    announce(f"centred fp32 translation shift={shift}")
    ref = orc.kde_exact(X, Q, 0.5)
    S, B = _run(stag, X, Q, 0.5, "fp32")
    err = rel_err(S, ref)
    print(f"[measured] centred fp32 shift {shift}: max rel err {err.max():.3e}, max bound {B.max():.3e}", flush=True)
    assert np.all(err <= B) and err.max() <= 1e-5


@pytest.mark.parametrize("n,d", [(1, 1), (2, 3), (31, 5), (33, 16), (100, 100), (4097, 7), (5000, 256), (20000, 40)])
def test_centred_fp32_shapes(stag, orc, n, d):
    """Ragged sizes of the grouping (single rows, groups smaller than a tile,
    several chunks, the largest tiled dimension), clustered and far from the
    origin, against the oracle; deterministic and independent of the other
    queries."""
    import torch
    rng = np.random.default_rng(n + 13 * d)
    means = rng.uniform(-20, 20, size=(4, d))
    X = (means[rng.integers(0, 4, size=n)] + rng.normal(size=(n, d))).astype(np.float32)
    Q = (X[rng.integers(0, n, size=130)] + 0.5 * rng.normal(size=(130, d))).astype(np.float32)
    a = 0.3 / d
    announce(f"centred fp32 n={n} d={d}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a, "fp32")
    err = rel_err(S, ref)
    assert np.all(err <= B) and err.max() <= 1e-5, (err.max(), B.max())
    S2, _ = _run(stag, X, Q, a, "fp32")
    assert np.array_equal(S, S2)
    S3, _ = _run(stag, X, Q[5:6], a, "fp32")
    assert S3[0] == S[5]


def test_underflow_beyond_fp64(stag, orc):
    # a query whose true density is below the fp64 range returns 0 (as the
    # oracle's exp of its log-sum does); the rescue raises no error
    X = np.zeros((64, 4), dtype=np.float32)
    Q = np.full((1, 4), 30.0, dtype=np.float32)  # a D = 3600 -> e^-3600
    S, B = _run(stag, X, Q, 1.0, "fp32")
    assert S[0] == 0.0 and orc.kde_exact(X, Q, 1.0)[0] == 0.0


@pytest.mark.parametrize("n,m,d", [(1, 1, 1), (5, 3, 2), (33, 129, 17), (4097, 130, 100), (8193, 1, 256),
                                   (4096, 128, 16), (700, 257, 255)])
@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_ragged_shapes(stag, orc, n, m, d, form):
    rng = np.random.default_rng(n * 7 + m + d)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Q = (X[rng.integers(0, n, size=m)] + 0.3 * rng.normal(size=(m, d))).astype(np.float32)
    a = 0.5 / d
    announce(f"ragged n={n} m={m} d={d} form={form}")
    ref = orc.kde_exact(X, Q, a)
    S, B = _run(stag, X, Q, a, form)
    err = rel_err(S, ref)
    assert np.all(err <= B), (err.max(), B.min())
    assert err.max() <= 1e-5


def test_all_points_equal_query(stag):
    q = np.array([[0.5, -1.25, 2.0, 3.0]], np.float32)
    X = np.repeat(q, 5000, axis=0)
    for form in FORMS:
        S, B = _run(stag, X, q, 0.7, form)
        assert abs(S[0] - 5000.0) / 5000.0 <= B[0]


def test_normalize_flag(stag, orc):
    X, Q, _ = synth.config_points(1, n=500, m=64)
    S, _ = _run(stag, X, Q, 0.5, "fp32", normalize=True)
    assert np.all(rel_err(S, orc.kde_exact(X, Q, 0.5) / 500) <= 1e-5)


def test_deterministic_and_batch_independent(stag):
    import torch
    X, Q, _ = synth.config_points(2, n=20000, m=1000)
    Xd, Qd = to_dev(X), to_dev(Q)
    for form in FORMS:
        S1 = stag.kde_exact(Xd, Qd, 0.05, form=form)
        S2 = stag.kde_exact(Xd, Qd, 0.05, form=form)
        sub = torch.arange(37, 1000, 97, device=Xd.device)
        S3 = stag.kde_exact(Xd, Qd[sub].contiguous(), 0.05, form=form)
        torch.cuda.synchronize()
        assert torch.equal(S1, S2)
        assert torch.equal(S1[sub], S3)  # a query's value does not depend on its batch


def test_config2_full_size_sampled(stag, orc):
    """n = m = 100,000, d = 64: full launch, oracle on 200 sampled queries,
    at the three bandwidths of the workload (a = 1 takes the underflow rescue
    for most queries)."""
    X, Q, _ = synth.config_points(2)
    rng = np.random.default_rng(2002)
    idx = np.sort(rng.choice(Q.shape[0], size=200, replace=False))
    for a in (0.01, 0.1, 1.0):
        ref = orc.kde_exact(X, Q[idx], a)
        for form in (FORMS if a < 1.0 else ["fp32", "fp16_split"]):
            announce(f"config2 full n=m=1e5 a={a} form={form}")
            S, B = _run(stag, X, Q, a, form)
            ok = ref > 1e-300  # densities below the fp64 range are 0 on both sides
            err = rel_err(S[idx][ok], ref[ok])
            assert np.all(err <= B[idx][ok]), (form, a, err.max())
            assert np.all(S[idx][~ok] == 0.0)
            if a == 0.01 and form in ("fp32", "fp16_split"):
                assert err.max() <= 1e-5, (form, err.max())


def test_config3_full_size_sampled(stag, orc):
    """n = 2,000,000, m = 200,000, d = 128, a = 0.01 (the headline workload):
    full launch, oracle on 1,000 sampled queries.  fp16 split, bf16 three-way
    and fp32 within 1e-5; every form within its per-result bound."""
    import torch
    X, Q, _ = synth.config_points(3)
    rng = np.random.default_rng(2003)
    idx = np.sort(rng.choice(Q.shape[0], size=1000, replace=False))
    ref = orc.kde_exact(X, Q[idx], 0.01)
    Xd, Qd = to_dev(X), to_dev(Q)
    for form in ["fp16_split", "bf16_split", "bf16_split3", "fp32"]:
        announce(f"config3 full n=2e6 m=2e5 d=128 a=0.01 form={form}")
        S, B = stag.kde_exact(Xd, Qd, 0.01, form=form, return_bound=True)
        torch.cuda.synchronize()
        S, B = S.cpu().numpy(), B.cpu().numpy()
        err = rel_err(S[idx], ref)
        print(f"[measured] config3 {form}: max rel err {err.max():.3e} over {len(idx)} queries", flush=True)
        assert np.all(err <= B[idx]), (form, err.max())
        assert np.all(np.isfinite(S))
        if form != "bf16_split":
            assert err.max() <= 1e-5, (form, err.max())
    # the workload's second bandwidth, a = 0.001, in the headline's form
    ref2 = orc.kde_exact(X, Q[idx], 0.001)
    announce("config3 full n=2e6 m=2e5 d=128 a=0.001 form=fp16_split")
    S, B = stag.kde_exact(Xd, Qd, 0.001, form="fp16_split", return_bound=True)
    torch.cuda.synchronize()
    S, B = S.cpu().numpy(), B.cpu().numpy()
    err = rel_err(S[idx], ref2)
    print(f"[measured] config3 a=0.001 fp16_split: max rel err {err.max():.3e}", flush=True)
    assert np.all(err <= B[idx]) and err.max() <= 1e-5, err.max()


def _auto_expected(bounds, eps, fp16_ok):
    for f in (["fp16_split"] if fp16_ok else []) + ["bf16_split", "bf16_split3"]:
        if bounds[f] <= eps:
            return f
    return "fp32"


@pytest.mark.parametrize("scale", [1.0, 1e5])
def test_auto_form_choice(stag, scale):
    """STAG_FORM_AUTO returns, bit for bit, the cheapest form (fp16 split when
    the operands fit fp16, bf16 split, bf16 three-way, fp32) whose largest
    per-result bound is <= eps, fp32 when none is."""
    import torch
    X, Q, _ = synth.config_points(2, n=9000, m=300)
    X, Q = (X * scale).astype(np.float32), (Q * scale).astype(np.float32)
    a = 0.01 / scale ** 2
    Xd, Qd = to_dev(X), to_dev(Q)
    res, bounds = {}, {}
    for f in FORMS:
        S, B = stag.kde_exact(Xd, Qd, a, form=f, return_bound=True)
        torch.cuda.synchronize()
        res[f], bounds[f] = S.cpu().numpy(), float(B.cpu().numpy().max())
    fp16_ok = scale == 1.0  # |x| ~ 5e5 is past fp16's range
    levels = sorted(set(bounds.values()))
    eps_list = [levels[0] / 2] + [math.sqrt(u * v) for u, v in zip(levels, levels[1:])] + [levels[-1] * 2]
    for eps in eps_list:
        announce(f"auto form scale={scale} eps={eps:.3e}")
        S = stag.kde_exact(Xd, Qd, a, form="auto", eps=eps)
        torch.cuda.synchronize()
        want = _auto_expected(bounds, eps, fp16_ok)
        assert np.array_equal(S.cpu().numpy(), res[want]), (eps, want, bounds)


def test_check_finite_flag(stag):
    import torch
    import paper_2407_07096_amd._lib as L
    X, Q, _ = synth.config_points(1, n=500, m=40)
    Xb = X.copy()
    Xb[17, 3] = np.nan
    Qb = Q.copy()
    Qb[5, 0] = np.inf
    announce("check finite flag")
    for Xi, Qi in [(Xb, Q), (X, Qb)]:
        with pytest.raises(L.StagError):
            stag.kde_exact(to_dev(Xi), to_dev(Qi), 0.5, form="fp32", check_finite=True)
    S = stag.kde_exact(to_dev(X), to_dev(Q), 0.5, form="fp32", check_finite=True)
    S0 = stag.kde_exact(to_dev(X), to_dev(Q), 0.5, form="fp32")
    torch.cuda.synchronize()
    assert np.array_equal(S.cpu().numpy(), S0.cpu().numpy())
    # without the flag the call runs and the NaN propagates to the affected results
    Sn = stag.kde_exact(to_dev(Xb), to_dev(Q), 0.5, form="fp32")
    torch.cuda.synchronize()
    assert np.all(np.isnan(Sn.cpu().numpy()))
