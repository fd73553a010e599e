"""GPU parity of the similarity-graph edge sampler (Sec. "The MS Algorithm")
against the oracle.

What is unique is compared exactly: sources, the draw for every draw whose
target lies farther than the arithmetic tolerance from a cumulative boundary
(the oracle reports that margin), and degrees/weights within the tolerance of
the kernel sums.  Draws inside the tolerance band must still be valid: the
chosen neighbour's cumulative interval, recomputed by the oracle, contains the
target up to the tolerance."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def _gpu(stag, X, a, s, **kw):
    import torch
    src, dst, w, deg = stag.simgraph_sample(to_dev(X), a, samples_per_node=s, **kw)
    torch.cuda.synchronize()
    return src.cpu().numpy(), dst.cpu().numpy(), w.cpu().numpy(), deg.cpu().numpy()


def _check_valid_draws(orc, X, a, s, seed, src, dst, bad_idx, tol):
    """Each listed draw's target must fall in the chosen j's cumulative
    interval (ascending j, j != i) widened by tol * rest_i."""
    for e in bad_idx:
        i, r = e // s, e % s
        row = orc.kernel_row(X, a, i)
        row[i] = 0.0
        c = np.cumsum(row)
        rest = c[-1]
        target = orc.draw_uniform(seed, i, r) * rest
        j = dst[e]
        lo = c[j - 1] if j > 0 else 0.0
        assert lo - tol * rest <= target <= c[j] + tol * rest, (e, i, j, lo, target, c[j])


@pytest.mark.parametrize("form,tol", [("fp32", 1e-4), ("fp16_split", 1e-4)])
def test_exact_mode_config1(stag, orc, form, tol):
    X, _, _ = synth.config_points(1)
    a, s, seed = 0.5, 10, 17
    announce(f"simgraph exact config1 n=1000 d=10 form={form}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="exact", form=form, seed=seed)
    osrc, odst, ow, odeg, mg = orc.simgraph_exact(X, a, s, seed, return_margin=True)
    assert np.array_equal(src, osrc)
    assert np.allclose(deg, odeg, rtol=tol)
    same = dst == odst
    firm = mg > tol
    assert np.all(same[firm]), np.nonzero(firm & ~same)[0][:10]
    _check_valid_draws(orc, X, a, s, seed, src, dst, np.nonzero(~same)[0], tol)
    assert np.all(dst != src) and np.all(dst >= 0)
    ok = same
    assert np.allclose(w[ok], ow[ok], rtol=tol)


@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_exact_mode_small_densities(stag, orc, form):
    # 40 outliers far from a cluster and from each other: their rows' kernel
    # values (~1e-125) lie below the fp32 range of the tile's terms and take
    # the underflow rescue; their draws and weights match the oracle's
    rng = np.random.default_rng(77)
    d = 8
    main = rng.normal(size=(2000, d))
    out = 20.0 + 6.0 * rng.normal(size=(40, d))
    X = np.concatenate([main, out]).astype(np.float32)
    a, s, seed, tol = 0.5, 8, 23, 1e-4
    announce(f"simgraph exact small densities n={len(X)} d={d} form={form}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="exact", form=form, seed=seed)
    osrc, odst, ow, odeg, mg = orc.simgraph_exact(X, a, s, seed, return_margin=True)
    assert np.array_equal(src, osrc)
    rows = np.arange(2000, len(X))
    orest = np.array([np.sum(np.delete(orc.kernel_row(X, a, i), i)) for i in rows])
    assert np.sum(orest < 2.0 ** -60) >= 30 and np.all(orest > 1e-300)  # the case is exercised
    same = dst == odst
    firm = mg > tol
    assert np.all(same[firm]), np.nonzero(firm & ~same)[0][:10]
    _check_valid_draws(orc, X, a, s, seed, src, dst, np.nonzero(~same)[0], tol)
    assert np.all(dst != src) and np.all(dst >= 0)
    assert np.allclose(w[same], ow[same], rtol=tol)
    e_out = np.arange(2000 * s, len(X) * s)
    werr = np.abs(w[e_out] - ow[e_out]) / ow[e_out]
    print(f"[measured] small densities {form}: outlier draws equal {np.mean(same[e_out]):.3f}, "
          f"max weight rel err {werr.max():.3e}", flush=True)
    # relative, since the weights are ~1e-60: the expanded distance at
    # ||x||^2 ~ 3000 gives ~5e-4 (the exponent's error grows with the norms)
    assert werr.max() <= 5e-3, werr.max()


@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_exact_mode_subnormal_row(stag, orc, form):
    """One outlier whose row sum lies in the fp64 subnormal range (~1e-315):
    its exponents' maximum is below -1024, where 2^{-m_i} alone overflows; the
    draws take 2^{E - m_i} in one exponent and match the oracle's."""
    rng = np.random.default_rng(78)
    d, a = 8, 0.5
    main = rng.normal(size=(2000, d))

    def log_rest(R):
        x0 = np.zeros(d)
        x0[0] = R
        D = ((main - x0) ** 2).sum(1)
        v = -a * D
        return v.max() + np.log(np.exp(v - v.max()).sum())

    lo, hi = 10.0, 60.0
    for _ in range(60):  # R with a row sum near 1e-315
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if log_rest(mid) > np.log(1e-315) else (lo, mid)
    x0 = np.zeros((1, d))
    x0[0, 0] = lo
    X = np.concatenate([main, x0]).astype(np.float32)
    s, seed, tol = 8, 29, 1e-4
    i = len(X) - 1
    orest = np.sum(np.delete(orc.kernel_row(X, a, i), i))
    assert 1e-320 < orest < 1e-308  # the case is exercised: subnormal row sum
    announce(f"simgraph exact subnormal row form={form}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="exact", form=form, seed=seed)
    osrc, odst, ow, odeg, mg = orc.simgraph_exact(X, a, s, seed, return_margin=True)
    e = np.arange(i * s, (i + 1) * s)
    assert np.all(dst[e] >= 0) and np.all(dst[e] != i)
    same = dst[e] == odst[e]
    assert np.all(same[mg[e] > tol])
    _check_valid_draws(orc, X, a, s, seed, src, dst, e[~same], tol)
    assert deg[i] == odeg[i] == 1.0  # deg = 1 + rest_i rounds to 1 in binary64
    assert np.all(np.abs(w[e][same] - ow[e][same]) <= 5e-3 * ow[e][same])


@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_exact_mode_wide_rows(stag, orc, form):
    """d = 784 (the wide fp32 and split tiles), sparse non-negative data, a = 1e-3."""
    X = synth.sparse_uniform(3000, 784, 1004)
    a, s, seed = 1e-3, 12, 5
    announce(f"simgraph exact n=3000 d=784 form={form}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="exact", form=form, seed=seed)
    osrc, odst, ow, odeg, mg = orc.simgraph_exact(X, a, s, seed, return_margin=True)
    assert np.allclose(deg, odeg, rtol=1e-5)
    same = dst == odst
    assert np.all(same[mg > 1e-5])
    _check_valid_draws(orc, X, a, s, seed, src, dst, np.nonzero(~same)[0], 1e-5)


@pytest.mark.parametrize("d,form", [(64, "fp32"), (100, "fp16_split"), (256, "fp32")])
def test_exact_mode_fused_draw_widths(stag, orc, d, form):
    """d = 64, 100 and 256 (the fused draw kernel: a lane half reads its row
    four 16-byte pieces at a time, then the remaining pieces), n = 4500 (two
    4096-row chunks, a ragged last tile), clustered data: degrees within
    1e-5, draws equal to the oracle's outside the tolerance band and valid
    inside it."""
    mix = synth.mixture(d, 8, 8100 + d, sigma=(0.5, 1.5), box=3.0)
    X = synth.sample(mix, 4500, 8200 + d)
    a, s, seed, tol = 1.0 / d, 9, 41, 1e-4
    announce(f"simgraph exact fused draws n=4500 d={d} form={form}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="exact", form=form, seed=seed)
    osrc, odst, ow, odeg, mg = orc.simgraph_exact(X, a, s, seed, return_margin=True)
    assert np.array_equal(src, osrc)
    assert np.allclose(deg, odeg, rtol=1e-5)
    assert np.all(dst >= 0) and np.all(dst != src)
    same = dst == odst
    assert np.all(same[mg > tol])
    _check_valid_draws(orc, X, a, s, seed, src, dst, np.nonzero(~same)[0], tol)
    assert np.all(np.abs(w[same] - ow[same]) <= 1e-4 * ow[same])


@pytest.mark.parametrize("form", ["fp32", "fp16_split"])
def test_exact_mode_wide_scalar_rows_rescue(stag, orc, form):
    """d = 301 > 256 (draws sorted by tile before the row step) with rows
    that are not a multiple of 4 (element-wise staging and differences),
    n = 1501 (a ragged last tile) and one outlier whose row sum (~1e-100)
    takes the underflow rescue (shifted exponents): every draw matches the
    oracle's outside the tolerance band and is valid inside it."""
    rng = np.random.default_rng(81)
    d, a = 301, 0.005
    main = rng.normal(size=(1500, d))

    def log_rest(R):
        x0 = np.zeros(d)
        x0[0] = R
        v = -a * ((main - x0) ** 2).sum(1)
        return v.max() + np.log(np.exp(v - v.max()).sum())

    lo, hi = 0.0, 1000.0
    for _ in range(60):  # R with a row sum near 1e-100
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if log_rest(mid) > np.log(1e-100) else (lo, mid)
    x0 = np.zeros((1, d))
    x0[0, 0] = lo
    X = np.concatenate([main, x0]).astype(np.float32)
    s, seed, tol = 9, 31, 1e-4
    i = len(X) - 1
    orest = np.sum(np.delete(orc.kernel_row(X, a, i), i))
    assert 1e-110 < orest < 2.0 ** -60  # the rescue is exercised
    announce(f"simgraph exact n={len(X)} d={d} scalar rows + rescue form={form}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="exact", form=form, seed=seed)
    osrc, odst, ow, odeg, mg = orc.simgraph_exact(X, a, s, seed, return_margin=True)
    assert np.array_equal(src, osrc)
    assert np.allclose(deg, odeg, rtol=1e-5)
    assert np.all(dst >= 0) and np.all(dst != src)
    same = dst == odst
    assert np.all(same[mg > tol])
    _check_valid_draws(orc, X, a, s, seed, src, dst, np.nonzero(~same)[0], tol)
    assert np.all(np.abs(w[same] - ow[same]) <= 1e-4 * ow[same])


@pytest.mark.parametrize("form", ["fp32", "fp16_split", "bf16_split"])
def test_exact_kde_wide_rows(stag, orc, form):
    """Exact KDE through the wide tiles (256 < d <= 1024) with ragged n, m:
    within the bound, and within 1e-5 for fp32 and fp16 split."""
    import torch
    rng = np.random.default_rng(3)
    for n, m, d in [(4100, 70, 784), (33, 5, 300), (5000, 129, 1024), (4200, 300, 832)]:
        X = rng.uniform(0, 1, size=(n, d)).astype(np.float32) * (rng.uniform(size=(n, d)) > 0.8)
        Q = X[rng.integers(0, n, size=m)] + 0.01 * rng.normal(size=(m, d)).astype(np.float32)
        Q = Q.astype(np.float32)
        announce(f"wide exact n={n} m={m} d={d} form={form}")
        S, B = stag.kde_exact(to_dev(X), to_dev(Q), 1e-3, form=form, return_bound=True)
        torch.cuda.synchronize()
        ref = orc.kde_exact(X, Q, 1e-3)
        err = np.abs(S.cpu().numpy() - ref) / ref
        print(f"[measured] wide {form} d={d}: max rel err {err.max():.3e}, max bound {B.cpu().numpy().max():.3e}",
              flush=True)
        assert np.all(err <= B.cpu().numpy())
        if form != "bf16_split":
            assert err.max() <= 1e-5


def test_exact_mode_config4_full_sampled(stag, orc):
    """n = 70,000, d = 784 (config 4): full GPU run, oracle on 48 nodes."""
    X = synth.sparse_uniform(70_000, 784, 1004)
    a, seed = 1e-3, 4004
    announce("simgraph exact config4 full n=70000 d=784")
    src, dst, w, deg = _gpu(stag, X, a, 0, mode="exact", form="fp32", seed=seed)
    s = 17
    assert src.shape[0] == 70_000 * s
    assert np.all(dst >= 0) and np.all(dst != src) and np.all(w > 0)
    rng = np.random.default_rng(1)
    nodes = rng.choice(70_000, size=48, replace=False)
    for i in nodes:
        row = orc.kernel_row(X, a, int(i))
        assert abs(deg[i] - row.sum()) <= 1e-5 * row.sum()
        _check_valid_draws(orc, X, a, s, seed, src, dst, np.arange(i * s, (i + 1) * s), 1e-5)


def test_lsh_mode_config4_full(stag):
    """n = 70,000, d = 784, a = 1e-3 in CKNS mode: every draw valid, weights
    positive, degree estimates near the exact mode's, runs deterministic."""
    X = synth.sparse_uniform(70_000, 784, 1004)
    a, seed = 1e-3, 4004
    kw = dict(eps=0.5, k1=1, k2_constant=8, p_offset=3, lsh_seed=3004)
    announce("simgraph lsh config4 full n=70000 d=784")
    src, dst, w, deg = _gpu(stag, X, a, 0, mode="lsh", seed=seed, **kw)
    s = 17
    assert src.shape[0] == 70_000 * s
    assert np.array_equal(src, np.repeat(np.arange(70_000), s))
    ok = dst >= 0
    assert ok.mean() > 0.99
    assert np.all(dst[ok] != src[ok]) and np.all(dst[ok] < 70_000) and np.all(w[ok] > 0)
    _, _, _, deg_e = _gpu(stag, X, a, 0, mode="exact", form="fp32", seed=seed)
    rel = np.abs(deg - deg_e) / deg_e
    print(f"[measured] config4 CKNS degrees vs exact: median {np.median(rel):.3e}, max {rel.max():.3e}", flush=True)
    assert np.median(rel) < 0.05
    src2, dst2, w2, deg2 = _gpu(stag, X, a, 0, mode="lsh", seed=seed, **kw)
    assert np.array_equal(dst, dst2) and np.array_equal(w, w2) and np.array_equal(deg, deg2)


def test_lsh_mode_784d_matches_oracle(stag, orc):
    """The CKNS mode at d = 784 (the wide-row paths) against the oracle on a
    reduced sparse workload."""
    X = synth.sparse_uniform(3000, 784, 1004)
    n, d = X.shape
    a = 1e-3
    kw = dict(eps=0.5, k1=1, k2_constant=8, p_offset=3)
    G0, B = _lsh_inputs(orc, n, d, a, 33, **kw)
    s, seed = 6, 78
    announce("simgraph lsh 784-d n=3000")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="lsh", seed=seed, G0=to_dev(G0), b=to_dev(B), lsh_seed=0, **kw)
    osrc, odst, ow, odeg, mg = orc.simgraph_lsh(X, a, s, seed, G0, B, lsh_seed=0, **kw)
    assert np.array_equal(src, osrc)
    assert np.allclose(deg, odeg, rtol=1e-9)
    same = dst == odst
    assert np.all(same[mg > 1e-9]) and same.mean() > 0.99
    ok = same & (dst >= 0)
    assert np.allclose(w[ok], ow[ok], rtol=1e-9)


def _lsh_inputs(orc, n, d, a, seed, **kw):
    sh = orc.lsh_derive(n, a, **kw)
    npj = sh["K1"] * sh["J"] * sh["L"] * sh["K"]
    return synth.e2lsh_randomness(npj, d, seed)


@pytest.mark.parametrize("cfg", [1, 2])
def test_lsh_mode_matches_oracle(stag, orc, cfg):
    if cfg == 1:
        X, _, _ = synth.config_points(1, n=1200, m=1)
        a = 0.05
    else:
        X, _, _ = synth.config_points(2, n=3000, m=1)
        a = 0.01
    n, d = X.shape
    kw = dict(eps=0.5, k1=2, k2_constant=4)
    G0, B = _lsh_inputs(orc, n, d, a, 31, **kw)
    s, seed = 8, 77
    announce(f"simgraph lsh config{cfg} n={n}")
    src, dst, w, deg = _gpu(stag, X, a, s, mode="lsh", seed=seed, eps=0.5, G0=to_dev(G0), b=to_dev(B), k1=2,
                            k2_constant=4, lsh_seed=0)
    osrc, odst, ow, odeg, mg = orc.simgraph_lsh(X, a, s, seed, G0, B, lsh_seed=0, **kw)
    assert np.array_equal(src, osrc)
    assert np.allclose(deg, odeg, rtol=1e-9)
    same = dst == odst
    firm = mg > 1e-9
    assert np.all(same[firm])
    assert same.mean() > 0.99
    ok = same & (dst >= 0)
    assert np.allclose(w[ok], ow[ok], rtol=1e-9)
