"""GPU parity of the KDE-tree edge sampler (Sec. "The MS Algorithm" with the
random-sampling estimator per tree node) against the FP64 oracle, through
the C ABI entry point stag_simgraph_sample_tree.

Bar: sources identical; every destination identical except where a
decision's target lies within 1e-9 (relative) of its boundary in the oracle
(the two sides add the same fp64 values in different orders, so only such
draws may differ; none is expected); degrees and weights within 1e-12
relative; every destination in range and different from its source;
results bit-identical across runs."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu

MARGIN = 1e-9


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def _gpu(stag, X, a, s, t, t_deg, seed, Xd=None):
    import torch
    src, dst, w, deg = stag.simgraph_sample_tree(to_dev(X) if Xd is None else Xd, a, s, t, t_deg, seed)
    torch.cuda.synchronize()
    return src.cpu().numpy(), dst.cpu().numpy(), w.cpu().numpy(), deg.cpu().numpy()


def _compare(got, ref, rows=None):
    src, dst, w, deg = got
    osrc, odst, ow, odeg, omg = ref
    if rows is not None:
        lo, hi = rows
        s = len(osrc) // (hi - lo)
        src, dst, w = src[lo * s:hi * s], dst[lo * s:hi * s], w[lo * s:hi * s]
    assert np.array_equal(src, osrc)
    diff = dst != odst
    assert np.all(omg[diff] < MARGIN), (int(diff.sum()), omg[diff].max())
    same = ~diff
    np.testing.assert_allclose(w[same], ow[same], rtol=1e-12, atol=0)
    np.testing.assert_allclose(deg, odeg, rtol=1e-12, atol=0)
    return int(diff.sum())


def _valid(src, dst, n):
    assert np.all(dst != src) and dst.min() >= 0 and dst.max() < n


@pytest.mark.parametrize("n,d,a,s,t,t_deg", [
    (2, 3, 1.0, 5, 4, 1), (33, 3, 0.8, 7, 5, 20), (97, 1, 2.0, 6, 1, 97), (300, 8, 0.5, 9, 8, 64),
    (1000, 64, 0.01, 10, 32, 128), (4099, 64, 0.05, 4, 16, 4099), (500, 300, 0.002, 3, 32, 50),
    (200, 1024, 0.0005, 2, 7, 300), (2500, 10, 0.3, 5, 3, 2)])
def test_parity_shapes(stag, orc, n, d, a, s, t, t_deg):
    rng = np.random.default_rng(n + d)
    if d == 64:
        X, _, _ = synth.config_points(2, n=n, m=1)
    else:
        X = (rng.normal(size=(n, d)) * 2.0).astype(np.float32)
    announce(f"tree sampler n={n} d={d} a={a} s={s} t={t} t_deg={t_deg}")
    got = _gpu(stag, X, a, s, t, t_deg, 17 + n)
    _valid(got[0], got[1], n)
    ref = orc.simgraph_tree(X, a, s, t, t_deg, 17 + n)
    nd = _compare(got, ref)
    print(f"[measured] tree n={n} d={d}: {nd} of {n * s} draws differ (all within the margin)", flush=True)


def test_zero_kernel_rule_bitexact(stag, orc):
    # all kernel values underflow: no floating-point decision is left, so
    # every draw is fixed by the row-count rule and the leaf uniform
    n = 75
    X = (np.arange(n, dtype=np.float32)[:, None] * np.float32(100.0)).repeat(2, axis=1)
    announce("tree sampler zero-kernel rule n=75")
    got = _gpu(stag, X, 1.0, 5, 4, 10, 7)
    ref = orc.simgraph_tree(X, 1.0, 5, 4, 10, 7)
    assert np.array_equal(got[1], ref[1]) and np.all(got[2] == 0.0) and np.all(got[3] == 1.0)


def test_unaligned_rows_and_determinism(stag):
    # X starting 4 bytes past a 16-byte boundary takes the scalar row loads;
    # the values are the same, bit for bit
    import torch
    X, _, _ = synth.config_points(2, n=3000, m=1)
    announce("tree sampler unaligned X, repeat")
    buf = torch.empty(X.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(X.reshape(-1)).cuda()
    Xu = buf[1:].view(X.shape)
    assert Xu.data_ptr() % 16 == 4
    a1 = _gpu(stag, X, 0.01, 6, 24, 256, 5)
    a2 = _gpu(stag, X, 0.01, 6, 24, 256, 5)
    a3 = _gpu(stag, X, 0.01, 6, 24, 256, 5, Xd=Xu)
    for u, v, z in zip(a1, a2, a3):
        assert np.array_equal(u, v) and np.array_equal(u, z)


def test_full_size_sampled_rows(stag, orc):
    """n = 100,000, d = 64 mixture, a = 0.01, s = 17, t = 32, 1024 degree
    samples: the whole launch, validity everywhere, oracle parity on 200 rows
    (degrees of every row)."""
    X, _, _ = synth.config_points(2)
    n = len(X)
    announce("tree sampler full n=1e5 d=64 s=17 t=32 t_deg=1024")
    got = _gpu(stag, X, 0.01, 17, 32, 1024, 99)
    _valid(got[0], got[1], n)
    assert np.all(got[2] > 0) and np.all(np.isfinite(got[2]))
    ref = orc.simgraph_tree(X, 0.01, 17, 32, 1024, 99, rows=(51200, 51400))
    nd = _compare(got, ref, rows=(51200, 51400))
    print(f"[measured] tree full size: {nd} of 3400 sampled draws differ", flush=True)


def test_config4_sampled_rows(stag, orc):
    """n = 70,000, d = 784, sparse non-negative data (entries 0 with
    probability 0.8, else U[0,1]), a = 1e-3, 17 draws per node, t = 16, 64
    degree samples: the whole launch, oracle parity on 100 rows."""
    X = synth.sparse_uniform(70_000, 784, 1004)
    n = len(X)
    announce("tree sampler config4 n=70000 d=784 s=17 t=16 t_deg=64")
    got = _gpu(stag, X, 1e-3, 17, 16, 64, 5)
    _valid(got[0], got[1], n)
    ref = orc.simgraph_tree(X, 1e-3, 17, 16, 64, 5, rows=(35000, 35100))
    nd = _compare(got, ref, rows=(35000, 35100))
    print(f"[measured] tree config4: {nd} of 1700 sampled draws differ", flush=True)
