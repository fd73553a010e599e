"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, validates arguments before touching the
device, and its host-only collision probability agrees with the oracle."""
import ctypes as C

import pytest

import paper_2407_07096_amd as stag
from paper_2407_07096_amd import _lib


def test_library_exports_every_declared_symbol():
    lib = stag.load()
    names = stag.declared_symbols()
    assert "stag_kde_exact" in names and "stag_e2lsh_hash" in names
    missing = [s for s in names if not hasattr(lib, s)]
    assert not missing, missing
    assert b"gfx950" in lib.stag_version()


@pytest.mark.parametrize("c", [0.0, 0.1, 0.5, 1.0, 2.0, 4.0, 8.0])
@pytest.mark.parametrize("K,L", [(1, 1), (8, 16), (9, 17)])
def test_collision_probability_host(orc, c, K, L):
    assert stag.collision_probability(c, K, L) == pytest.approx(orc.boosted_probability(c, K, L), rel=1e-12,
                                                                abs=1e-300)


def test_draws_per_node_rule():
    # 0 means ceil(log2 n), at least one draw; explicit counts pass through
    assert [stag.draws_per_node(n) for n in (1, 2, 3, 4, 5, 1024, 1025, 70_000, 100_000)] == \
        [1, 1, 2, 2, 3, 10, 11, 17, 17]
    assert stag.draws_per_node(100, 7) == 7
    with pytest.raises(stag.StagError):
        stag.draws_per_node(100, 65)
    with pytest.raises(stag.StagError):
        stag.draws_per_node(0, 0)


def test_collision_probability_rejects():
    import math
    assert math.isnan(stag.collision_probability(-1.0))
    assert math.isnan(stag.collision_probability(1.0, 0, 1))


def test_invalid_arguments_rejected_before_launch():
    lib = stag.load()
    null = C.c_void_p(0)
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    st = lib.stag_kde_exact(null, 10, fake, 10, 4, 1.0, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "NULL" in stag.last_error()
    st = lib.stag_kde_exact(fake, 10, fake, 10, 4, -1.0, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "a must be" in stag.last_error()
    st = lib.stag_kde_exact(fake, 0, fake, 10, 4, 1.0, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kde_exact(fake, 10, fake, 10, 4, 1.0, 0.0, 9, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kde_exact(fake, 10, fake, 10, 4, 1.0, 0.0, 0, 0x80, fake, null, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 4, 3, 1.0, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "unknown kernel" in stag.last_error()
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 4, -1, 1.0, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 4, 1, 0.0, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "a must be" in stag.last_error()
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 4, 2, 1e200, 0.0, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "out of range" in stag.last_error()
    # d > 256: fp32, fp16 split and bf16 split only (bf16 three-way is not)
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 300, 1, 1.0, 0.0, 3, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    # STAG_FORM_AUTO needs eps > 0; unknown forms and flags
    st = lib.stag_kde_exact(fake, 10, fake, 10, 4, 1.0, 0.0, 4, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "eps" in stag.last_error()
    st = lib.stag_kde_exact(fake, 10, fake, 10, 4, 1.0, 1e-3, 7, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "unknown form" in stag.last_error()
    # the adaptive fp16 form (6): Gaussian sums with d <= 256 only
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 4, 2, 1.0, 0.0, 6, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED and "Gaussian" in stag.last_error()
    st = lib.stag_kde_exact(fake, 10, fake, 10, 300, 1.0, 0.0, 6, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    # the fp16 centred form (5): Gaussian sums with d <= 256 only
    st = lib.stag_kde_exact_kernel(fake, 10, fake, 10, 4, 1, 1.0, 0.0, 5, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED and "Gaussian" in stag.last_error()
    st = lib.stag_kde_exact(fake, 10, fake, 10, 300, 1.0, 0.0, 5, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    st = lib.stag_kde_exact_noalloc(fake, 10, fake, 10, 300, 1.0, 5, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    st = lib.stag_kde_exact(fake, 10, fake, 10, 4, 1.0, 0.0, 0, 4, fake, null, null)
    assert st == _lib.STAG_E_INVAL
    # the no-allocation variant: scratch limit, AUTO and CHECK_FINITE refused before any device work
    st = lib.stag_kde_exact_noalloc(fake, 3_000_000, fake, 300_000, 64, 0.1, 2, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "scratch" in stag.last_error()
    st = lib.stag_kde_exact_noalloc(fake, 100, fake, 100, 8, 0.1, 4, 0, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    st = lib.stag_kde_exact_noalloc(fake, 100, fake, 100, 8, 0.1, 0, 2, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    st = lib.stag_kde_exact_noalloc(null, 100, fake, 100, 8, 0.1, 0, 0, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "NULL" in stag.last_error()
    it = C.c_int32(0)
    st = lib.stag_spectral_embedding(10, fake, fake, fake, 5, 0, 1e-8, 10, 0, null, fake, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL and "k must be" in stag.last_error()
    st = lib.stag_spectral_embedding(10, fake, fake, fake, 5, 57, 1e-8, 10, 0, null, fake, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_spectral_embedding(3, fake, fake, fake, 5, 4, 1e-8, 10, 0, null, fake, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_spectral_embedding(10, null, fake, fake, 5, 2, 1e-8, 10, 0, null, fake, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL and "NULL" in stag.last_error()
    st = lib.stag_spectral_embedding(10, fake, fake, fake, 5, 2, 0.0, 10, 0, null, fake, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_spectral_cluster(0, fake, fake, fake, 5, 2, 0, fake, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kmeans(fake, 10, 2, 11, 0, 10, null, fake, null, null, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kmeans(fake, 10000, 100, 50, 0, 10, null, fake, null, null, C.byref(it), null)
    assert st == _lib.STAG_E_UNSUPPORTED
    st = lib.stag_kmeans(fake, 10, 2, 3, 0, 0, null, fake, null, null, C.byref(it), null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kde_random_sample(fake, 10, fake, 10, 4, 1.0, 0, 1, 0, fake, null, null, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_kde_random_sample(fake, 10, null, 10, 4, 1.0, 5, 1, 0, fake, null, null, null)
    assert st == _lib.STAG_E_INVAL and "NULL" in stag.last_error()
    st = lib.stag_e2lsh_hash(fake, 10, 4, fake, fake, 0, 3, fake, null, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_e2lsh_hash(fake, 10, 4, fake, fake, 2, 3, null, null, null)
    assert st == _lib.STAG_E_INVAL
    h = C.c_void_p(0)
    st = lib.stag_e2lsh_table_create(fake, 10, 4, fake, fake, 2, 65, C.byref(h), null)
    assert st == _lib.STAG_E_INVAL and h.value is None
    st = lib.stag_e2lsh_table_create(fake, 0, 4, fake, fake, 2, 3, C.byref(h), null)
    assert st == _lib.STAG_E_INVAL and h.value is None
    st = lib.stag_e2lsh_table_create(null, 10, 4, fake, fake, 2, 3, C.byref(h), null)
    assert st == _lib.STAG_E_INVAL and "NULL" in stag.last_error()
    st = lib.stag_e2lsh_table_count(null, fake, 3, fake, null)
    assert st == _lib.STAG_E_INVAL
    st = lib.stag_e2lsh_table_neighbours(fake, fake, 0, fake, fake, null)
    assert st == _lib.STAG_E_INVAL
    lib.stag_e2lsh_table_destroy(null)
    # KDE-tree sampler: (n, d, a, s, est_samples, degree_samples)
    for args, msg in [((1, 4, 1.0, 0, 8, 8), "n"), ((10, 0, 1.0, 0, 8, 8), "d >= 1"), ((10, 4, 0.0, 0, 8, 8), "a must"),
                      ((10, 4, 1.0, 65, 8, 8), "samples_per_node"), ((10, 4, 1.0, 0, 0, 8), "est_samples"),
                      ((10, 4, 1.0, 0, 33, 8), "est_samples"), ((10, 4, 1.0, 0, 8, 0), "degree_samples"),
                      ((2 ** 26, 4, 1.0, 64, 8, 8), "2^31")]:
        n, d, a, s_, t, td = args
        st = lib.stag_simgraph_sample_tree(fake, n, d, a, s_, t, td, 1, fake, fake, fake, null, null)
        assert st == _lib.STAG_E_INVAL and msg in stag.last_error(), (args, stag.last_error())
    st = lib.stag_simgraph_sample_tree(fake, 10, 1025, 1.0, 0, 8, 8, 1, fake, fake, fake, null, null)
    assert st == _lib.STAG_E_UNSUPPORTED
    st = lib.stag_simgraph_sample_tree(null, 10, 4, 1.0, 0, 8, 8, 1, fake, fake, fake, null, null)
    assert st == _lib.STAG_E_INVAL and "NULL" in stag.last_error()


@pytest.mark.parametrize("n", [1, 7, 1000, 100_000, 2_000_000])
@pytest.mark.parametrize("kw", [dict(), dict(k1=10, k2_constant=5, p_offset=1, min_mu=1e-4),
                                dict(k1=1, k2_constant=8, p_offset=1), dict(eps=0.2), dict(eps=0.9, k2_constant=3)])
def test_lsh_parameter_reading_matches_oracle(orc, n, kw):
    kw = dict(kw)
    eps = kw.pop("eps", 0.5)
    got = stag.lsh_derive(n, 0.01, eps, **kw)
    ref = orc.lsh_derive(n, 0.01, eps, **kw)
    for k in ("J", "L", "K", "K1"):
        assert got[k] == ref[k], (k, got, ref)
    assert got["mu_min"] == ref["mu_min"]


def test_lsh_parameter_validation():
    with pytest.raises(stag.StagError):
        stag.lsh_derive(100, 0.01, 1.5)
    with pytest.raises(stag.StagError):
        stag.lsh_derive(100, -1.0, 0.5)
    with pytest.raises(stag.StagError):
        stag.lsh_derive(100, 0.01, 0.5, k2_constant=65)


@pytest.mark.parametrize("eps,mu,m,delta", [(0.1, 1e-3, 1000, 0.01), (0.5, 0.2, 1, 0.5), (0.05, 1e-5, 10**6, 1e-3)])
def test_rs_sample_size_matches_oracle(orc, eps, mu, m, delta):
    assert stag.rs_sample_size(eps, mu, m, delta) == orc.rs_sample_size(eps, mu, m, delta)


def test_rs_sample_size_rejects():
    for args in [(0.0, 0.1, 10, 0.1), (1.0, 0.1, 10, 0.1), (0.1, 0.0, 10, 0.1), (0.1, 0.1, 0, 0.1),
                 (0.1, 0.1, 10, 1.0)]:
        assert stag.rs_sample_size(*args) == 0
