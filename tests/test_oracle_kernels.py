"""Pins of the oracle's exponential and logistic kernel densities
(Sec. "Kernel Density Estimation": the three kernel functions and the
density K(q) = S(q)/n), against values fixed by the mathematics rather than by
the oracle's own formulas."""
import math

import numpy as np
import pytest

import oracle

KERNELS = ("gaussian", "exponential", "logistic")


@pytest.mark.parametrize(
    "kernel,a,r,want",
    [
        # hand-derived points: e^{-a r} = 1/2 at a r = ln 2, 1/3 at a r = ln 3
        ("exponential", 1.0, math.log(2.0), 0.5),
        ("exponential", 2.0, math.log(3.0) / 2.0, 1.0 / 3.0),
        # logistic 4/(2 + e^u + e^-u): e^u = 3 gives 4/(16/3) = 3/4, e^u = 2 gives 8/9
        ("logistic", 1.0, math.log(3.0), 0.75),
        ("logistic", 0.5, 2.0 * math.log(2.0), 8.0 / 9.0),
        ("gaussian", 1.0, math.sqrt(math.log(2.0)), 0.5),
        ("gaussian", 0.25, 2.0 * math.sqrt(math.log(4.0)), 0.25),
    ],
)
def test_kernel_special_values(kernel, a, r, want):
    assert oracle.kernel_value(kernel, a, r) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("kernel", KERNELS)
def test_kernel_shape_conditions(kernel):
    # the paper's conditions on a kernel function: values in [0, 1], k(0) = 1,
    # non-increasing in the distance (up to the rounding of 2 + e^u + e^-u,
    # one ulp of 1.0, near r = 0)
    r = np.concatenate([[0.0], np.geomspace(1e-8, 60.0, 400)])
    k = np.array([oracle.kernel_value(kernel, 0.7, float(v)) for v in r])
    assert k[0] == 1.0
    assert np.all(k >= 0.0) and np.all(k <= 1.0)
    assert np.all(np.diff(k) <= 2.3e-16)


def test_distance_is_euclidean_not_squared():
    # 3-4-5 triangle in the plane: r = 5.  With a = ln2/5 the exponential kernel
    # is exactly 1/2; with a = ln3/5 the logistic kernel is exactly 3/4.
    Q = np.array([[0.0, 0.0]], dtype=np.float32)
    X = np.array([[3.0, 4.0]], dtype=np.float32)
    assert oracle.kde_kernel(X, Q, math.log(2.0) / 5.0, "exponential")[0] == pytest.approx(0.5, rel=1e-15)
    assert oracle.kde_kernel(X, Q, math.log(3.0) / 5.0, "logistic")[0] == pytest.approx(0.75, rel=1e-15)


def test_exponential_geometric_series():
    # d = 1, x_i = i (i = 0..n-1), q = 0: S = sum_i e^{-a i} = (1 - e^{-a n}) / (1 - e^{-a})
    n, a = 300, 0.05
    X = np.arange(n, dtype=np.float32)[:, None]
    Q = np.zeros((1, 1), dtype=np.float32)
    want = -math.expm1(-a * n) / -math.expm1(-a)
    assert oracle.kde_kernel(X, Q, a, "exponential")[0] == pytest.approx(want, rel=1e-13)


def test_logistic_is_squared_hyperbolic_secant():
    # 4/(2 + e^u + e^-u) = 1/cosh(u/2)^2: brute force with the other form
    rng = np.random.default_rng(11)
    X = rng.normal(size=(57, 5)).astype(np.float32)
    Q = rng.normal(size=(9, 5)).astype(np.float32)
    a = 0.8
    r = np.sqrt(((Q[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1))
    want = (1.0 / np.cosh(a * r / 2.0) ** 2).sum(1)
    np.testing.assert_allclose(oracle.kde_kernel(X, Q, a, "logistic"), want, rtol=1e-13)


@pytest.mark.parametrize("kernel", KERNELS)
def test_all_points_at_the_query(kernel):
    # k(0) = 1: S(q) = n when every x_i equals q
    q = np.array([[0.3, -1.25, 2.0]], dtype=np.float32)
    X = np.repeat(q, 37, axis=0)
    assert oracle.kde_kernel(X, q, 1.3, kernel)[0] == 37.0


def test_gaussian_matches_the_max_shift_oracle():
    # two independent formulations of the Gaussian sum agree
    rng = np.random.default_rng(5)
    X = rng.normal(size=(300, 7)).astype(np.float32)
    Q = rng.normal(size=(20, 7)).astype(np.float32)
    np.testing.assert_allclose(oracle.kde_kernel(X, Q, 0.4, "gaussian"), oracle.kde_exact(X, Q, 0.4), rtol=1e-13)


def test_exponential_monotone_in_bandwidth():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(200, 4)).astype(np.float32)
    Q = rng.normal(size=(10, 4)).astype(np.float32)
    s = [oracle.kde_kernel(X, Q, a, k) for k in ("exponential", "logistic") for a in (0.2, 0.5, 1.0)]
    for k in range(2):
        assert np.all(s[3 * k] > s[3 * k + 1]) and np.all(s[3 * k + 1] > s[3 * k + 2])
