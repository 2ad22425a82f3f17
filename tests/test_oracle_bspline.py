"""Pins of the oracle's B-spline layer against what Sec. 3.1 fixes."""
import math

import numpy as np
import pytest

from oracle import bspline as bs


@pytest.mark.parametrize("p", range(0, 7))
@pytest.mark.parametrize("n", [1, 3, 8])
def test_partition_of_unity_and_nonnegative(n, p):
    # Sec. 3.1: non-negative partition of unity on [0, 1)
    x = np.random.default_rng(n * 10 + p).random(200)
    B = bs.basis(n, p, x)
    assert B.shape == (200, n + p)
    assert B.min() >= 0.0
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 7))
def test_local_support(p):
    n = 9
    xi = bs.knots(n, p)
    x = np.linspace(0, 1, 1001)[:-1]
    B = bs.basis(n, p, x)
    for i in range(n + p):  # supp N_{i+1} = [xi_{i+1}, xi_{i+p+2}]
        outside = (x < xi[i]) | (x > xi[i + p + 1])
        assert np.all(B[outside, i] == 0.0)


@pytest.mark.parametrize("p", range(1, 7))
def test_vanishing_at_boundary(p):
    # Sec. 3.1: N_i(0) = N_i(1) = 0 for i = 2..n+p-1; N_1(0) = N_{n+p}(1^-) = 1
    n = 6
    B0 = bs.basis(n, p, [0.0])[0]
    assert B0[0] == 1.0 and np.all(B0[1:] == 0.0)
    B1 = bs.basis(n, p, [1.0 - 1e-13])[0]
    assert abs(B1[-1] - 1.0) < 1e-10 and np.all(np.abs(B1[1:-1]) < 1e-10)


@pytest.mark.parametrize("p", range(1, 7))
def test_central_bsplines_are_shifted_cardinal(p):
    # Sec. 3.1: N_i^p(x) = phi_p(n x - i + p + 1), i = p+1..n
    n = 2 * p + 5
    x = np.random.default_rng(p).random(300)
    B = bs.basis(n, p, x)
    for i in range(p + 1, n + 1):
        np.testing.assert_allclose(B[:, i - 1], bs.cardinal(p, n * x - i + p + 1), atol=1e-13)


def _eulerian_row(p):
    """phi_p at the integers 1..p are the Eulerian numbers A(p, k)/p!."""
    out = []
    for k in range(p):
        out.append(sum((-1) ** j * math.comb(p + 1, j) * (k + 1 - j) ** p for j in range(k + 2)))
    return np.array(out, dtype=float) / math.factorial(p)


@pytest.mark.parametrize("p", range(1, 9))
def test_cardinal_integer_values(p):
    np.testing.assert_allclose(bs.cardinal(p, np.arange(1, p + 1)), _eulerian_row(p), rtol=1e-14)


def test_cardinal_known_values():
    np.testing.assert_allclose(bs.cardinal(3, [1, 2, 3]), np.array([1, 4, 1]) / 6, rtol=1e-15)
    np.testing.assert_allclose(bs.cardinal(5, [1, 2, 3, 4, 5]), np.array([1, 26, 66, 26, 1]) / 120, rtol=1e-15)
    np.testing.assert_allclose(bs.cardinal(7, range(1, 8)),
                               np.array([1, 120, 1191, 2416, 1191, 120, 1]) / 5040, rtol=1e-14)


@pytest.mark.parametrize("p", range(1, 7))
def test_cardinal_symmetry_support_integral(p):
    t = np.linspace(-1, p + 2, 2001)
    np.testing.assert_allclose(bs.cardinal(p, t), bs.cardinal(p, p + 1 - t), atol=1e-14)
    assert np.all(bs.cardinal(p, t[(t < 0) | (t > p + 1)]) == 0.0)
    # integral of phi_p is 1
    tt = np.linspace(0, p + 1, 200001)
    assert abs(np.trapezoid(bs.cardinal(p, tt), tt) - 1.0) < 1e-8


@pytest.mark.parametrize("p", range(2, 7))
def test_cardinal_derivative_matches_finite_difference(p):
    t = np.random.default_rng(p).uniform(0.05, p + 0.95, 200)
    t = t[np.abs(t - np.round(t)) > 1e-3]
    h = 1e-6
    fd = (bs.cardinal(p, t + h) - bs.cardinal(p, t - h)) / (2 * h)
    np.testing.assert_allclose(bs.cardinal_deriv(p, t, 1), fd, atol=1e-7)


@pytest.mark.parametrize("p", range(1, 7))
def test_bspline_derivative_matches_finite_difference(p):
    n = 5
    x = np.random.default_rng(p).uniform(0.01, 0.99, 100)
    x = x[np.abs(x * n - np.round(x * n)) > 1e-3]
    h = 1e-7
    fd = (bs.basis(n, p, x + h) - bs.basis(n, p, x - h)) / (2 * h)
    np.testing.assert_allclose(bs.basis_deriv(n, p, x), fd, atol=2e-6 * n)


@pytest.mark.parametrize("p1,p2,r1,r2", [(2, 2, 0, 0), (3, 3, 1, 1), (2, 3, 0, 1), (3, 2, 1, 0), (3, 3, 0, 2)])
def test_cardinal_inner_product_identity(p1, p2, r1, r2):
    # Sec. 3.1: int phi_{p1}^{(r1)}(t) phi_{p2}^{(r2)}(t+tau) dt = (-1)^{r1} phi^{(r1+r2)}_{p1+p2+1}(p1+1+tau)
    t = np.linspace(0, p1 + 1, 400001)
    for tau in [-2.0, -1.0, 0.0, 0.5, 1.0, 1.7]:
        lhs = np.trapezoid(bs.cardinal_deriv(p1, t, r1) * bs.cardinal_deriv(p2, t + tau, r2), t)
        rhs = (-1) ** r1 * bs.cardinal_deriv(p1 + p2 + 1, p1 + 1 + tau, r1 + r2)
        assert abs(lhs - rhs) < 2e-4
