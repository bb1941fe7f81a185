"""Pins of the oracle's Gauss-Legendre rule and Lagrange basis (Section II-B,
Eqs. (6)-(7)) against the library rule, exact moments and polynomial
exactness."""

import numpy as np
import pytest

from oracle.quadrature import gauss_legendre, lagrange, lagrange_deriv


@pytest.mark.parametrize("n", range(1, 11))
def test_gl_matches_library_rule(n):
    x, w = gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 2e-15 * n
    assert abs(np.sum(w) - 2.0) < 1e-14


@pytest.mark.parametrize("n", range(1, 11))
def test_gl_exact_moments(n):
    x, w = gauss_legendre(n)
    for m in range(2 * n):
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** m) - exact) < 1e-14
    # degree 2n is not integrated exactly (pins the number of points)
    m = 2 * n
    assert abs(np.dot(w, x ** m) - 2.0 / (m + 1)) > 1e-6


@pytest.mark.parametrize("p", range(0, 8))
def test_lagrange_polynomial_exactness(p):
    xi, _ = gauss_legendre(p + 1)
    rng = np.random.default_rng(p)
    x = rng.uniform(-1, 1, 17)
    L = lagrange(xi, x)
    dL = lagrange_deriv(xi, x)
    for m in range(p + 1):
        assert np.max(np.abs(L @ xi ** m - x ** m)) < 1e-13
        dexact = m * x ** (m - 1) if m > 0 else np.zeros_like(x)
        assert np.max(np.abs(dL @ xi ** m - dexact)) < 1e-11
    # cardinality at the nodes
    assert np.array_equal(lagrange(xi, xi), np.eye(p + 1))


@pytest.mark.parametrize("p", range(0, 8))
def test_lagrange_identities(p):
    xi, w = gauss_legendre(p + 1)
    lm = lagrange(xi, [-1.0])[0]
    lp = lagrange(xi, [1.0])[0]
    D = lagrange_deriv(xi, xi)           # D[a, i] = l_i'(xi_a)
    assert abs(lm.sum() - 1.0) < 1e-14 and abs(lp.sum() - 1.0) < 1e-14
    assert np.max(np.abs(D.sum(axis=1))) < 1e-12
    # free-stream identity: sum_a w_a l_i'(xi_a) = l_i(1) - l_i(-1)
    assert np.max(np.abs(w @ D - (lp - lm))) < 1e-12
    # symmetry of the Gauss-Legendre points: l_i(-1) = l_{N-1-i}(1)
    assert np.max(np.abs(lm - lp[::-1])) < 1e-13
