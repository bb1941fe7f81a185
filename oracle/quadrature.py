"""Gauss-Legendre quadrature and the 1-D Lagrange nodal basis.

Section II-B: the solution and test functions are Lagrange interpolation
polynomials through N = p+1 points per direction (Eqs. (6)-(7)), and the
integrals are evaluated by Gauss-Legendre quadrature at those same points
(collocation).  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

import numpy as np


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [-1, 1] (the rule Section II-B names).

    Golub-Welsch: the nodes are the eigenvalues of the symmetric tridiagonal
    Jacobi matrix of the Legendre three-term recurrence (off-diagonal
    k/sqrt(4k^2-1)); each weight is 2 times the squared first component of
    the normalised eigenvector.  Returns (nodes ascending, weights).
    """
    if n < 1:
        raise ValueError("need at least one Gauss-Legendre point")
    if n == 1:
        return np.array([0.0]), np.array([2.0])
    k = np.arange(1, n, dtype=np.float64)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    jacobi = np.diag(beta, 1) + np.diag(beta, -1)
    nodes, vecs = np.linalg.eigh(jacobi)
    weights = 2.0 * vecs[0, :] ** 2
    return nodes, weights


def lagrange(nodes, x):
    """Matrix L[q, s] = l_s(x_q) of Eq. (7): the product over i != s of
    (x - xi_i) / (xi_s - xi_i)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for s in range(n):
        for i in range(n):
            if i != s:
                out[:, s] *= (x - nodes[i]) / (nodes[s] - nodes[i])
    return out


def lagrange_deriv(nodes, x):
    """Matrix dL[q, s] = l_s'(x_q): the product rule applied to Eq. (7),
    sum over m != s of 1/(xi_s - xi_m) times the product over i != s, m of
    (x - xi_i)/(xi_s - xi_i)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for s in range(n):
        for m in range(n):
            if m == s:
                continue
            term = np.full(len(x), 1.0 / (nodes[s] - nodes[m]))
            for i in range(n):
                if i != s and i != m:
                    term = term * (x - nodes[i]) / (nodes[s] - nodes[i])
            out[:, s] += term
    return out
