"""Pins of the oracle's five-stage fourth-order low-storage Runge-Kutta
scheme (Sections II-B, IV and V): the classical order conditions in exact
rational arithmetic, the stability polynomial of the floating-point stepper,
its temporal convergence rate, and the first-stage overwrite."""

from fractions import Fraction as Fr

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.dg import DG


def _butcher():
    """Butcher tableau of the 2N-storage recursion K_j = a_j K_{j-1} + dt f(Y_j),
    y_j = y_{j-1} + b_j K_j, in exact fractions: the weight of f(Y_m) in y_i
    is sum_{j=m..i} b_j prod_{l=m+1..j} a_l."""
    a, b, s = lserk.A_FRAC, lserk.B_FRAC, lserk.NSTAGES

    def weight(m, i):
        tot = Fr(0)
        for j in range(m, i + 1):
            prod = Fr(1)
            for l in range(m + 1, j + 1):
                prod *= a[l]
            tot += b[j] * prod
        return tot
    A = [[weight(m, i - 1) if m <= i - 1 else Fr(0) for m in range(s)] for i in range(s)]
    bb = [weight(m, s - 1) for m in range(s)]
    c = [sum(r) for r in A]
    return A, bb, c


def test_order_conditions_exact():
    A, b, c = _butcher()
    s = len(b)
    Ac = [sum(A[i][j] * c[j] for j in range(s)) for i in range(s)]
    conds = [
        (sum(b), Fr(1)),
        (sum(b[i] * c[i] for i in range(s)), Fr(1, 2)),
        (sum(b[i] * c[i] ** 2 for i in range(s)), Fr(1, 3)),
        (sum(b[i] * Ac[i] for i in range(s)), Fr(1, 6)),
        (sum(b[i] * c[i] ** 3 for i in range(s)), Fr(1, 4)),
        (sum(b[i] * c[i] * Ac[i] for i in range(s)), Fr(1, 8)),
        (sum(b[i] * sum(A[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)), Fr(1, 12)),
        (sum(b[i] * sum(A[i][j] * Ac[j] for j in range(s)) for i in range(s)), Fr(1, 24)),
    ]
    for got, want in conds:
        assert abs(got - want) < Fr(1, 10 ** 20)
    # the published stage times are the row sums of the tableau
    for i in range(s):
        assert abs(c[i] - lserk.C_FRAC[i]) < Fr(1, 10 ** 20)


def test_float_coefficients_are_rounded_fractions():
    for fl, fr in zip(lserk.A + lserk.B, lserk.A_FRAC + lserk.B_FRAC):
        assert fl == fr.numerator / fr.denominator
    assert lserk.A[0] == 0.0


def test_stability_polynomial():
    """One step of y' = z y multiplies y by R(z) = sum_{k<=4} z^k/k! + g z^5."""
    zs = 0.6 * np.exp(2j * np.pi * np.arange(6) / 6)
    vals = []
    for z in zs:
        Q = np.array([1.0 + 0j])
        res = np.zeros_like(Q)
        lserk.step(Q, res, 1.0, lambda y, z=z: z * y)
        vals.append(Q[0])
    V = np.vander(zs, 6, increasing=True)
    coef = np.linalg.solve(V, np.array(vals))
    assert np.max(np.abs(coef[:5] - np.array([1, 1, 1 / 2, 1 / 6, 1 / 24]))) < 1e-12
    assert abs(coef[5]) > 1e-4    # a genuine fifth-order term: not the classical RK4


def test_temporal_order_on_smooth_nonlinear_system():
    """Pendulum y0' = y1, y1' = -sin(y0): a smooth autonomous nonlinear
    system, so all eight fourth-order trees matter.  (The DG system itself
    is only Lipschitz: the face flux switches branches of max and |.|.)"""
    def f(y):
        return np.array([y[1], -np.sin(y[0])])
    y0 = np.array([1.2, 0.3])
    T = 4.0
    ref = lserk.integrate(y0, T / 4096, 4096, f)
    errs = []
    for ns in (16, 32, 64):
        errs.append(np.max(np.abs(lserk.integrate(y0, T / ns, ns, f) - ref)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 3.8), (errs, rates)


def test_first_stage_overwrites_register():
    n, p = (2, 1, 1), 1
    dg = DG(n, p)
    Q = W.random_smooth(n, p, seed=12)
    Qa, Qb = Q.copy(), Q.copy()
    ra = np.full_like(Q, np.nan)
    rb = np.zeros_like(Q)
    lserk.step(Qa, ra, 1e-3, dg.rhs)
    lserk.step(Qb, rb, 1e-3, dg.rhs)
    assert np.array_equal(Qa, Qb) and np.all(np.isfinite(Qa))
