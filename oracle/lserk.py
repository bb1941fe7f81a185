"""Five-stage, fourth-order, low-storage explicit Runge-Kutta (LSERK45).

Sections II-B, IV and V: the time integrator is a low-storage explicit
five-stage fourth-order Runge-Kutta method.  The paper does not print its
coefficients; the reading taken here is the standard 2N-storage (5,4) scheme
of Carpenter and Kennedy (1994), the one tabulated in the nodal DG textbook
the paper cites (Hesthaven and Warburton, 2007).

Two registers Q and res.  Stage s = 1..5:
    res <- a_s res + dt RHS(Q)        (a_1 = 0: stage 1 overwrites res)
    Q   <- Q + b_s res
The right-hand side is autonomous, so the stage times c_s are not used.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

from fractions import Fraction

import numpy as np

A_FRAC = (
    Fraction(0),
    Fraction(-567301805773, 1357537059087),
    Fraction(-2404267990393, 2016746695238),
    Fraction(-3550918686646, 2091501179385),
    Fraction(-1275806237668, 842570457699),
)
B_FRAC = (
    Fraction(1432997174477, 9575080441755),
    Fraction(5161836677717, 13612068292357),
    Fraction(1720146321549, 2090206949498),
    Fraction(3134564353537, 4481467310338),
    Fraction(2277821191437, 14882151754819),
)
C_FRAC = (
    Fraction(0),
    Fraction(1432997174477, 9575080441755),
    Fraction(2526269341429, 6820363962896),
    Fraction(2006345519317, 3224310063776),
    Fraction(2802321613138, 2924317926251),
)

A = tuple(float(x) for x in A_FRAC)
B = tuple(float(x) for x in B_FRAC)
C = tuple(float(x) for x in C_FRAC)
NSTAGES = 5


def stage(s, Q, res, dt, rhs):
    """Stage s (0-based) in place on the two registers; returns (Q, res)."""
    R = rhs(Q)
    if s == 0:
        res[...] = dt * R
    else:
        res[...] = A[s] * res + dt * R
    Q[...] = Q + B[s] * res
    return Q, res


def step(Q, res, dt, rhs):
    """One LSERK45 time step (five stages) in place."""
    for s in range(NSTAGES):
        stage(s, Q, res, dt, rhs)
    return Q, res


def integrate(Q0, dt, nsteps, rhs):
    """Advance a copy of Q0 by ``nsteps`` steps; returns the final state."""
    Q = np.array(Q0, copy=True)
    res = np.zeros_like(Q)
    for _ in range(nsteps):
        step(Q, res, dt, rhs)
    return Q
