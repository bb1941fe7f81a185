"""Pointwise physics of the 3-D compressible Euler equations.

Section II-A: conservative variables Q = (rho, rho u, rho v, rho w, rho E),
Cartesian flux columns F^1, F^2, F^3 of Eq. (2) with total enthalpy
H = E + p/rho, and the ideal-gas closure of Eq. (3) with gamma = 1.4 by
default.  Section II-B: the face flux F* is the Lax-Friedrichs flux.

Every function accepts real or complex arrays.  For complex input the
non-smooth operations (absolute value, maximum) branch on the real part, so
that a complex-step derivative follows the branch that the real evaluation
takes.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

import numpy as np


def _abs(x):
    """|x| branching on the real part (x itself for complex-step use)."""
    return np.where(np.real(x) >= 0.0, x, -x)


def _max(a, b):
    """max(a, b) branching on real parts; ties select ``a``."""
    return np.where(np.real(a) >= np.real(b), a, b)


def pressure(q, gamma):
    """Eq. (3) solved for p: p = (gamma - 1)(rho E - |rho u|^2 / (2 rho))."""
    rho, mx, my, mz, en = q[0], q[1], q[2], q[3], q[4]
    return (gamma - 1.0) * (en - 0.5 * (mx * mx + my * my + mz * mz) / rho)


def flux(q, d, gamma):
    """Column F^(d+1) of Eq. (2) for d = 0, 1, 2 (x, y, z).

    F^d = (rho u_d, rho u u_d + p e_1[d], rho v u_d + p e_2[d],
           rho w u_d + p e_3[d], rho u_d H) with rho H = rho E + p.
    Returns an array shaped like ``q``.
    """
    p = pressure(q, gamma)
    ud = q[1 + d] / q[0]
    out = [q[1 + d], q[1] * ud, q[2] * ud, q[3] * ud, (q[4] + p) * ud]
    out[1 + d] = out[1 + d] + p
    return np.stack(out)


def sound_speed(q, gamma):
    """c = sqrt(gamma p / rho) for the ideal gas of Eq. (3)."""
    return np.sqrt(gamma * pressure(q, gamma) / q[0])


def lax_friedrichs(q_minus, q_plus, d, gamma):
    """Local Lax-Friedrichs flux in the +d direction across a face whose
    -d side carries ``q_minus`` and whose +d side carries ``q_plus``.

    F* = (F^d(Q-) + F^d(Q+))/2 - (lambda/2)(Q+ - Q-), with the local wave
    speed lambda = max(|u_d-| + c-, |u_d+| + c+) at the face point.
    The paper names the Lax-Friedrichs flux without fixing the wave-speed
    estimate; this local, per-face-point reading is the one the whole build
    uses.
    """
    fm = flux(q_minus, d, gamma)
    fp = flux(q_plus, d, gamma)
    lam_m = _abs(q_minus[1 + d] / q_minus[0]) + sound_speed(q_minus, gamma)
    lam_p = _abs(q_plus[1 + d] / q_plus[0]) + sound_speed(q_plus, gamma)
    lam = _max(lam_m, lam_p)
    return 0.5 * (fm + fp) - 0.5 * lam * (q_plus - q_minus)
