"""Derivatives of the DG right-hand side and of RK trajectories, by the
complex step.

The right-hand side of Eq. (5) is a real-analytic function of Q away from
the kinks of the Lax-Friedrichs wave speed (max and |.|).  Evaluating it at
Q + i h U with a tiny h gives J U = Im(RHS(Q + i h U)) / h to roundoff, with
no subtractive cancellation; the non-smooth operations branch on the real
part (oracle.euler), so the derivative taken is that of the branch the real
evaluation follows.  The transpose J^T V is obtained from the dense Jacobian
(columns J e_k), affordable on tiny meshes only.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

import numpy as np

from . import lserk

H = 1e-30


def jvp(dg, Q, U, h=H):
    """J(Q) U, J = d RHS / d Q."""
    Qc = np.asarray(Q, dtype=np.complex128) + 1j * h * np.asarray(U)
    return np.imag(dg.rhs(Qc)) / h


def jacobian(dg, Q, h=H):
    """Dense Jacobian [5 E N^3, 5 E N^3], one complex-step column per
    unknown (flattened in the array layout of Q)."""
    n = Q.size
    J = np.empty((n, n))
    E = np.zeros(n)
    for k in range(n):
        E[k] = 1.0
        J[:, k] = jvp(dg, Q, E.reshape(Q.shape), h).ravel()
        E[k] = 0.0
    return J


def vjp_dense(dg, Q, V, h=H):
    """J(Q)^T V from the dense Jacobian (tiny meshes)."""
    return (jacobian(dg, Q, h).T @ np.asarray(V).ravel()).reshape(Q.shape)


def kinetic_energy_after(dg, Q0, dt, nsteps):
    """Integrated kinetic energy |rho u|^2 / (2 rho) after ``nsteps`` LSERK45
    steps from Q0 (works for complex states)."""
    Q = lserk.integrate(Q0, dt, nsteps, dg.rhs)
    return dg.integrals(Q)[5]


def ke_directional_derivative(dg, Q0, U, dt, nsteps, h=H):
    """d/de KE(Q_nsteps(Q0 + e U)) at e = 0, by the complex step through the
    whole trajectory."""
    Qc = np.asarray(Q0, dtype=np.complex128) + 1j * h * np.asarray(U)
    return float(np.imag(kinetic_energy_after(dg, Qc, dt, nsteps)) / h)
