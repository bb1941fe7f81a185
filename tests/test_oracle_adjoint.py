"""Pins of the oracle's complex-step derivatives against central finite
differences of the oracle's own real evaluation, and against the free-stream
property of the linearised operator."""

import numpy as np

import workloads as W
from oracle import adjoint
from oracle.dg import DG


def test_jvp_matches_central_differences():
    n, p = (2, 3, 2), 2
    dg = DG(n, p, L=(1.0, 1.1, 0.9))
    Q = W.random_smooth(n, p, seed=3, L=(1.0, 1.1, 0.9), noise=0.05)
    rng = np.random.default_rng(4)
    for _ in range(3):
        U = rng.standard_normal(Q.shape) * np.abs(Q).reshape(5, -1).mean(1).reshape(5, 1, 1, 1, 1, 1, 1)
        jv = adjoint.jvp(dg, Q, U)
        h = 1e-6
        fd = (dg.rhs(Q + h * U) - dg.rhs(Q - h * U)) / (2 * h)
        assert np.max(np.abs(jv - fd)) <= 1e-6 * np.max(np.abs(jv))


def test_linearised_free_stream():
    """At a uniform state, a uniform perturbation is again a uniform state,
    so J U = 0 (to the summand scale)."""
    n, p = (2, 2, 3), 3
    dg = DG(n, p)
    Q = W.uniform_state(n, p, 1.2, (0.4, -0.3, 0.2), 1.7)
    U = np.ones_like(Q) * np.array([0.3, -0.2, 0.5, 0.1, 0.7]).reshape(5, 1, 1, 1, 1, 1, 1)
    jv = adjoint.jvp(dg, Q, U)
    assert np.max(np.abs(jv)) <= 1e-12 * np.max(np.abs(dg.rhs(W.random_smooth(n, p, seed=1))))


def test_dense_jacobian_columns_and_transpose():
    n, p = (1, 2, 1), 1
    dg = DG(n, p)
    Q = W.random_smooth(n, p, seed=5, noise=0.05)
    J = adjoint.jacobian(dg, Q)
    rng = np.random.default_rng(6)
    U = rng.standard_normal(Q.shape)
    V = rng.standard_normal(Q.shape)
    assert np.allclose(J @ U.ravel(), adjoint.jvp(dg, Q, U).ravel(), rtol=0, atol=1e-12 * np.abs(J).max())
    lhs = np.dot(adjoint.jvp(dg, Q, U).ravel(), V.ravel())
    rhs = np.dot(U.ravel(), adjoint.vjp_dense(dg, Q, V).ravel())
    assert abs(lhs - rhs) <= 1e-12 * np.abs(J).max() * np.linalg.norm(U) * np.linalg.norm(V)


def test_trajectory_derivative_matches_central_differences():
    n, p = (2, 2, 2), 2
    L = (2 * np.pi,) * 3
    dg = DG(n, p, L=L)
    Q0 = W.perturbed_tgv(n, p, seed=1, L=L)
    dt = dg.dt_cfl(Q0, 0.3)
    U = W.gaussian_directions(Q0, 1, seed0=1000)[0]
    d_cs = adjoint.ke_directional_derivative(dg, Q0, U, dt, 4)
    h = 1e-6
    fp = adjoint.kinetic_energy_after(dg, Q0 + h * U, dt, 4)
    fm = adjoint.kinetic_energy_after(dg, Q0 - h * U, dt, 4)
    d_fd = (fp - fm) / (2 * h)
    # central differences carry a roundoff error ~ eps |KE| / h and a
    # truncation error ~ h^2; the complex step carries neither
    floor = 20 * np.finfo(float).eps * abs(fp) / h
    assert abs(d_cs - d_fd) <= floor + 1e-6 * abs(d_cs)
    assert abs(d_cs) > 100 * floor
