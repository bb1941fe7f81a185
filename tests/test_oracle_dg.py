"""Pins of the oracle's DG right-hand side (Section II-B, Eq. (5)) against
facts that the paper and the mathematics fix: free-stream preservation,
discrete conservation, invariance of the advected density wave, its
convergence rate, the p = 0 reduction to first-order Rusanov finite volume,
the reduction to the textbook 1-D nodal DG operator for data that vary along
one axis, and translation/axis-permutation equivariance.

The brute-force finite-volume and 1-D codes below are written independently
of ``oracle/`` (scalar loops, numpy's library Gauss-Legendre rule,
barycentric differentiation)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG, basis3d, tensor_points
from oracle.quadrature import gauss_legendre
from oracle import lserk

GAMMA = 1.4


# --------------------------------------------------------------------------
# independent scalar Euler helpers (test-side, used by the brute-force codes)
def _prim(q):
    rho = q[0]
    u = [q[1] / rho, q[2] / rho, q[3] / rho]
    p = (GAMMA - 1.0) * (q[4] - 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    return rho, u, p


def _flux_scalar(q, d):
    rho, u, p = _prim(q)
    f = [rho * u[d], rho * u[0] * u[d], rho * u[1] * u[d], rho * u[2] * u[d],
         (q[4] + p) * u[d]]
    f[1 + d] += p
    return f


def _rusanov_scalar(ql, qr, d):
    rl, ul, pl = _prim(ql)
    rr, ur, pr = _prim(qr)
    sl = abs(ul[d]) + math.sqrt(GAMMA * pl / rl)
    sr = abs(ur[d]) + math.sqrt(GAMMA * pr / rr)
    s = max(sl, sr)
    fl = _flux_scalar(ql, d)
    fr = _flux_scalar(qr, d)
    return [0.5 * (fl[m] + fr[m]) - 0.5 * s * (qr[m] - ql[m]) for m in range(5)]


def _summand_scale(dg, Q):
    """max over nodes and fields of sum_d (2/h_d)|F^d| max_i sum_a |w_a D_ai / w_i|:
    the magnitude of the terms that cancel in the right-hand side."""
    from oracle.euler import flux
    q = Q.reshape(5, -1)
    xi, w = gauss_legendre(dg.N)
    from oracle.quadrature import lagrange_deriv
    D = lagrange_deriv(xi, xi)
    dh = np.max(np.sum(np.abs(w[:, None] * D / w[None, :]), axis=0)) if dg.N > 1 else 1.0
    s = 0.0
    for d in range(3):
        s = s + (2.0 / dg.h[d]) * np.abs(flux(q, d, GAMMA))
    return float(np.max(s)) * max(dh, 1.0)


# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_mass_matrix_is_collocated_diagonal(p):
    dg = DG((2, 3, 4), p, L=(1.0, 0.7, 1.9))
    diag = dg.J * dg.wq
    off = dg.M - np.diag(np.diag(dg.M))
    assert np.max(np.abs(off)) < 1e-15 * np.max(diag)
    assert np.max(np.abs(np.diag(dg.M) - diag) / diag) < 1e-14


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_free_stream_preservation(p):
    rng = np.random.default_rng(100 + p)
    n = (3, 2, 4)
    for _ in range(3):
        rho = rng.uniform(0.5, 2.0)
        vel = tuple(rng.uniform(-2, 2, 3))
        pres = rng.uniform(0.5, 3.0)
        dg = DG(n, p, L=tuple(rng.uniform(0.5, 2.0, 3)))
        Q = W.uniform_state(n, p, rho, vel, pres)
        R = dg.rhs(Q)
        assert np.max(np.abs(R)) <= 1e-13 * _summand_scale(dg, Q)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_discrete_conservation(p):
    n = (3, 4, 2)
    L = (1.0, 1.3, 0.7)
    dg = DG(n, p, L=L)
    Q = W.random_smooth(n, p, seed=p, L=L, noise=0.05)
    R = dg.rhs(Q)
    w = (dg.J * dg.wq)
    r = R.reshape(5, -1, dg.N3)
    total = np.einsum("fet,t->f", r, w)
    absum = np.einsum("fet,t->f", np.abs(r), w)
    assert np.all(np.abs(total) <= 1e-13 * absum)
    # and the oracle's integrals agree with that sum
    assert np.allclose(dg.integrals(R)[:5], total, rtol=0, atol=1e-13 * absum.max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_density_wave_invariance(p):
    """With velocity and pressure uniform every equation is a multiple of the
    mass equation: RHS_m = u RHS_rho, RHS_E = |u|^2/2 RHS_rho."""
    vel = (0.3, -0.5, 0.7)
    n = (3, 3, 2)
    dg = DG(n, p)
    Q = W.density_wave(n, p, amp=0.25, k=(1, -1, 2), vel=vel, pres=1.3)
    R = dg.rhs(Q)
    scale = _summand_scale(dg, Q)
    for d in range(3):
        assert np.max(np.abs(R[1 + d] - vel[d] * R[0])) <= 1e-13 * scale
    assert np.max(np.abs(R[4] - 0.5 * sum(v * v for v in vel) * R[0])) <= 1e-13 * scale
    assert np.max(np.abs(R[0])) > 1e-3 * scale  # non-trivial


def _l2_density_error(dg, Qf, t, amp, k, vel):
    xo, wo = gauss_legendre(dg.N + 3)
    pts, ow = tensor_points(xo, wo)
    B = basis3d(dg.nodes, pts)
    rho = Qf[0].reshape(-1, dg.N3) @ B.T
    ez, ey, ex = np.unravel_index(np.arange(dg.E), (dg.nz, dg.ny, dg.nx))
    X = ex[:, None] * dg.h[0] + (pts[None, :, 0] + 1) * dg.h[0] / 2
    Y = ey[:, None] * dg.h[1] + (pts[None, :, 1] + 1) * dg.h[1] / 2
    Z = ez[:, None] * dg.h[2] + (pts[None, :, 2] + 1) * dg.h[2] / 2
    exact = W.density_wave_exact(X, Y, Z, t, amp=amp, k=k, vel=vel)
    return math.sqrt(np.sum((rho - exact) ** 2 * ow[None, :]) * dg.J)


def _wave_error(n, p, k, T, cfl=0.3):
    dg = DG(n, p)
    vel = (1.0, 1.0, 1.0)
    Q = W.density_wave(n, p, amp=0.2, k=k, vel=vel)
    dt = dg.dt_cfl(Q, cfl)
    ns = int(math.ceil(T / dt))
    Qf = lserk.integrate(Q, T / ns, ns, dg.rhs)
    return _l2_density_error(dg, Qf, T, 0.2, k, vel)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("p,ns", [(1, (8, 16, 32)), (2, (8, 16, 32)), (3, (4, 8, 16)), (4, (8, 16))])
def test_density_wave_convergence_rate_axis(axis, p, ns):
    """Closed-form advected wave along one axis on an n x 1 x 1 mesh
    (rotated to each axis): L2 error at T = 0.1 converges at rate ~ p+1."""
    k = [0, 0, 0]
    k[axis] = 1
    errs = []
    for n in ns:
        mesh = [1, 1, 1]
        mesh[axis] = n
        errs.append(_wave_error(tuple(mesh), p, tuple(k), 0.1))
    rate = math.log2(errs[-2] / errs[-1])
    assert rate >= p + 0.7, (errs, rate)


@pytest.mark.parametrize("p", [1, 3])
def test_density_wave_convergence_rate_diagonal(p):
    """The fully 3-D wave rho = 1 + 0.2 sin(2 pi (x + y + z - 3 t)) of the
    first workload (u = v = w = 1, pressure 1)."""
    errs = [_wave_error((n, n, n), p, (1, 1, 1), 0.02) for n in (4, 8)]
    rate = math.log2(errs[0] / errs[1])
    assert rate >= p + 0.7, (errs, rate)


# --------------------------------------------------------------------------
def _fv_rusanov_rhs(Q, h):
    """First-order finite volume with the Rusanov flux, scalar loops."""
    _, nz, ny, nx = Q.shape
    out = np.zeros_like(Q)
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                c = (ez, ey, ex)
                qc = list(Q[(slice(None),) + c])
                for d in range(3):
                    up = list(c)
                    dn = list(c)
                    ax = 2 - d
                    size = (nz, ny, nx)[ax]
                    up[ax] = (up[ax] + 1) % size
                    dn[ax] = (dn[ax] - 1) % size
                    qu = list(Q[(slice(None),) + tuple(up)])
                    qd = list(Q[(slice(None),) + tuple(dn)])
                    fp = _rusanov_scalar(qc, qu, d)
                    fm = _rusanov_scalar(qd, qc, d)
                    for m in range(5):
                        out[(m,) + c] -= (fp[m] - fm[m]) / h[d]
    return out


def test_p0_is_rusanov_finite_volume():
    n = (4, 3, 5)
    L = (1.0, 0.8, 1.5)
    dg = DG(n, 0, L=L)
    Q = W.random_smooth(n, 0, seed=3, L=L, noise=0.2)
    R = dg.rhs(Q)
    ref = _fv_rusanov_rhs(Q.reshape(5, n[2], n[1], n[0]), dg.h)
    assert np.max(np.abs(R.reshape(ref.shape) - ref)) <= 1e-13 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
def _textbook_1d_dg(q, h, N, d):
    """1-D collocated nodal DG along axis d (Hesthaven-Warburton form):
    dq_i/dt = (2/h)/w_i [sum_a w_a D_ai F(q_a) - l_i(1) F*_R + l_i(-1) F*_L],
    with D from barycentric weights.  q[5, n, N] -> same shape."""
    xi, w = np.polynomial.legendre.leggauss(N)
    lam = np.array([1.0 / np.prod([xi[i] - xi[m] for m in range(N) if m != i]) for i in range(N)])
    D = np.zeros((N, N))
    for a in range(N):
        for i in range(N):
            if a != i:
                D[a, i] = (lam[i] / lam[a]) / (xi[a] - xi[i])
        D[a, a] = -sum(D[a, i] for i in range(N) if i != a)

    def lag_at(x):
        return np.array([np.prod([(x - xi[m]) / (xi[i] - xi[m]) for m in range(N) if m != i])
                         for i in range(N)])
    lp, lm = lag_at(1.0), lag_at(-1.0)
    _, n, _ = q.shape
    out = np.zeros_like(q)
    for e in range(n):
        qe = q[:, e, :]
        fl = np.array([_flux_scalar(qe[:, a], d) for a in range(N)]).T  # [5, N]
        right = _rusanov_scalar(list(qe @ lp), list(q[:, (e + 1) % n, :] @ lm), d)
        left = _rusanov_scalar(list(q[:, (e - 1) % n, :] @ lp), list(qe @ lm), d)
        for i in range(N):
            vol = (fl * (w * D[:, i])[None, :]).sum(axis=1)
            out[:, e, i] = (2.0 / h) / w[i] * (vol - lp[i] * np.array(right) + lm[i] * np.array(left))
    return out


@pytest.mark.parametrize("p", [1, 2, 4])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_reduces_to_textbook_1d_dg(p, d):
    N = p + 1
    n1 = 5
    rng = np.random.default_rng(10 * p + d)
    # a 1-D state varying along axis d, with transverse velocities
    rho = rng.uniform(0.7, 1.3, (n1, N))
    u = rng.uniform(-0.6, 0.6, (3, n1, N))
    pr = rng.uniform(0.7, 1.5, (n1, N))
    q1 = W.conserved(rho, u[0], u[1], u[2], pr)          # [5, n1, N]
    mesh = [2, 3, 2]
    mesh[d] = n1
    L = [1.0, 1.2, 0.9]
    dg = DG(tuple(mesh), p, L=tuple(L))
    # broadcast into the 3-D layout Q[f, ez, ey, ex, k, j, i]
    Q = np.zeros(dg.shape)
    e_ax, n_ax = 3 - d, 6 - d
    for e in range(n1):
        for a in range(N):
            idx = [slice(None)] * 7
            idx[e_ax] = e
            idx[n_ax] = a
            Q[tuple(idx)] = q1[:, e, a].reshape(5, 1, 1, 1, 1)
    R = dg.rhs(Q)
    ref = _textbook_1d_dg(q1, dg.h[d], N, d)
    scale = _summand_scale(dg, Q)
    for e in range(n1):
        for a in range(N):
            idx = [slice(None)] * 7
            idx[e_ax] = e
            idx[n_ax] = a
            got = R[tuple(idx)].reshape(5, -1)
            assert np.max(np.abs(got - ref[:, e, a][:, None])) <= 1e-13 * scale


# --------------------------------------------------------------------------
def test_translation_equivariance():
    n = (4, 3, 5)
    dg = DG(n, 2, L=(1.0, 0.9, 1.1))
    Q = W.random_smooth(n, 2, seed=5, L=(1.0, 0.9, 1.1), noise=0.05)
    R = dg.rhs(Q)
    for ax in (1, 2, 3):
        Rs = dg.rhs(np.roll(Q, 1, axis=ax))
        assert np.max(np.abs(Rs - np.roll(R, 1, axis=ax))) <= 1e-14 * np.max(np.abs(R))


def test_axis_permutation_equivariance():
    """Swapping x and y (mesh sizes, lengths, node axes and momentum
    components) permutes the right-hand side the same way."""
    n = (4, 3, 2)
    L = (1.0, 0.9, 1.1)
    dg = DG(n, 2, L=L)
    Q = W.random_smooth(n, 2, seed=6, L=L, noise=0.05)
    R = dg.rhs(Q)

    def swap_xy(A):
        B = np.swapaxes(np.swapaxes(A, 2, 3), 5, 6)
        return B[[0, 2, 1, 3, 4]]
    dg2 = DG((n[1], n[0], n[2]), 2, L=(L[1], L[0], L[2]))
    R2 = dg2.rhs(np.ascontiguousarray(swap_xy(Q)))
    assert np.max(np.abs(R2 - swap_xy(R))) <= 1e-13 * np.max(np.abs(R))


# --------------------------------------------------------------------------
def test_integrals_closed_form():
    """A state linear in x inside the domain is interpolated exactly for
    p >= 1, so its integrals have closed forms: int rho = V (1 + Lx/2)."""
    n = (3, 2, 4)
    L = (1.5, 0.8, 1.2)
    p = 2
    dg = DG(n, p, L=L)
    X, Y, Z = W.node_coords(n, p, L)
    rho = 1.0 + X
    u = np.full_like(rho, 0.5)
    Q = W.conserved(rho, u, 0 * u, 0 * u, np.ones_like(rho))
    I = dg.integrals(Q)
    V = L[0] * L[1] * L[2]
    assert abs(I[0] - V * (1 + L[0] / 2)) < 1e-13
    assert abs(I[1] - 0.5 * V * (1 + L[0] / 2)) < 1e-13
    assert abs(I[5] - 0.125 * V * (1 + L[0] / 2)) < 1e-13   # KE = rho u^2 / 2
    assert abs(I[4] - (V / 0.4 + 0.125 * V * (1 + L[0] / 2))) < 1e-12


def test_max_rate_uniform_closed_form():
    n = (2, 3, 4)
    L = (1.0, 1.5, 2.0)
    dg = DG(n, 1, L=L)
    Q = W.uniform_state(n, 1, 1.2, (0.5, -0.25, 1.0), 0.9)
    c = math.sqrt(1.4 * 0.9 / 1.2)
    h = np.array(L) / np.array(n)
    expect = sum((abs(v) + c) / hh for v, hh in zip((0.5, -0.25, 1.0), h))
    assert abs(dg.max_rate(Q) - expect) < 1e-13 * expect


def test_check_state():
    n = (2, 2, 2)
    dg = DG(n, 1)
    Q = W.uniform_state(n, 1, 1.0, (0.1, 0.2, 0.3), 1.0)
    assert dg.check_state(Q)
    Q2 = Q.copy()
    Q2[0, 0, 0, 0, 0, 0, 0] = -1.0
    assert not dg.check_state(Q2)
    Q3 = Q.copy()
    Q3[4, 1, 1, 1, 1, 1, 1] = 0.0    # negative pressure
    assert not dg.check_state(Q3)
    Q4 = Q.copy()
    Q4[2, 0, 1, 0, 1, 0, 1] = np.nan
    assert not dg.check_state(Q4)
