"""The nodal DG right-hand side of the 3-D Euler equations, as its plain
definition.

Section II-B, Eq. (5): for every element Omega_k and every test function
psi_s = phi_s,

    int phi_s dQ/dt  =  int (F . grad) phi_s  -  oint (F* . n) phi_s,

with phi_s the tensor product of the 1-D Lagrange polynomials of Eq. (7)
through N = p+1 Gauss-Legendre points per direction, the volume and face
integrals evaluated by Gauss-Legendre quadrature at those same points
(collocation, Section I and II-B), F* the local Lax-Friedrichs flux, and the
mesh a periodic Cartesian grid of nx*ny*nz equal boxes (Sections I and V).

This module evaluates that definition densely: the basis, its gradients and
its face traces are evaluated at the quadrature points as N^3-column
matrices, every contraction is a dense matrix product over all N^3 nodes
(O(N^6) per element, no sum factorisation), and the mass matrix is formed by
an independent over-integration with N+2 points per direction and solved
densely.  Nothing assumes that the mass matrix is diagonal.

Array layout (the data format shared with the inputs): Q[f, ez, ey, ex, k, j, i]
with the fields f = rho, rho u, rho v, rho w, rho E, element indices ex
fastest among elements and i (the x node index) fastest inside an element.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

import numpy as np

from .quadrature import gauss_legendre, lagrange, lagrange_deriv
from .euler import flux, lax_friedrichs, pressure, sound_speed

NFIELDS = 5


def basis3d(nodes, pts, deriv=None):
    """Values of the tensor-product basis phi_t(xi, eta, zeta) =
    l_i(xi) l_j(eta) l_k(zeta), t = (k N + j) N + i, at the reference
    points ``pts`` [m, 3].  With ``deriv`` = d the factor along reference
    axis d is differentiated.  Returns B[m, t]."""
    pts = np.asarray(pts, dtype=np.float64)
    n = len(nodes)
    fac = []
    for d in range(3):
        if deriv == d:
            fac.append(lagrange_deriv(nodes, pts[:, d]))
        else:
            fac.append(lagrange(nodes, pts[:, d]))
    b = fac[2][:, :, None, None] * fac[1][:, None, :, None] * fac[0][:, None, None, :]
    return b.reshape(len(pts), n ** 3)


def tensor_points(x1d, w1d):
    """Tensor grid of a 1-D rule: points [(c M + b) M + a] = (x_a, x_b, x_c)
    with weight w_a w_b w_c."""
    m = len(x1d)
    c, b, a = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    pts = np.stack([x1d[a], x1d[b], x1d[c]], axis=1)
    return pts, w1d[a] * w1d[b] * w1d[c]


def face_points(x1d, w1d, d, side):
    """Face quadrature on the face xi_d = side (side = -1 or +1): the tensor
    grid of the two tangential Gauss-Legendre rules in increasing axis order,
    the lower tangential axis fastest.  Returns (points [N^2, 3], weights)."""
    m = len(x1d)
    hi, lo = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    lo, hi = lo.ravel(), hi.ravel()
    tang = [a for a in range(3) if a != d]
    pts = np.zeros((m * m, 3))
    pts[:, d] = float(side)
    pts[:, tang[0]] = x1d[lo]
    pts[:, tang[1]] = x1d[hi]
    return pts, w1d[lo] * w1d[hi]


class DG:
    """Periodic Cartesian mesh of nx*ny*nz elements on [0,Lx]x[0,Ly]x[0,Lz]
    with polynomial degree p (N = p+1 points per direction) and ratio of
    specific heats gamma."""

    def __init__(self, n, p, L=(1.0, 1.0, 1.0), gamma=1.4):
        self.nx, self.ny, self.nz = (int(v) for v in n)
        if min(self.nx, self.ny, self.nz) < 1 or p < 0:
            raise ValueError("mesh sizes must be >= 1 and p >= 0")
        self.p = int(p)
        self.N = self.p + 1
        self.N3 = self.N ** 3
        self.L = np.asarray(L, dtype=np.float64)
        self.gamma = float(gamma)
        self.h = self.L / np.array([self.nx, self.ny, self.nz], dtype=np.float64)
        hx, hy, hz = self.h
        # Affine map x = x0 + (xi + 1) h / 2 per direction: d xi_d / d x_d = 2/h_d,
        # volume Jacobian h_x h_y h_z / 8, face Jacobians (product of the two
        # tangential half-widths).
        self.J = hx * hy * hz / 8.0
        self.Jf = np.array([hy * hz / 4.0, hx * hz / 4.0, hx * hy / 4.0])
        self.nodes, self.weights = gauss_legendre(self.N)
        # Volume quadrature at the collocated Gauss-Legendre points.
        self.qpts, self.wq = tensor_points(self.nodes, self.weights)
        self.Phi = basis3d(self.nodes, self.qpts)
        self.Grad = [basis3d(self.nodes, self.qpts, deriv=d) * (2.0 / self.h[d])
                     for d in range(3)]
        # Face matrices and weights for the faces xi_d = -1 and xi_d = +1.
        self.Bface = {}
        self.wface = None
        for d in range(3):
            for side in (-1, 1):
                fp, fw = face_points(self.nodes, self.weights, d, side)
                self.Bface[(d, side)] = basis3d(self.nodes, fp)
                self.wface = fw
        # Mass matrix by over-integration (N+2 points per direction), dense.
        xo, wo = gauss_legendre(self.N + 2)
        opts, ow = tensor_points(xo, wo)
        po = basis3d(self.nodes, opts)
        self.M = self.J * (po.T * ow[None, :]) @ po

    # ------------------------------------------------------------------ utils
    @property
    def E(self):
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (NFIELDS, self.nz, self.ny, self.nx, self.N, self.N, self.N)

    def num_dof(self):
        """Solution nodes E N^3 (the paper's DOF count, Section V)."""
        return self.E * self.N3

    def _axis(self, d):
        """Array axis of direction d in the [f, ez, ey, ex, t] view."""
        return 3 - d

    # -------------------------------------------------------------------- rhs
    def rhs(self, Q):
        """dQ/dt of Eq. (5): M^{-1} (V - S) per element, returned in the
        layout of ``Q``.  Works for real and complex Q."""
        Q = np.asarray(Q)
        if Q.shape != self.shape:
            raise ValueError(f"Q has shape {Q.shape}, expected {self.shape}")
        N3 = self.N3
        q = Q.reshape(NFIELDS, self.nz, self.ny, self.nx, N3)
        flat = q.reshape(-1, N3)
        # Solution at the volume quadrature points: Q_h(x_q) = sum_t Q_t phi_t(x_q).
        qq = (flat @ self.Phi.T).reshape(q.shape)
        # Volume term of Eq. (5): V_s = sum_q J w_q sum_d F^d(Q_h(x_q)) d phi_s/d x_d (x_q).
        V = np.zeros(q.shape, dtype=np.result_type(Q.dtype, np.float64))
        for d in range(3):
            Fd = flux(qq, d, self.gamma) * (self.J * self.wq)
            V += (Fd.reshape(-1, N3) @ self.Grad[d]).reshape(q.shape)
        # Surface term of Eq. (5): S_s = sum over faces of oint (F* . n_out) phi_s.
        S = np.zeros_like(V)
        for d in range(3):
            ax = self._axis(d)
            Bp = self.Bface[(d, 1)]
            Bm = self.Bface[(d, -1)]
            # Traces on the +d face of every element (its own side) and on the
            # -d face of its +d neighbour (the other side of the same face).
            q_minus = (flat @ Bp.T).reshape(q.shape[:-1] + (-1,))
            q_nbr = np.roll(q, -1, axis=ax)
            q_plus = (q_nbr.reshape(-1, N3) @ Bm.T).reshape(q.shape[:-1] + (-1,))
            fstar = lax_friedrichs(q_minus, q_plus, d, self.gamma)
            fw = fstar * (self.Jf[d] * self.wface)
            # Element e, face +d, n_out = +e_d.
            S += (fw.reshape(-1, fw.shape[-1]) @ Bp).reshape(q.shape)
            # Neighbour e+1, its face -d, n_out = -e_d.
            contrib = (fw.reshape(-1, fw.shape[-1]) @ Bm).reshape(q.shape)
            S -= np.roll(contrib, 1, axis=ax)
        rhs = np.linalg.solve(self.M, (V - S).reshape(-1, N3).T).T
        return rhs.reshape(self.shape)

    # -------------------------------------------------------------- integrals
    def integrals(self, Q):
        """Domain integrals of the five conserved fields and of the kinetic
        energy |rho u|^2/(2 rho), by the nodal Gauss-Legendre rule
        (sum_e J sum_q w_q (.)(x_q)); exact for the polynomial Q_h.
        Returns 6 numbers."""
        q = np.asarray(Q).reshape(NFIELDS, -1, self.N3)
        w = self.J * self.wq
        cons = np.einsum("fet,t->f", q, w)
        ke = np.einsum("et,t->", 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0], w)
        return np.concatenate([cons, [ke]])

    def max_rate(self, Q):
        """max over nodes of sum_d (|u_d| + c) / h_d  (units 1/time)."""
        q = np.asarray(Q).reshape(NFIELDS, -1)
        c = sound_speed(q, self.gamma)
        r = sum((np.abs(q[1 + d] / q[0]) + c) / self.h[d] for d in range(3))
        return float(np.max(r))

    def dt_cfl(self, Q, cfl):
        """Time step dt = CFL / ((2p+1) max_rate(Q)).  The paper gives no CFL
        rule; this one is a reading of ours, used only to pick dt."""
        return cfl / ((2 * self.p + 1) * self.max_rate(Q))

    def check_state(self, Q):
        """True when every node has finite values, rho > 0 and p > 0."""
        q = np.asarray(Q).reshape(NFIELDS, -1)
        if not np.all(np.isfinite(q)):
            return False
        return bool(np.all(q[0] > 0) and np.all(pressure(q, self.gamma) > 0))
