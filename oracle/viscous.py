"""Viscous (Navier-Stokes) terms on the same nodal DG discretisation, as
their plain definition.

The paper names CartDG's viscous formulation (Section III, Fig. 2: the CPU
code's sustained performance is quoted for it) but prints no viscous
discretisation.  The reading taken here, for the oracle and the GPU alike:

  Physics.  Compressible Navier-Stokes with constant dynamic viscosity mu,
  Stokes' hypothesis, Fourier heat conduction at constant Prandtl number Pr,
  and the ideal gas of Eq. (3) with gas constant 1, so that the temperature
  is T = p / rho, c_p = gamma / (gamma - 1) and the conductivity is
  kappa = mu c_p / Pr:
      tau_kd = mu (du_k/dx_d + du_d/dx_k - 2/3 delta_kd div u),
      F_v^d  = (0, tau_1d, tau_2d, tau_3d, u_k tau_kd + kappa dT/dx_d),
  and the equations read dQ/dt + div F(Q) = div F_v(Q, grad Q).

  Discretisation (Bassi & Rebay's first scheme, "BR1").  The primitive
  quantities P = (u, v, w, T) are represented by their nodal interpolants
  P_h on the collocated Gauss-Legendre basis of Eqs. (6)-(7).  Their
  gradient theta_d is the weak derivative with the central face value:
      int theta_d phi = -int P_h dphi/dx_d + oint {P_h} n_d phi,
  {.} the mean of the two sides' traces.  The viscous flux is evaluated at
  the nodes from (Q, theta) and represented by its nodal interpolant F_v,h;
  it enters Eq. (5) next to the inviscid flux with the central face value:
      int phi dQ/dt = int (F - F_v,h) . grad phi - oint (F* - {F_v,h}) . n phi.

Everything is evaluated densely with the matrices of ``oracle.dg.DG``
(volume quadrature, basis gradients, face traces, over-integrated mass
matrix solved densely), element by element over all elements at once.
TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

import numpy as np

from .dg import DG, NFIELDS
from .euler import pressure


class NavierStokesDG(DG):
    """``oracle.dg.DG`` plus the viscous terms above.  mu >= 0 (mu = 0 gives
    the Euler right-hand side exactly), prandtl > 0."""

    def __init__(self, n, p, L=(1.0, 1.0, 1.0), gamma=1.4, mu=0.0, prandtl=0.72):
        super().__init__(n, p, L=L, gamma=gamma)
        self.mu = float(mu)
        self.prandtl = float(prandtl)
        self.kappa = self.mu * (self.gamma / (self.gamma - 1.0)) / self.prandtl

    # ------------------------------------------------------------- pieces
    def primitives(self, Q):
        """Nodal (u, v, w, T) with T = p / rho, shaped [4, nz, ny, nx, N3]."""
        q = np.asarray(Q).reshape(NFIELDS, self.nz, self.ny, self.nx, self.N3)
        rho = q[0]
        T = pressure(q, self.gamma) / rho
        return np.stack([q[1] / rho, q[2] / rho, q[3] / rho, T])

    def _weak_derivative(self, X, d):
        """M^{-1} (-int X_h dphi/dx_d + oint {X_h} n_d phi) per element for
        every field of X [nf, nz, ny, nx, N3] (nodal values), the central
        face value {X_h} being the mean of the traces of both elements."""
        N3 = self.N3
        nf = X.shape[0]
        flat = X.reshape(-1, N3)
        Xq = (flat @ self.Phi.T).reshape(X.shape)                    # X_h at the quadrature points
        V = ((Xq * (self.J * self.wq)).reshape(-1, N3) @ self.Grad[d]).reshape(X.shape)
        ax = 3 - d + 0                                                 # axis of direction d in [f, z, y, x, t]
        Bp, Bm = self.Bface[(d, 1)], self.Bface[(d, -1)]
        own = (flat @ Bp.T).reshape(X.shape[:-1] + (-1,))             # trace on the +d face
        nbr = (np.roll(X, -1, axis=ax).reshape(-1, N3) @ Bm.T).reshape(X.shape[:-1] + (-1,))
        mean = 0.5 * (own + nbr) * (self.Jf[d] * self.wface)
        S = (mean.reshape(-1, mean.shape[-1]) @ Bp).reshape(X.shape)           # +d face, n_d = +1
        S -= np.roll((mean.reshape(-1, mean.shape[-1]) @ Bm).reshape(X.shape), 1, axis=ax)  # -d face of e+1
        out = np.linalg.solve(self.M, (S - V).reshape(-1, N3).T).T
        return out.reshape((nf,) + X.shape[1:])

    def gradients(self, Q):
        """theta[d, k]: the BR1 gradient along x_d of primitive k (u, v, w, T)
        at the nodes, shaped [3, 4, nz, ny, nx, N3]."""
        P = self.primitives(Q)
        return np.stack([self._weak_derivative(P, d) for d in range(3)])

    def viscous_flux(self, Q, theta):
        """F_v^d at the nodes for d = 0, 1, 2, shaped [3, 5, nz, ny, nx, N3]."""
        P = self.primitives(Q)
        vel = P[:3]
        grad_u = theta[:, :3]                  # grad_u[d, k] = du_k / dx_d
        div = grad_u[0, 0] + grad_u[1, 1] + grad_u[2, 2]
        out = np.zeros((3, NFIELDS) + P.shape[1:], dtype=np.result_type(P.dtype, theta.dtype))
        for d in range(3):
            en = self.kappa * theta[d, 3]
            for k in range(3):
                tau = self.mu * (grad_u[d, k] + grad_u[k, d])
                if k == d:
                    tau = tau - (2.0 / 3.0) * self.mu * div
                out[d, 1 + k] = tau
                en = en + vel[k] * tau
            out[d, 4] = en
        return out

    def rhs_viscous(self, Q):
        """The viscous part of dQ/dt: M^{-1} (-int F_v,h . grad phi +
        oint {F_v,h} . n phi), in the layout of Q."""
        Q = np.asarray(Q)
        if Q.shape != self.shape:
            raise ValueError(f"Q has shape {Q.shape}, expected {self.shape}")
        Fv = self.viscous_flux(Q, self.gradients(Q))
        total = np.zeros(Fv.shape[1:], dtype=Fv.dtype)
        for d in range(3):
            total += self._weak_derivative(Fv[d], d)
        return total.reshape(self.shape)

    def rhs(self, Q):
        """dQ/dt of the Navier-Stokes equations: the Euler right-hand side of
        Eq. (5) plus the viscous part."""
        R = super().rhs(Q)
        if self.mu == 0.0:
            return R
        return R + self.rhs_viscous(Q)

    def dt_cfl(self, Q, cfl):
        """The Euler time step of ``DG.dt_cfl`` limited by the viscous one:
        dt = CFL / ((2p+1) max_rate + (2p+1)^2 nu_max sum_d 1/h_d^2), with
        nu_max the larger of mu/rho and kappa/(rho c_v) over the nodes.  The
        paper gives no rule; this reading only picks dt."""
        q = np.asarray(Q).reshape(NFIELDS, -1)
        cv = 1.0 / (self.gamma - 1.0)
        nu = float(np.max(np.maximum(self.mu / q[0], self.kappa / (q[0] * cv))))
        k = 2 * self.p + 1
        rate = k * self.max_rate(Q) + k * k * nu * float(np.sum(1.0 / self.h ** 2))
        return cfl / rate
