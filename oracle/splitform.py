"""Kinetic-energy-preserving split-form volume term on the same nodal DG
discretisation, as its plain definition.

The paper cites kinetic-energy-preserving flux schemes in its authors' DG
framework (reference list) without printing one.  The reading taken here,
for the oracle and the GPU alike:

  Two-point flux (Kennedy & Gruber's split of the convective terms, which
  satisfies Jameson's kinetic-energy-preservation condition: the momentum
  flux is the mass flux times the mean velocity plus a pressure term), in
  direction d with {a} = (a_L + a_R)/2, e = E/rho the specific total energy:
      f_S^rho    = {rho}{u_d}
      f_S^(rho u_k) = {rho}{u_d}{u_k} + {p} delta_kd
      f_S^(rho E) = {rho}{u_d}{e} + {p}{u_d}
  consistent (f_S(Q, Q) = F^d(Q) of Eq. (2)) and symmetric.

  Volume term (flux differencing on the collocated Gauss-Legendre basis,
  whose nodes do not include the element ends): along every d-line of an
  element the N nodes are coupled to the two face points by the
  "hybridised" summation-by-parts operator
      Q_N = [[Q - E^T B E / 2,  E^T B / 2], [-B E / 2,  B / 2]],
  Q = M D (M = diag(w), D_ia = l_a'(xi_i)), E (2 x N) the face
  interpolation matrix (rows l_a(-1), l_a(+1)), B = diag(-1, +1), acting on
  the N nodal states and the two face traces q~ = E q.  Per line,
      M dq/dt = -(2/h_d) ( [I, E^T] (2 Q_N o F_S) 1 + E^T B (F* - F^d(q~)) ),
  (2 Q_N o F_S) 1 the row sums of Q_N times the two-point fluxes between the
  line's N + 2 states, F* the local Lax-Friedrichs flux of the standard
  scheme at the two face points, summed over the three directions.  With the
  central two-point flux (F^d(Q_L) + F^d(Q_R))/2 this is algebraically the
  weak form of Eq. (5) that ``oracle.dg.DG`` evaluates.

Evaluated per line with dense (N+2) x (N+2) operators for all lines of all
elements at once.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

import numpy as np

from .dg import DG, NFIELDS
from .euler import flux, lax_friedrichs, pressure
from .quadrature import lagrange, lagrange_deriv


def kg_flux(qa, qb, d, gamma):
    """Kennedy-Gruber two-point flux in direction d between states qa and qb
    (arrays [5, ...] broadcasting against each other)."""
    ra, rb = qa[0], qb[0]
    ua = [qa[1 + k] / ra for k in range(3)]
    ub = [qb[1 + k] / rb for k in range(3)]
    pa, pb = pressure(qa, gamma), pressure(qb, gamma)
    ea, eb = qa[4] / ra, qb[4] / rb
    rho = 0.5 * (ra + rb)
    ud = 0.5 * (ua[d] + ub[d])
    pm = 0.5 * (pa + pb)
    mass = rho * ud
    out = [mass]
    for k in range(3):
        m = mass * (0.5 * (ua[k] + ub[k]))
        if k == d:
            m = m + pm
        out.append(m)
    out.append(mass * (0.5 * (ea + eb)) + pm * ud)
    return np.stack(np.broadcast_arrays(*out))


def central_flux(qa, qb, d, gamma):
    """The central two-point flux (F^d(qa) + F^d(qb)) / 2."""
    return 0.5 * (flux(qa, d, gamma) + flux(qb, d, gamma))


class SplitFormDG(DG):
    """``oracle.dg.DG`` with the split-form volume term above.  two_point is
    ``kg_flux`` (default) or any symmetric consistent two-point flux."""

    def __init__(self, n, p, L=(1.0, 1.0, 1.0), gamma=1.4, two_point=kg_flux):
        super().__init__(n, p, L=L, gamma=gamma)
        self.two_point = two_point
        N = self.N
        x = self.nodes
        self.D = lagrange_deriv(x, x)                   # D[i, a] = l_a'(xi_i)
        self.Q1 = np.diag(self.weights) @ self.D
        self.E1 = np.vstack([lagrange(x, [-1.0]), lagrange(x, [1.0])])   # (2, N)
        self.B1 = np.diag([-1.0, 1.0])
        Qn = np.zeros((N + 2, N + 2))
        Qn[:N, :N] = self.Q1 - 0.5 * self.E1.T @ self.B1 @ self.E1
        Qn[:N, N:] = 0.5 * self.E1.T @ self.B1
        Qn[N:, :N] = -0.5 * self.B1 @ self.E1
        Qn[N:, N:] = 0.5 * self.B1
        self.QN = Qn

    def _lines(self, q, d):
        """View of q [f, nz, ny, nx, N, N, N] as lines along direction d:
        [f, nz, ny, nx, N, N, N(line)] with the line index last."""
        ax = {0: 6, 1: 5, 2: 4}[d]
        return np.moveaxis(q, ax, -1)

    def rhs(self, Q):
        """dQ/dt of the split form, in the layout of Q."""
        Q = np.asarray(Q)
        if Q.shape != self.shape:
            raise ValueError(f"Q has shape {Q.shape}, expected {self.shape}")
        N = self.N
        out = np.zeros(Q.shape, dtype=np.result_type(Q.dtype, np.float64))
        for d in range(3):
            lines = self._lines(Q, d)                                  # [..., N]
            tr = np.einsum("fa,...a->...f", self.E1, lines)           # traces [..., 2]: (-1, +1)
            st = np.concatenate([lines, tr], axis=-1)                 # N + 2 states per line
            Fs = self.two_point(st[..., :, None], st[..., None, :], d, self.gamma)   # [5, ..., N+2, N+2]
            vol = np.einsum("ij,...ij->...i", 2.0 * self.QN, Fs)      # row sums [5, ..., N+2]
            r = vol[..., :N] + np.einsum("fi,...f->...i", self.E1, vol[..., N:])
            # the local Lax-Friedrichs flux on the two faces of every line:
            # the -d face pairs the -d neighbour's + trace with our - trace
            ax = 3 - d
            t_minus, t_plus = tr[..., 0], tr[..., 1]
            nbr_plus = np.roll(t_plus, 1, axis=ax)                    # -d neighbour's +d trace
            nbr_minus = np.roll(t_minus, -1, axis=ax)                 # +d neighbour's -d trace
            fstar = np.stack([lax_friedrichs(nbr_plus, t_minus, d, self.gamma),
                              lax_friedrichs(t_plus, nbr_minus, d, self.gamma)], axis=-1)
            corr = fstar - flux(tr, d, self.gamma)
            r = r + np.einsum("fi,f,...f->...i", self.E1, np.diag(self.B1), corr)
            r = r / self.weights                                       # M^{-1} per line
            out += np.moveaxis(-(2.0 / self.h[d]) * r, -1, {0: 6, 1: 5, 2: 4}[d])
        return out
