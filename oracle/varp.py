"""Variable polynomial degree per element on the periodic Cartesian mesh, as
its plain definition.

The paper's framework adapts the degree element by element (hp-adaptation,
Sections I and III) and names it future work for the GPU code.  The reading
taken here, for the oracle and the GPU alike: the geometry stays the
conforming Cartesian mesh; every element e carries its own degree p_e
(N_e = p_e + 1 Gauss-Legendre points per direction) and the weak form of
Eq. (5) on its own collocated basis; a face between elements of degrees p
and q is integrated on a mortar: the tensor Gauss-Legendre rule of
max(p, q) + 1 points per tangential direction, at whose points both
elements' traces are evaluated (each element's polynomial evaluated there
exactly), the local Lax-Friedrichs flux is formed, and the flux times each
side's test functions is summed.  Both sides use the same flux values and
weights, so the scheme conserves; where the degrees agree the mortar rule
is the elements' own face rule and the scheme is the standard one.

State layout: Q[f, t] over the concatenated nodes of all elements, element
index e = (ez ny + ey) nx + ex ascending, node index i fastest inside an
element (Q[f, off[e] : off[e+1]] is element e's [N_e, N_e, N_e] block, k
slowest).  Evaluated densely per element with the matrices of
``oracle.dg.DG`` built for one element of each degree; the mass matrix is
over-integrated and solved densely.  TEST INFRASTRUCTURE ONLY (see
``oracle/__init__``).
"""

import numpy as np

from .dg import DG, NFIELDS, basis3d
from .euler import flux, lax_friedrichs, pressure, sound_speed
from .quadrature import gauss_legendre


class VariableDegreeDG:
    """Periodic nx*ny*nz mesh on [0,Lx]x[0,Ly]x[0,Lz]; degrees[ez, ey, ex]
    (0..7) per element."""

    def __init__(self, n, degrees, L=(1.0, 1.0, 1.0), gamma=1.4):
        self.nx, self.ny, self.nz = (int(v) for v in n)
        self.deg = np.asarray(degrees, dtype=int).reshape(self.nz, self.ny, self.nx)
        if self.deg.min() < 0:
            raise ValueError("degrees must be >= 0")
        self.L = np.asarray(L, dtype=np.float64)
        self.gamma = float(gamma)
        self.h = self.L / np.array([self.nx, self.ny, self.nz], dtype=np.float64)
        # one single-element DG per degree (element-sized domain): its basis,
        # gradient and mass matrices are those of every element of that degree
        self.ref = {int(p): DG((1, 1, 1), int(p), L=tuple(self.h), gamma=gamma) for p in np.unique(self.deg)}
        flat = self.deg.ravel()
        self.N3 = np.array([(p + 1) ** 3 for p in flat])
        self.off = np.concatenate([[0], np.cumsum(self.N3)])

    @property
    def E(self):
        return self.nx * self.ny * self.nz

    def num_dof(self):
        return int(self.off[-1])

    def element(self, Q, e):
        return np.asarray(Q)[:, self.off[e]:self.off[e + 1]]

    def index(self, ex, ey, ez):
        return (ez % self.nz) * self.nx * self.ny + (ey % self.ny) * self.nx + (ex % self.nx)

    def coords(self, e):
        ez, r = divmod(e, self.nx * self.ny)
        ey, ex = divmod(r, self.nx)
        return ex, ey, ez

    def _mortar(self, d, side, p, m):
        """Points (reference coordinates of the element of degree p on its
        face xi_d = side) of the mortar rule with m + 1 points per tangential
        direction, its weights, and the element's basis at them."""
        x, w = gauss_legendre(m + 1)
        hi, lo = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
        lo, hi = lo.ravel(), hi.ravel()
        tang = [a for a in range(3) if a != d]
        pts = np.zeros((len(lo), 3))
        pts[:, d] = float(side)
        pts[:, tang[0]] = x[lo]
        pts[:, tang[1]] = x[hi]
        return w[lo] * w[hi], basis3d(self.ref[p].nodes, pts)

    def rhs(self, Q):
        """dQ/dt of Eq. (5) per element with mortar faces, in the layout of Q."""
        Q = np.asarray(Q)
        if Q.shape != (NFIELDS, self.num_dof()):
            raise ValueError(f"Q has shape {Q.shape}, expected {(NFIELDS, self.num_dof())}")
        dt = np.result_type(Q.dtype, np.float64)
        V = np.zeros(Q.shape, dtype=dt)
        S = np.zeros(Q.shape, dtype=dt)
        for e in range(self.E):
            ex, ey, ez = self.coords(e)
            p = int(self.deg[ez, ey, ex])
            ref = self.ref[p]
            q = self.element(Q, e)                                    # [5, N3]
            qq = q @ ref.Phi.T                                        # at the quadrature points
            sl = slice(self.off[e], self.off[e + 1])
            for d in range(3):
                V[:, sl] += (flux(qq, d, self.gamma) * (ref.J * ref.wq)) @ ref.Grad[d]
                # the +d face of e, shared with its +d neighbour
                nb = self.index(ex + (d == 0), ey + (d == 1), ez + (d == 2))
                nex, ney, nez = self.coords(nb)
                pn = int(self.deg[nez, ney, nex])
                m = max(p, pn)
                wf, Bm_own = self._mortar(d, 1, p, m)
                _, Bm_nbr = self._mortar(d, -1, pn, m)
                qm = q @ Bm_own.T                                     # e's trace at the mortar points
                qp = self.element(Q, nb) @ Bm_nbr.T                   # the neighbour's trace there
                fstar = lax_friedrichs(qm, qp, d, self.gamma) * (ref.Jf[d] * wf)
                S[:, sl] += fstar @ Bm_own                            # n = +e_d for e
                snb = slice(self.off[nb], self.off[nb + 1])
                S[:, snb] -= fstar @ Bm_nbr                           # n = -e_d for the neighbour
        out = np.zeros(Q.shape, dtype=dt)
        for e in range(self.E):
            ex, ey, ez = self.coords(e)
            ref = self.ref[int(self.deg[ez, ey, ex])]
            sl = slice(self.off[e], self.off[e + 1])
            out[:, sl] = np.linalg.solve(ref.M, (V[:, sl] - S[:, sl]).T).T
        return out

    def integrals(self, Q):
        """Integrals of the five conserved fields by each element's nodal rule."""
        out = np.zeros(NFIELDS)
        for e in range(self.E):
            ex, ey, ez = self.coords(e)
            ref = self.ref[int(self.deg[ez, ey, ex])]
            out += self.element(Q, e) @ (ref.J * ref.wq)
        return out

    def max_rate(self, Q):
        """max over nodes of sum_d (|u_d| + c) / h_d."""
        q = np.asarray(Q)
        c = sound_speed(q, self.gamma)
        return float(np.max(sum((np.abs(q[1 + d] / q[0]) + c) / self.h[d] for d in range(3))))

    def dt_cfl(self, Q, cfl):
        """dt = CFL / ((2 p_max + 1) max_rate) (a reading, as for DG.dt_cfl)."""
        return cfl / ((2 * int(self.deg.max()) + 1) * self.max_rate(Q))

    def check_state(self, Q):
        q = np.asarray(Q)
        return bool(np.all(np.isfinite(q)) and np.all(q[0] > 0) and np.all(pressure(q, self.gamma) > 0))


def pack(blocks):
    """Concatenate per-element states [5, N, N, N] (element order) into the
    [5, total] layout."""
    return np.ascontiguousarray(np.concatenate([b.reshape(NFIELDS, -1) for b in blocks], axis=1))
