"""Cells refined once (2 x 2 x 2 children) on the periodic Cartesian mesh,
with a degree per element, as its plain definition: the hp setting of the
paper's adaptive framework (Sections I and III name it).

Mesh: an nx x ny x nz periodic base mesh of cells of size h = L / n; a cell
is either one element (level 0) or, when refined, eight elements of size
h / 2 (level 1).  Elements are numbered cell by cell, c = (cz ny + cy) nx + cx
ascending; a refined cell's children in the order (kz, ky, kx), kx fastest.
Every element carries its own degree and the scheme of Eq. (5) on its own
collocated basis and size.

Faces: every (sub-)face between two elements is integrated on a mortar: the
tensor Gauss-Legendre rule of max(p_a, p_b) + 1 points per tangential
direction on the smaller of the two faces (a whole face where both are the
same size; a fine element's face, a quarter of the coarse face, where a
refined cell meets an unrefined one).  At those points (physical positions
on the face) both elements' polynomials are evaluated exactly, the local
Lax-Friedrichs flux is formed once, and the flux times each side's test
functions is integrated with the sub-face's own area element.  Both sides use
the same flux values and weights, so the scheme conserves; without
refinement it is ``oracle.varp.VariableDegreeDG``, and with every cell
refined the conforming mesh of 2n cells.

State layout: Q[f, t] over the concatenated nodes of all elements in element
order (Q[f, off[e] : off[e+1]] is element e's [N_e]^3 block, i fastest).
Evaluated densely per element and per face.  TEST INFRASTRUCTURE ONLY (see
``oracle/__init__``).
"""

import numpy as np

from .dg import DG, NFIELDS, basis3d
from .euler import flux, lax_friedrichs, pressure, sound_speed
from .quadrature import gauss_legendre


class RefinedMeshDG:
    """refine[cz, cy, cx] in {0, 1}; degrees: one per element in element
    order (0..7)."""

    def __init__(self, n, refine, degrees, L=(1.0, 1.0, 1.0), gamma=1.4):
        self.nx, self.ny, self.nz = (int(v) for v in n)
        self.refine = np.asarray(refine, dtype=int).reshape(self.nz, self.ny, self.nx)
        self.L = np.asarray(L, dtype=np.float64)
        self.gamma = float(gamma)
        self.hc = self.L / np.array([self.nx, self.ny, self.nz], dtype=np.float64)
        # elements: (cell index, level, child (kx, ky, kz), origin, size)
        self.cell, self.level, self.child, self.x0, self.size = [], [], [], [], []
        self.first = np.zeros(self.nx * self.ny * self.nz + 1, dtype=int)   # first element of each cell
        for c in range(self.nx * self.ny * self.nz):
            cz, r = divmod(c, self.nx * self.ny)
            cy, cx = divmod(r, self.nx)
            self.first[c] = len(self.cell)
            base = np.array([cx, cy, cz]) * self.hc
            if self.refine[cz, cy, cx]:
                for kz in range(2):
                    for ky in range(2):
                        for kx in range(2):
                            k = np.array([kx, ky, kz])
                            self._add(c, 1, k, base + k * self.hc / 2, self.hc / 2)
            else:
                self._add(c, 0, np.zeros(3, dtype=int), base, self.hc)
        self.first[-1] = len(self.cell)
        self.deg = np.asarray(degrees, dtype=int).reshape(-1)
        if self.deg.size != self.E:
            raise ValueError(f"{self.deg.size} degrees for {self.E} elements")
        if self.deg.min() < 0:
            raise ValueError("degrees must be >= 0")
        self.N3 = (self.deg + 1) ** 3
        self.off = np.concatenate([[0], np.cumsum(self.N3)])
        self._ref = {}
        self.faces = self._faces()

    def _add(self, c, lev, k, x0, h):
        self.cell.append(c)
        self.level.append(lev)
        self.child.append(k)
        self.x0.append(np.asarray(x0, dtype=np.float64))
        self.size.append(np.asarray(h, dtype=np.float64))

    @property
    def E(self):
        return len(self.cell)

    def num_dof(self):
        return int(self.off[-1])

    def element(self, Q, e):
        return np.asarray(Q)[:, self.off[e]:self.off[e + 1]]

    def ref(self, e):
        """One-element DG of element e's degree and size: its basis, gradient,
        mass matrix and nodal weights."""
        key = (int(self.deg[e]), self.level[e])
        if key not in self._ref:
            self._ref[key] = DG((1, 1, 1), key[0], L=tuple(self.size[e]), gamma=self.gamma)
        return self._ref[key]

    def _cell_of(self, cx, cy, cz):
        return ((cz % self.nz) * self.ny + (cy % self.ny)) * self.nx + (cx % self.nx)

    def _faces(self):
        """Every (sub-)face once, as (a, b, d): element a on its +d face, b on
        its -d face (b is a's +d neighbour)."""
        out = []
        for e in range(self.E):
            c = self.cell[e]
            cz, r = divmod(c, self.nx * self.ny)
            cy, cx = divmod(r, self.nx)
            for d in range(3):
                k = self.child[e]
                if self.level[e] == 1 and k[d] == 0:
                    kk = k.copy()
                    kk[d] = 1
                    out.append((e, self.first[c] + (kk[2] * 2 + kk[1]) * 2 + kk[0], d))
                    continue
                step = [0, 0, 0]
                step[d] = 1
                cn = self._cell_of(cx + step[0], cy + step[1], cz + step[2])
                if not self.refine.reshape(-1)[cn]:
                    out.append((e, self.first[cn], d))
                elif self.level[e] == 1:
                    kk = k.copy()
                    kk[d] = 0
                    out.append((e, self.first[cn] + (kk[2] * 2 + kk[1]) * 2 + kk[0], d))
                else:
                    for k2 in range(2):
                        for k1 in range(2):
                            kk = [0, 0, 0]
                            t = [a for a in range(3) if a != d]
                            kk[t[0]], kk[t[1]] = k1, k2
                            out.append((e, self.first[cn] + (kk[2] * 2 + kk[1]) * 2 + kk[0], d))
        return out

    def _face_rule(self, a, b, d):
        """Mortar points of face (a, b, d) as reference coordinates of a and
        of b, the weights times the (sub-)face's area element."""
        m = max(int(self.deg[a]), int(self.deg[b])) + 1
        x, w = gauss_legendre(m)
        t = [q for q in range(3) if q != d]
        small = a if self.size[a][t[0]] <= self.size[b][t[0]] else b
        hi, lo = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        lo, hi = lo.ravel(), hi.ravel()
        # physical tangential positions on the smaller face
        pos = np.zeros((len(lo), 3))
        for j, (ax, idx) in enumerate(((t[0], lo), (t[1], hi))):
            pos[:, ax] = self.x0[small][ax] + (x[idx] + 1.0) * self.size[small][ax] / 2.0
        area = self.size[small][t[0]] * self.size[small][t[1]] / 4.0
        ra = np.zeros_like(pos)
        rb = np.zeros_like(pos)
        ra[:, d], rb[:, d] = 1.0, -1.0
        for ax in t:
            ra[:, ax] = 2.0 * (pos[:, ax] - self.x0[a][ax]) / self.size[a][ax] - 1.0
            rb[:, ax] = 2.0 * (pos[:, ax] - self.x0[b][ax]) / self.size[b][ax] - 1.0
        return ra, rb, w[lo] * w[hi] * area

    def rhs(self, Q):
        """dQ/dt of Eq. (5) per element with mortar (sub-)faces."""
        Q = np.asarray(Q)
        if Q.shape != (NFIELDS, self.num_dof()):
            raise ValueError(f"Q has shape {Q.shape}, expected {(NFIELDS, self.num_dof())}")
        dt = np.result_type(Q.dtype, np.float64)
        V = np.zeros(Q.shape, dtype=dt)
        S = np.zeros(Q.shape, dtype=dt)
        for e in range(self.E):
            ref = self.ref(e)
            q = self.element(Q, e)
            qq = q @ ref.Phi.T
            sl = slice(self.off[e], self.off[e + 1])
            for d in range(3):
                V[:, sl] += (flux(qq, d, self.gamma) * (ref.J * ref.wq)) @ ref.Grad[d]
        for a, b, d in self.faces:
            ra, rb, wf = self._face_rule(a, b, d)
            Ba = basis3d(self.ref(a).nodes, ra)
            Bb = basis3d(self.ref(b).nodes, rb)
            qm = self.element(Q, a) @ Ba.T
            qp = self.element(Q, b) @ Bb.T
            fstar = lax_friedrichs(qm, qp, d, self.gamma) * wf
            S[:, self.off[a]:self.off[a + 1]] += fstar @ Ba
            S[:, self.off[b]:self.off[b + 1]] -= fstar @ Bb
        out = np.zeros(Q.shape, dtype=dt)
        for e in range(self.E):
            sl = slice(self.off[e], self.off[e + 1])
            out[:, sl] = np.linalg.solve(self.ref(e).M, (V[:, sl] - S[:, sl]).T).T
        return out

    def coords(self, e):
        """Node coordinates (X, Y, Z) of element e, each [N, N, N] (k, j, i)."""
        xi = self.ref(e).nodes
        K, J, I = np.meshgrid(xi, xi, xi, indexing="ij")
        x0, h = self.x0[e], self.size[e]
        return (x0[0] + (I + 1.0) * h[0] / 2.0, x0[1] + (J + 1.0) * h[1] / 2.0, x0[2] + (K + 1.0) * h[2] / 2.0)

    def integrals(self, Q):
        """Integrals of the five conserved fields by each element's nodal rule."""
        out = np.zeros(NFIELDS)
        for e in range(self.E):
            ref = self.ref(e)
            out += self.element(Q, e) @ (ref.J * ref.wq)
        return out

    def max_rate(self, Q):
        """max over elements and nodes of sum_d (|u_d| + c) / h_d."""
        best = 0.0
        for e in range(self.E):
            q = self.element(Q, e)
            c = sound_speed(q, self.gamma)
            r = sum((np.abs(q[1 + d] / q[0]) + c) / self.size[e][d] for d in range(3))
            best = max(best, float(np.max(r)))
        return best

    def dt_cfl(self, Q, cfl):
        """dt = CFL / ((2 p_max + 1) max_rate) (a reading, as for DG.dt_cfl)."""
        return cfl / ((2 * int(self.deg.max()) + 1) * self.max_rate(Q))

    def check_state(self, Q):
        q = np.asarray(Q)
        return bool(np.all(np.isfinite(q)) and np.all(q[0] > 0) and np.all(pressure(q, self.gamma) > 0))
