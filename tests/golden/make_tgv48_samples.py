"""Writes tests/golden/tgv48_p4_50steps.npz from the oracle alone.

Workload (one GPU's share at its real size): Taylor-Green vortex on
[0, 2 pi]^3, 48^3 elements, p = 4, Mach 0.1, dt from CFL 0.3 of the initial
state, 50 LSERK45 steps.  The full oracle run takes tens of minutes on the
host; stored are dt, the domain integrals of Q_0 and Q_50, the full-field
L2 norms of Q_50 and of Q_50 - Q_0 per field (nodal quadrature), and the
oracle's Q_50 on 64 seeded sampled elements (all 125 nodes, 5 fields), so
that GPU runs can report their L2 error against the oracle on those
elements.

    python tests/golden/make_tgv48_samples.py
"""

import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import lserk  # noqa: E402
from oracle.dg import DG  # noqa: E402

N_ELEM, P, STEPS, NSAMPLE, SEED = 48, 4, 50, 64, 4848


def l2(dg, X):
    w = (dg.J * dg.wq)
    x = X.reshape(5, -1, dg.N3)
    return np.sqrt(np.einsum("fet,t->f", x * x, w))


def main():
    L = (2 * math.pi,) * 3
    dg = DG((N_ELEM,) * 3, P, L=L)
    Q0 = W.tgv(N_ELEM, P)
    dt = dg.dt_cfl(Q0, 0.3)
    Q = Q0.copy()
    res = np.zeros_like(Q)
    t0 = time.time()
    for n in range(STEPS):
        lserk.step(Q, res, dt, dg.rhs)
        print(f"step {n + 1}/{STEPS} {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(SEED)
    idx = rng.choice(N_ELEM ** 3, size=NSAMPLE, replace=False)
    ez, r = np.divmod(idx, N_ELEM * N_ELEM)
    ey, ex = np.divmod(r, N_ELEM)
    samples = Q[:, ez, ey, ex]                    # [5, NSAMPLE, N, N, N]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv48_p4_50steps.npz")
    np.savez(out, dt=dt, steps=STEPS, elems=np.stack([ex, ey, ez], 1), samples=samples,
             integrals0=dg.integrals(Q0), integrals=dg.integrals(Q), l2=l2(dg, Q),
             l2_change=l2(dg, Q - Q0))
    print("wrote", out)


if __name__ == "__main__":
    main()
