"""Writes tests/golden/adjoint_c5.json from the oracle alone.

Workload (adjoint configuration): Taylor-Green vortex on [0, 2 pi]^3,
16^3 elements, p = 3, Mach 0.1, seeded smooth perturbations of amplitude
1e-2 on every primitive (workloads.perturbed_tgv, seed 1).  dt from CFL 0.3
of the initial state; objective KE = integrated kinetic energy after 40
LSERK45 steps.  Stored: dt, KE(Q_40), integrals of Q_40, and the exact
directional derivatives dKE/dQ0 . U_k (complex step through the whole
trajectory, oracle.adjoint) for the seeded Gaussian directions
U_k = workloads.gaussian_directions(Q0, ., seed0=1000)[k].

    python tests/golden/make_adjoint_c5.py [ndirections]
"""

import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import adjoint, lserk  # noqa: E402
from oracle.dg import DG  # noqa: E402

N_ELEM, P, STEPS, SEED, SEED0 = 16, 3, 40, 1, 1000


def main():
    ndir = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    L = (2 * math.pi,) * 3
    dg = DG((N_ELEM,) * 3, P, L=L)
    Q0 = W.perturbed_tgv(N_ELEM, P, seed=SEED, amp=1e-2, L=L)
    dt = dg.dt_cfl(Q0, 0.3)
    Qf = lserk.integrate(Q0, dt, STEPS, dg.rhs)
    ints = dg.integrals(Qf)
    dirs = W.gaussian_directions(Q0, ndir, seed0=SEED0)
    derivs = []
    for k, U in enumerate(dirs):
        t0 = time.time()
        derivs.append(adjoint.ke_directional_derivative(dg, Q0, U, dt, STEPS))
        print(f"direction {k}: {derivs[-1]:.17e} ({time.time() - t0:.0f} s)", flush=True)
    rec = {
        "citation": "Objective and workload of the adjoint configuration; derivatives by the oracle's "
                    "complex step through 40 LSERK45 steps (Sections II-B, IV-V).",
        "script": "tests/golden/make_adjoint_c5.py",
        "n": N_ELEM, "p": P, "steps": STEPS, "seed": SEED, "amp": 1e-2, "mach": 0.1,
        "dt": dt, "ke_final": float(ints[5]), "integrals_final": [float(v) for v in ints],
        "direction_seed0": SEED0,
        "directional_derivatives": derivs,
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_c5.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
