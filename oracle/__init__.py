"""Plain, slow FP64 CPU oracle for the nodal DG Euler right-hand side and its
low-storage Runge-Kutta time stepper (Kirby & Mavriplis, "GPU-Accelerated
Discontinuous Galerkin Methods", Sections II and IV).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP path.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_2006_15698_amd``)
never imports, calls or links anything here, and nothing here imports the
product path.  The two share no code; the only common module is the seeded
input generator package ``workloads``, which holds no DG arithmetic.

What the oracle computes is the plain definition of the method: the weak form
of Eq. (5) with the collocated Gauss-Legendre nodal basis of Eqs. (6)-(7),
evaluated with dense per-element operators (O(N^6) per element, no sum
factorisation), a dense over-integrated mass matrix, and the local
Lax-Friedrichs face flux.  Every function cites the passage it follows.

Parity status per function (each pin lives in ``tests/test_oracle_*.py``):
  quadrature.gauss_legendre      pinned (library GL rule, exact moments)
  quadrature.lagrange[_deriv]    pinned (polynomial exactness, partition of unity)
  euler.*                        pinned (hand-computed fixture, LF consistency
                                 and conservation, 1-D Rusanov special case)
  dg.rhs                         pinned (free stream, conservation, density-wave
                                 invariance and convergence rate, p=0 finite
                                 volume, 1-D reduction, equivariance)
  dg.integrals / max_rate        pinned (closed-form integrals)
  lserk.*                        pinned (order conditions, stability polynomial,
                                 temporal convergence rate)
  adjoint.*                      pinned (complex-step vs central differences,
                                 dot-product identity)
  viscous.NavierStokesDG         pinned (mu = 0 is Euler, free stream,
                                 conservation, gradient convergence, symmetric
                                 negative heat-conduction operator, shear-wave
                                 rate convergence, independent 1-D BR1 code)
  splitform.SplitFormDG          pinned (central two-point flux reproduces the
                                 weak form of dg.DG, hand-worked Kennedy-Gruber
                                 fixture, consistency and symmetry, free stream,
                                 conservation, density-wave convergence)
  varp.VariableDegreeDG          pinned (one degree is dg.DG, free stream and
                                 conservation across degree jumps, rate
                                 convergence with mixed degrees, axis
                                 permutation equivariance)
  hp.RefinedMeshDG               pinned (no refinement is varp, all cells
                                 refined is dg.DG on the twice finer mesh,
                                 face coverage, free stream and conservation
                                 across hanging faces, rate convergence with
                                 half the cells refined)
"""

from . import quadrature, euler, dg, lserk, viscous, splitform, varp, hp  # noqa: F401
