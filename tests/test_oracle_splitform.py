"""Pins of the kinetic-energy-preserving split-form oracle,
``oracle/splitform.py``.

What fixes it, independently of the oracle's own code:
  - with the central two-point flux (F(Q_L) + F(Q_R))/2 the hybridised
    flux-differencing operator is algebraically the weak form of Eq. (5), so
    it must reproduce ``oracle.dg.DG`` (itself pinned by free stream,
    conservation, convergence, finite-volume and 1-D reductions) to rounding:
    this pins the operator, the face coupling, the interface correction and
    the metric scaling;
  - the Kennedy-Gruber flux against values worked by hand from its
    definition (tests/golden/kg_flux_pointwise.json), its consistency
    f_S(Q, Q) = F(Q) and its symmetry;
  - any symmetric consistent two-point flux in this form keeps a uniform
    state uniform and conserves mass, momentum and energy on a periodic mesh;
  - the density wave converges to its closed form.
"""

import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.dg import DG
from oracle.euler import flux
from oracle.splitform import SplitFormDG, central_flux, kg_flux

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kg_flux_pointwise.json")


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_central_two_point_flux_is_the_weak_form(p):
    n, L = (3, 4, 2), (1.0, 0.8, 1.3)
    Q = W.random_smooth(n, p, seed=40 + p, L=L, noise=0.05)
    a = SplitFormDG(n, p, L=L, two_point=central_flux).rhs(Q)
    b = DG(n, p, L=L).rhs(Q)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_kg_flux_hand_worked_values():
    g = json.load(open(GOLD))
    qa = np.array(g["state_a"]["conserved"])
    qb = np.array(g["state_b"]["conserved"])
    for d, key in enumerate(("x", "y", "z")):
        got = kg_flux(qa, qb, d, g["gamma"])
        assert np.allclose(got, g["flux"][key]["values"], rtol=0, atol=1e-14), (key, got)


def test_kg_flux_consistent_and_symmetric():
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 2.0, 50)
    u = rng.uniform(-1, 1, (3, 50))
    pres = rng.uniform(0.5, 3.0, 50)
    qa = W.conserved(rho, u[0], u[1], u[2], pres)
    qb = W.conserved(rho[::-1], u[2], u[0], -u[1], pres[::-1])
    for d in range(3):
        assert np.allclose(kg_flux(qa, qa, d, 1.4), flux(qa, d, 1.4), rtol=1e-14, atol=1e-14)
        assert np.array_equal(kg_flux(qa, qb, d, 1.4), kg_flux(qb, qa, d, 1.4))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_split_form_free_stream(p):
    n, L = (3, 2, 2), (1.0, 0.7, 1.1)
    Q = W.uniform_state(n, p, 1.3, (0.4, -0.2, 0.7), 2.1)
    R = SplitFormDG(n, p, L=L).rhs(Q)
    assert np.max(np.abs(R)) <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_split_form_conserves(p):
    n, L = (3, 4, 2), (1.0, 0.9, 1.2)
    Q = W.random_smooth(n, p, seed=60 + p, L=L, noise=0.05)
    ora = SplitFormDG(n, p, L=L)
    R = ora.rhs(Q).reshape(5, -1, ora.N3)
    w = ora.J * ora.wq
    total = np.einsum("fet,t->f", R, w)
    scale = np.einsum("fet,t->f", np.abs(R), w)
    assert np.all(np.abs(total) <= 1e-13 * scale)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_split_form_density_wave_converges(p):
    """rho = 1 + 0.2 sin(2 pi (x + y)), u = v = 1, w = 0, p = 1 advected to
    t = 0.02: the max-norm density error falls at the finest refinement at
    least like h^(p + 0.5) (measured 1.94, 2.62, 4.16 at p = 1, 2, 3)."""
    errs = []
    for m in (4, 8, 16):
        n = (m, m, 1)
        T = 0.02
        Q0 = W.density_wave(n, p, k=(1, 1, 0))
        ora = SplitFormDG(n, p)
        steps = int(math.ceil(T / ora.dt_cfl(Q0, 0.25)))
        Q = lserk.integrate(Q0, T / steps, steps, ora.rhs)
        X, Y, Z = W.node_coords(n, p, (1.0, 1.0, 1.0))
        errs.append(np.max(np.abs(Q[0] - W.density_wave_exact(X, Y, Z, T, k=(1, 1, 0)))))
    rate = math.log(errs[-2] / errs[-1], 2)
    assert rate >= p + 0.5, (errs, rate)
