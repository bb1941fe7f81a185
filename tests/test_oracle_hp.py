"""Pins of the refined-mesh (hp) oracle, ``oracle/hp.py``.

What fixes it, independently of the oracle's own code:
  - without refinement it is the variable-degree scheme (``oracle.varp``,
    pinned on its own);
  - with every cell refined it is the standard scheme on the conforming mesh
    of twice as many cells per direction (``oracle.dg.DG``), element by
    element after renumbering;
  - every element face is covered exactly once by the faces the oracle
    integrates (the two elements of each face touch, and the overlaps of
    their face rectangles add up to each element face's area);
  - a uniform state stays uniform across hanging faces and degree jumps;
  - both sides of every (sub-)face use the same flux values and weights, so
    mass, momentum and energy are conserved;
  - on smooth data with half of the cells refined the rate of the advected
    density wave converges to its exact value like h^p.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle.hp import RefinedMeshDG
from oracle.varp import VariableDegreeDG


def _smooth(X, Y, Z):
    tp = 2 * np.pi
    return (1 + 0.2 * np.sin(tp * (X + 0.5 * Y + Z)), 0.3 + 0.1 * np.cos(tp * Y), 0 * X - 0.2 + 0.05 * np.sin(tp * Z),
            0 * X + 0.1, 1 + 0.1 * np.sin(tp * Z) * np.cos(tp * X))


def _n_elem(refine):
    return int(np.sum(1 + 7 * np.asarray(refine)))


def test_no_refinement_is_the_variable_degree_scheme():
    n, L = (3, 2, 2), (1.0, 0.8, 1.2)
    deg = W.random_degrees(n, 0, 5, 31)
    r0 = np.zeros((n[2], n[1], n[0]), dtype=int)
    Q = W.hp_state(n, r0, deg.reshape(-1), _smooth, L=L)
    R = RefinedMeshDG(n, r0, deg.reshape(-1), L=L).rhs(Q)
    Rv = VariableDegreeDG(n, deg, L=L).rhs(Q)
    assert np.max(np.abs(R - Rv)) <= 1e-13 * np.max(np.abs(Rv))


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_all_refined_is_the_twice_finer_mesh(p):
    n, L = (3, 2, 2), (1.0, 0.8, 1.2)
    r1 = np.ones((n[2], n[1], n[0]), dtype=int)
    hp = RefinedMeshDG(n, r1, np.full(_n_elem(r1), p), L=L)
    Q = W.hp_state(n, r1, np.full(hp.E, p), _smooth, L=L)
    R = hp.rhs(Q)
    dg = DG((2 * n[0], 2 * n[1], 2 * n[2]), p, L=L)
    Qd = np.zeros(dg.shape)
    where = []
    for e in range(hp.E):
        cz, r = divmod(hp.cell[e], n[0] * n[1])
        cy, cx = divmod(r, n[0])
        k = hp.child[e]
        ex, ey, ez = 2 * cx + k[0], 2 * cy + k[1], 2 * cz + k[2]
        Qd[:, ez, ey, ex] = hp.element(Q, e).reshape(5, p + 1, p + 1, p + 1)
        where.append((ex, ey, ez))
    Rd = dg.rhs(Qd)
    err = max(np.max(np.abs(hp.element(R, e) - Rd[:, ez, ey, ex].reshape(5, -1))) for e, (ex, ey, ez) in
              enumerate(where))
    assert err <= 1e-13 * np.max(np.abs(Rd))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_every_element_face_is_covered_once(seed):
    n, L = (3, 4, 2), (1.0, 0.8, 1.2)
    ref = W.random_refinement(n, 0.5, seed)
    hp = RefinedMeshDG(n, ref, np.ones(_n_elem(ref), dtype=int), L=L)
    area = {}
    for a, b, d in hp.faces:
        t = [q for q in range(3) if q != d]
        # the overlap of the two face rectangles, from the elements' extents
        s = 1.0
        for ax in t:
            lo = max(hp.x0[a][ax], hp.x0[b][ax])
            hi = min(hp.x0[a][ax] + hp.size[a][ax], hp.x0[b][ax] + hp.size[b][ax])
            assert hi > lo
            s *= hi - lo
        # the faces touch: a's +d face is b's -d face (periodically)
        gap = (hp.x0[a][d] + hp.size[a][d] - hp.x0[b][d]) % hp.L[d]
        assert min(gap, hp.L[d] - gap) <= 1e-12
        for e, side in ((a, 1), (b, 0)):
            area[(e, 2 * d + side)] = area.get((e, 2 * d + side), 0.0) + s
    for e in range(hp.E):
        for d in range(3):
            t = [q for q in range(3) if q != d]
            full = hp.size[e][t[0]] * hp.size[e][t[1]]
            for side in (0, 1):
                assert abs(area[(e, 2 * d + side)] - full) <= 1e-14 * full


def test_uniform_state_across_hanging_faces():
    n, L = (3, 2, 2), (1.0, 0.8, 1.2)
    ref = W.random_refinement(n, 0.5, 4)
    deg = np.random.default_rng(5).integers(0, 5, _n_elem(ref))
    hp = RefinedMeshDG(n, ref, deg, L=L)
    Q = W.hp_state(n, ref, deg, lambda X, Y, Z: (0 * X + 1.3, 0 * X + 0.4, 0 * X - 0.2, 0 * X + 0.7, 0 * X + 2.1),
                   L=L)
    # rates are of order (speed + sound speed) / h_fine times the state: 1e-12 of that
    assert np.max(np.abs(hp.rhs(Q))) <= 1e-12 * 3.0 / (hp.hc.min() / 2) * 10


def test_conservation_across_hanging_faces():
    n, L = (3, 2, 2), (1.0, 0.8, 1.2)
    ref = W.random_refinement(n, 0.5, 6)
    deg = np.random.default_rng(7).integers(1, 5, _n_elem(ref))
    hp = RefinedMeshDG(n, ref, deg, L=L)
    R = hp.rhs(W.hp_state(n, ref, deg, _smooth, L=L))
    tot, sc = hp.integrals(R), hp.integrals(np.abs(R))
    assert np.all(np.abs(tot) <= 1e-13 * sc)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rate_converges_with_half_the_cells_refined(p):
    """rho = 1 + 0.2 sin(2 pi (x + y)), u = v = 1, pressure 1 on [0,1]^2 x
    [0, 1/4] meshes of m x m x 1 cells with the cells of x < 1/2 refined:
    d rho/dt = -(rho_x + rho_y) exactly; the max-norm error of the rate falls
    like h^p (measured mean rates of the two refinements 0.98, 1.93, 2.89 at
    p = 1, 2, 3)."""
    errs = []
    for m in (4, 8, 16):
        n, L = (m, m, 1), (1.0, 1.0, 0.25)
        ref = np.zeros((1, m, m), dtype=int)
        ref[:, :, : m // 2] = 1
        deg = np.full(_n_elem(ref), p)
        Q0 = W.hp_state(n, ref, deg, lambda X, Y, Z: (1 + 0.2 * np.sin(2 * np.pi * (X + Y)), 0 * X + 1.0,
                                                     0 * X + 1.0, 0 * X, 0 * X + 1.0), L=L)
        R = RefinedMeshDG(n, ref, deg, L=L).rhs(Q0)
        exact = W.hp_state(n, ref, deg, lambda X, Y, Z: (-0.8 * np.pi * np.cos(2 * np.pi * (X + Y)), 0 * X, 0 * X,
                                                         0 * X, 0 * X), L=L)[0]
        errs.append(np.max(np.abs(R[0] - exact)))
    rates = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert 0.5 * (rates[0] + rates[1]) >= p - 0.25, (errs, rates)
