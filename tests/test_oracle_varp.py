"""Pins of the variable-degree oracle, ``oracle/varp.py``.

What fixes it, independently of the oracle's own code:
  - with one degree everywhere the mortar rule is every element's own face
    rule, so it must reproduce ``oracle.dg.DG`` (pinned on its own);
  - a uniform state stays uniform across degree jumps (each element's
    polynomial is evaluated exactly at the mortar points, the mortar rule
    integrates the face terms of a constant exactly);
  - both sides of a face use the same flux values and weights, so mass,
    momentum and energy are conserved;
  - on smooth data with random degrees p or p + 1 per element the rate of
    the advected density wave converges to its exact value like h^p;
  - permuting the axes of the mesh, of the degree field and of the momentum
    permutes the rate (the mortar code treats every direction alike).
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle.varp import VariableDegreeDG


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_one_degree_is_the_standard_scheme(p):
    n, L = (3, 2, 4), (1.0, 0.8, 1.2)
    Q = W.random_smooth(n, p, seed=70 + p, L=L, noise=0.05)
    R = VariableDegreeDG(n, np.full((4, 2, 3), p), L=L).rhs(np.ascontiguousarray(Q.reshape(5, -1)))
    Rd = DG(n, p, L=L).rhs(Q).reshape(5, -1)
    assert np.max(np.abs(R - Rd)) <= 1e-13 * np.max(np.abs(Rd))


def _smooth(X, Y, Z):
    tp = 2 * np.pi
    return (1 + 0.2 * np.sin(tp * (X + Y + Z)), 0.3 + 0.1 * np.cos(tp * Y), 0 * X - 0.2, 0 * X + 0.1,
            1 + 0.1 * np.sin(tp * Z))


def test_uniform_state_across_degree_jumps():
    n, L = (3, 2, 4), (1.0, 0.8, 1.2)
    deg = W.random_degrees(n, 0, 5, 7)
    v = VariableDegreeDG(n, deg, L=L)
    Q = W.varp_state(n, deg, lambda X, Y, Z: (0 * X + 1.3, 0 * X + 0.4, 0 * X - 0.2, 0 * X + 0.7, 0 * X + 2.1), L=L)
    assert np.max(np.abs(v.rhs(Q))) <= 1e-12 * 3.0 / v.h.min() * 10


def test_conservation_across_degree_jumps():
    n, L = (3, 2, 4), (1.0, 0.8, 1.2)
    deg = W.random_degrees(n, 1, 5, 8)
    v = VariableDegreeDG(n, deg, L=L)
    R = v.rhs(W.varp_state(n, deg, _smooth, L=L))
    tot, sc = np.zeros(5), np.zeros(5)
    for e in range(v.E):
        ex, ey, ez = v.coords(e)
        ref = v.ref[int(v.deg[ez, ey, ex])]
        blk = v.element(R, e)
        tot += blk @ (ref.J * ref.wq)
        sc += np.abs(blk) @ (ref.J * ref.wq)
    assert np.all(np.abs(tot) <= 1e-13 * sc)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rate_converges_with_mixed_degrees(p):
    """rho = 1 + 0.2 sin(2 pi (x + y)), u = v = 1, p = 1: d rho/dt =
    -(rho_x + rho_y) exactly; the max-norm error of the rate with degrees
    p or p + 1 per element (seeded) falls like h^p (measured mean rates of
    the last two refinements 0.97, 1.95, 2.96 at p = 1, 2, 3)."""
    errs = []
    for m in (4, 8, 16, 32):
        n = (m, m, 1)
        deg = W.random_degrees(n, p, p + 1, 100 + m)
        Q0 = W.varp_state(n, deg, lambda X, Y, Z: (1 + 0.2 * np.sin(2 * np.pi * (X + Y)), 0 * X + 1.0,
                                                   0 * X + 1.0, 0 * X, 0 * X + 1.0))
        R = VariableDegreeDG(n, deg).rhs(Q0)
        exact = W.varp_state(n, deg, lambda X, Y, Z: (-0.8 * np.pi * np.cos(2 * np.pi * (X + Y)), 0 * X, 0 * X,
                                                      0 * X, 0 * X))[0]
        errs.append(np.max(np.abs(R[0] - exact)))
    rates = [math.log(errs[i] / errs[i + 1], 2) for i in range(3)]
    assert 0.5 * (rates[1] + rates[2]) >= p - 0.25, (errs, rates)


def test_axis_permutation_equivariance():
    """Swap x and z: the mesh sizes, the degree field, the lengths and the
    momentum components swap, and the rate swaps with them."""
    n, L = (3, 2, 4), (1.0, 0.8, 1.2)
    deg = W.random_degrees(n, 1, 4, 9)
    v = VariableDegreeDG(n, deg, L=L)
    Q = W.varp_state(n, deg, _smooth, L=L)
    R = v.rhs(Q)
    nt, Lt = (n[2], n[1], n[0]), (L[2], L[1], L[0])
    degt = np.transpose(deg, (2, 1, 0))
    vt = VariableDegreeDG(nt, degt, L=Lt)
    # element (ex, ey, ez) of the original is element (ez, ey, ex) of the swap;
    # its node (i, j, k) is node (k, j, i) there; rho u <-> rho w
    Qt = np.zeros_like(Q)
    for e in range(v.E):
        ex, ey, ez = v.coords(e)
        N = int(deg[ez, ey, ex]) + 1
        blk = v.element(Q, e).reshape(5, N, N, N)
        et = vt.index(ez, ey, ex)
        Qt[:, vt.off[et]:vt.off[et + 1]] = np.transpose(blk, (0, 3, 2, 1))[[0, 3, 2, 1, 4]].reshape(5, -1)
    Rt = vt.rhs(Qt)
    for e in range(v.E):
        ex, ey, ez = v.coords(e)
        N = int(deg[ez, ey, ex]) + 1
        et = vt.index(ez, ey, ex)
        back = np.transpose(Rt[:, vt.off[et]:vt.off[et + 1]].reshape(5, N, N, N), (0, 3, 2, 1))[[0, 3, 2, 1, 4]]
        assert np.max(np.abs(back.reshape(5, -1) - v.element(R, e))) <= 1e-12 * np.max(np.abs(R))
