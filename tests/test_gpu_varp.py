"""Variable degree per element on the GPU (dg_varp_*) against the oracle's
``VariableDegreeDG``: one degree everywhere is bitwise the single-degree
library, mixed degrees 0..7 on ragged meshes element by element, three
LSERK45 steps, conservation, the 48^3 Taylor-Green workload with
enstrophy-driven degrees 3..5 on sampled elements (3x3x3 periodic
patches), meshes one or two elements across, and the argument checks."""

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.euler import flux
from oracle.quadrature import gauss_legendre, lagrange_deriv
from oracle.varp import VariableDegreeDG
from tests.parity import TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(5, -1)


def varp_summand_scale(v, Q):
    """Per field: max over nodes of sum_d (2/h_d) |F^d_f| times the largest
    row sum of |w_a D_ai / w_i| over the degrees present (the size of the
    terms whose differences make up the rate)."""
    q = np.asarray(Q).reshape(5, -1)
    dh = 1.0
    for p in np.unique(v.deg):
        if p > 0:
            xi, w = gauss_legendre(int(p) + 1)
            D = lagrange_deriv(xi, xi)
            dh = max(dh, float(np.max(np.sum(np.abs(w[:, None] * D / w[None, :]), axis=0))))
    s = np.zeros_like(q)
    for d in range(3):
        s = s + (2.0 / v.h[d]) * np.abs(flux(q, d, v.gamma))
    return np.max(s, axis=1) * dh


def _err(v, Q, Rg, Ro):
    d = np.abs(Rg - Ro).max(axis=1)
    return d / (np.abs(Ro).max(axis=1) + varp_summand_scale(v, Q))


def _smooth(X, Y, Z):
    tp = 2 * np.pi
    return (1 + 0.2 * np.sin(tp * (X + 0.5 * Y + Z)), 0.3 + 0.1 * np.cos(tp * Y), 0 * X - 0.2 + 0.05 * np.sin(tp * Z),
            0 * X + 0.1, 1 + 0.1 * np.sin(tp * Z) * np.cos(tp * X))


@pytest.mark.parametrize("p,n", [(0, (4, 3, 5)), (1, (5, 3, 4)), (2, (4, 5, 3)), (3, (3, 4, 5)), (4, (4, 3, 3)),
                                 (5, (3, 2, 3)), (6, (2, 3, 2)), (7, (2, 2, 3))])
def test_one_degree_is_bitwise_the_single_degree_library(dgm, p, n):
    """The same arithmetic in the same order: rates and two RK steps agree
    bit for bit with dg_rhs / dg_rk_steps (the layouts coincide for one
    degree)."""
    import torch
    L = (1.0, 0.8, 1.3)
    print(f"[varp one degree p={p} n={n}]", flush=True)
    Q = W.random_smooth(n, p, seed=400 + p, L=L, noise=0.03)
    v = dgm.VariableDegree(n, np.full((n[2], n[1], n[0]), p), L=L)
    s = dgm.Solver(n, p, L=L)
    Rv = _host(v.rhs(_dev(Q)))
    Rs = _host(s.rhs(_dev(Q)))
    assert np.array_equal(Rv, Rs), np.max(np.abs(Rv - Rs))
    dt = 0.2 / ((2 * p + 1) * 8.0)
    Qa, Qb = _dev(Q), _dev(Q)
    ra, rb = torch.zeros_like(Qa), torch.zeros_like(Qb)
    v.step(Qa, ra, dt, nsteps=2)
    s.step(Qb, rb, dt, nsteps=2)
    assert torch.equal(Qa, Qb) and torch.equal(ra, rb)


@pytest.mark.parametrize("pmin,pmax,n,seed", [(0, 7, (3, 2, 3), 1), (1, 6, (4, 3, 5), 2), (2, 5, (5, 4, 3), 3),
                                              (3, 5, (6, 5, 4), 4), (0, 2, (7, 3, 2), 5), (4, 7, (2, 2, 2), 6)])
def test_mixed_degrees_vs_oracle(dgm, pmin, pmax, n, seed):
    L = (1.0, 0.8, 1.2)
    print(f"[varp mixed {pmin}..{pmax} n={n}]", flush=True)
    deg = W.random_degrees(n, pmin, pmax, 500 + seed)
    Q = W.varp_state(n, deg, _smooth, L=L)
    Q = Q * (1 + 0.01 * np.random.default_rng(seed).standard_normal(Q.shape))
    ora = VariableDegreeDG(n, deg, L=L)
    v = dgm.VariableDegree(n, deg, L=L)
    assert v.num_dof() == ora.num_dof()
    assert v.offsets == [int(x) for x in ora.off]
    Rg = _host(v.rhs(_dev(Q)))
    Ro = ora.rhs(Q)
    err = _err(ora, Q, Rg, Ro)
    print("scaled error per field", err)
    assert np.all(err <= TOL), err


def test_mixed_degree_steps_vs_oracle(dgm):
    import torch
    n, L = (4, 3, 3), (1.0, 1.1, 0.9)
    deg = W.random_degrees(n, 1, 4, 610)
    print("[varp steps]", flush=True)
    Q0 = W.varp_state(n, deg, _smooth, L=L)
    ora = VariableDegreeDG(n, deg, L=L)
    dt = ora.dt_cfl(Q0, 0.3)
    v = dgm.VariableDegree(n, deg, L=L)
    Q = _dev(Q0)
    res = torch.zeros_like(Q)
    v.step(Q, res, dt, nsteps=3)
    Qo = lserk.integrate(Q0, dt, 3, ora.rhs)
    m = np.abs(Qo).max(axis=1)
    scale = np.array([m[0], m[1:4].max(), m[1:4].max(), m[1:4].max(), m[4]])
    rate_scale = np.abs(ora.rhs(Q0)).max(axis=1) + varp_summand_scale(ora, Q0)
    # 15 stages, each adding at most TOL * dt * rate_scale and two roundings
    bar = 15 * (2 * np.finfo(float).eps * scale + TOL * dt * rate_scale)
    dq = np.abs(_host(Q) - Qo).max(axis=1)
    print("state error per field", dq, "bar", bar)
    assert np.all(dq <= bar)


def test_mixed_degree_conservation(dgm):
    """The nodal-rule integrals of the rate vanish: both sides of every
    mortar face use the same flux values and weights."""
    n, L = (5, 4, 3), (1.0, 0.8, 1.2)
    deg = W.random_degrees(n, 0, 6, 620)
    Q = W.varp_state(n, deg, _smooth, L=L)
    ora = VariableDegreeDG(n, deg, L=L)
    v = dgm.VariableDegree(n, deg, L=L)
    Rg = _host(v.rhs(_dev(Q)))
    tot = ora.integrals(Rg)
    sc = ora.integrals(np.abs(Rg))
    print("integrals of the rate", tot / sc)
    assert np.all(np.abs(tot) <= 1e-13 * sc)


def _patch(deg, off, Q, e, n):
    """3x3x3 periodic patch centred on element e: its degrees and state."""
    nx, ny, nz = n
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    pdeg = np.zeros((3, 3, 3), dtype=np.int64)
    blocks = []
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                g = ((ez + kz - 1) % nz) * nx * ny + ((ey + ky - 1) % ny) * nx + (ex + kx - 1) % nx
                pdeg[kz, ky, kx] = deg[g]
                blocks.append(Q[:, off[g]:off[g + 1]])
    return pdeg, np.ascontiguousarray(np.concatenate(blocks, axis=1))


def test_tgv48_enstrophy_degrees_sampled(dgm):
    """The benchmark workload (48^3 elements, degrees 3..5 from the initial
    enstrophy density, Taylor-Green vortex at Mach 0.1): the rate of 48
    sampled elements, each against the oracle on the 3x3x3 periodic patch
    around it (the rate of an element depends only on it and its six face
    neighbours), half of them chosen next to a degree jump."""
    n = (48, 48, 48)
    L = (2 * np.pi,) * 3
    deg3 = W.tgv_degrees(n)
    deg = deg3.reshape(-1)
    off = W.varp_offsets(deg)
    print("[varp tgv48 sampled]", flush=True)
    Q = W.varp_state(n, deg3, W.tgv_primitives, L=L)
    v = dgm.VariableDegree(n, deg3, L=L)
    Rg = _host(v.rhs(_dev(Q)))
    rng = np.random.default_rng(630)
    jump = np.zeros(deg3.shape, dtype=bool)
    for ax in range(3):
        for sh in (1, -1):
            jump |= deg3 != np.roll(deg3, sh, axis=ax)
    cand_j = np.flatnonzero(jump.reshape(-1))
    cand_c = np.flatnonzero(~jump.reshape(-1))
    elems = np.concatenate([rng.choice(cand_j, 24, replace=False), rng.choice(cand_c, 24, replace=False)])
    h = np.array(L) / np.array(n)
    worst = np.zeros(5)
    for e in elems:
        pdeg, pQ = _patch(deg, off, Q, int(e), n)
        ora = VariableDegreeDG((3, 3, 3), pdeg, L=tuple(3 * h))
        Ro = ora.element(ora.rhs(pQ), 13)
        Rge = Rg[:, off[e]:off[e + 1]]
        worst = np.maximum(worst, _err(ora, pQ, Rge, Ro))
    print("worst scaled error per field", worst)
    assert np.all(worst <= TOL), worst


def test_argument_checks(dgm):
    import torch
    with pytest.raises(dgm.DGError, match="degree 8"):
        dgm.VariableDegree((2, 2, 2), [1, 2, 3, 8, 1, 1, 1, 1])
    with pytest.raises(dgm.DGError, match="degree -1"):
        dgm.VariableDegree((2, 1, 1), [1, -1])
    v = dgm.VariableDegree((2, 2, 1), [1, 2, 3, 0])
    assert v.num_dof() == 8 + 27 + 64 + 1
    Q = v.empty()
    with pytest.raises(dgm.DGError, match="overlaps"):
        dgm.dg_varp_rhs(v.v, Q, Q)
    res = torch.zeros_like(Q)
    with pytest.raises(dgm.DGError, match="nsteps"):
        dgm.dg_varp_rk_steps(v.v, Q, res, 0.1, -1)
    with pytest.raises(dgm.DGError, match="not finite"):
        dgm.dg_varp_rk_steps(v.v, Q, res, float("nan"), 1)
    # a workspace that is too small is refused
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(dgm.DGError, match="workspace"):
        dgm.dg_varp_set_workspace(v.v, ws)


@pytest.mark.parametrize("n,deg", [((1, 1, 1), [3]), ((2, 1, 1), [1, 3]), ((1, 2, 1), [4, 0]),
                                   ((1, 1, 2), [2, 5]), ((2, 2, 1), [0, 1, 2, 3]), ((3, 1, 1), [7, 1, 4])])
def test_degenerate_meshes_vs_oracle(dgm, n, deg):
    """Meshes one or two elements across: an element is its own neighbour
    (1 x 1 x 1), or two distinct faces join the same pair of elements of
    different degrees (the + and - faces along a direction of length 2)."""
    L = (0.7, 1.1, 0.9)
    deg3 = np.array(deg).reshape(n[2], n[1], n[0])
    print(f"[varp degenerate n={n} degrees {deg}]", flush=True)
    Q = W.varp_state(n, deg3, _smooth, L=L)
    ora = VariableDegreeDG(n, deg3, L=L)
    v = dgm.VariableDegree(n, deg3, L=L)
    Rg = _host(v.rhs(_dev(Q)))
    Ro = ora.rhs(Q)
    err = _err(ora, Q, Rg, Ro)
    print("scaled error per field", err)
    assert np.all(err <= TOL), err
    tot = ora.integrals(Rg)
    assert np.all(np.abs(tot) <= 1e-13 * ora.integrals(np.abs(Rg)))
