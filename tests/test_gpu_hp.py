"""Refined cells with a degree per element on the GPU (dg_varp_create_refined)
against the oracle's ``RefinedMeshDG``: without refinement it is bitwise the
variable-degree library, with every cell refined and one degree bitwise the
single-degree library on the twice finer mesh; random refinements with
mixed degrees 0..7 element by element, three LSERK45 steps, conservation
across hanging faces, meshes one to three cells across, the Taylor-Green
hp workload (40^3 cells, enstrophy-driven refinement and degrees 3..5) on
sampled cells, the face traces written by the stage kernels against those
formed from the state (bitwise), and the argument checks."""

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.euler import flux
from oracle.hp import RefinedMeshDG
from oracle.quadrature import gauss_legendre, lagrange_deriv
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


def _dh(p):
    if p == 0:
        return 1.0
    xi, w = gauss_legendre(p + 1)
    D = lagrange_deriv(xi, xi)
    return max(1.0, float(np.max(np.sum(np.abs(w[:, None] * D / w[None, :]), axis=0))))


def hp_summand_scale(ora, Q, elems=None):
    """Per field: max over elements and nodes of sum_d (2/h_d) |F^d_f| with
    the element's own size, times the row-sum bound of its degree's
    differentiation (the size of the terms whose differences make up the
    rate)."""
    out = np.zeros(5)
    for e in (range(ora.E) if elems is None else elems):
        q = ora.element(Q, e)
        s = sum((2.0 / ora.size[e][d]) * np.abs(flux(q, d, ora.gamma)) for d in range(3))
        out = np.maximum(out, np.max(s, axis=1) * _dh(int(ora.deg[e])))
    return out


def _err(ora, Q, Rg, Ro, elems=None):
    return np.abs(Rg - Ro).max(axis=1) / (np.abs(Ro).max(axis=1) + hp_summand_scale(ora, Q, elems))


def _smooth(X, Y, Z):
    tp = 2 * np.pi
    return (1 + 0.2 * np.sin(tp * (X + 0.5 * Y + Z)), 0.3 + 0.1 * np.cos(tp * Y), 0 * X - 0.2 + 0.05 * np.sin(tp * Z),
            0 * X + 0.1, 1 + 0.1 * np.sin(tp * Z) * np.cos(tp * X))


def _n_elem(refine):
    return int(np.sum(1 + 7 * np.asarray(refine)))


def test_no_refinement_is_bitwise_the_variable_degree_library(dgm):
    import torch
    n, L = (4, 3, 5), (1.0, 0.8, 1.2)
    deg = W.random_degrees(n, 0, 7, 700)
    print("[hp no refinement]", flush=True)
    Q = W.varp_state(n, deg, _smooth, L=L)
    a = dgm.VariableDegree(n, deg, L=L)
    b = dgm.VariableDegree(n, deg.reshape(-1), L=L, refine=np.zeros((n[2], n[1], n[0]), dtype=int))
    assert b.E == a.E and b.offsets == a.offsets
    assert np.array_equal(_host(a.rhs(_dev(Q))), _host(b.rhs(_dev(Q))))
    dt = 0.2 / (15 * 8.0)
    Qa, Qb = _dev(Q), _dev(Q)
    ra, rb = torch.zeros_like(Qa), torch.zeros_like(Qb)
    a.step(Qa, ra, dt, nsteps=2)
    b.step(Qb, rb, dt, nsteps=2)
    assert torch.equal(Qa, Qb) and torch.equal(ra, rb)


@pytest.mark.parametrize("p,n", [(0, (3, 2, 3)), (1, (2, 3, 2)), (2, (3, 2, 2)), (3, (2, 2, 3)), (4, (2, 3, 1)),
                                 (5, (2, 1, 2)), (6, (1, 2, 2)), (7, (2, 1, 1))])
def test_all_refined_is_bitwise_the_twice_finer_mesh(dgm, p, n):
    """Every cell refined, one degree: the elements are those of the 2n mesh
    and every face conforming, so the rate and two RK steps agree bit for
    bit with the single-degree library on that mesh, element by element."""
    import torch
    L = (1.0, 0.8, 1.3)
    print(f"[hp all refined p={p} n={n}]", flush=True)
    r1 = np.ones((n[2], n[1], n[0]), dtype=int)
    E = _n_elem(r1)
    n2 = (2 * n[0], 2 * n[1], 2 * n[2])
    Qs = W.random_smooth(n2, p, seed=710 + p, L=L, noise=0.03)   # [5, ez, ey, ex, N^3] on the 2n mesh
    Qs = np.asarray(Qs).reshape(5, n2[2], n2[1], n2[0], -1)
    # element order of the refined mesh: cell by cell, children (kz, ky, kx)
    where = []
    for cz in range(n[2]):
        for cy in range(n[1]):
            for cx in range(n[0]):
                for kz in range(2):
                    for ky in range(2):
                        for kx in range(2):
                            where.append((2 * cz + kz, 2 * cy + ky, 2 * cx + kx))
    assert len(where) == E
    Qh = np.concatenate([Qs[:, z, y, x] for z, y, x in where], axis=1)
    v = dgm.VariableDegree(n, np.full(E, p), L=L, refine=r1)
    s = dgm.Solver(n2, p, L=L)

    def to_hp(R):
        R = np.asarray(R).reshape(5, n2[2], n2[1], n2[0], -1)
        return np.concatenate([R[:, z, y, x] for z, y, x in where], axis=1)

    Rv = _host(v.rhs(_dev(Qh)))
    Rs = to_hp(_host(s.rhs(_dev(Qs))))
    assert np.array_equal(Rv, Rs), np.max(np.abs(Rv - Rs))
    dt = 0.1 / ((2 * p + 1) * 8.0)
    Qa, Qb = _dev(Qh), _dev(Qs)
    ra, rb = torch.zeros_like(Qa), torch.zeros_like(Qb)
    v.step(Qa, ra, dt, nsteps=2)
    s.step(Qb, rb, dt, nsteps=2)
    assert np.array_equal(_host(Qa), to_hp(_host(Qb)))
    assert np.array_equal(_host(ra), to_hp(_host(rb)))


CASES = [(0, 7, (3, 2, 3), 0.5, 1), (1, 5, (4, 3, 3), 0.3, 2), (2, 4, (3, 4, 2), 0.7, 3), (3, 3, (4, 4, 3), 0.5, 4),
         (0, 2, (5, 3, 2), 0.4, 5), (4, 7, (2, 2, 2), 0.5, 6), (1, 1, (5, 4, 3), 0.25, 7)]


@pytest.mark.parametrize("pmin,pmax,n,frac,seed", CASES)
def test_random_refinement_vs_oracle(dgm, pmin, pmax, n, frac, seed):
    """Random cells refined, random degree per element: hanging faces
    between every pair of degrees in the range, sibling faces and
    fine-fine faces across cells, element by element within the bar."""
    L = (1.0, 0.8, 1.2)
    ref = W.random_refinement(n, frac, 720 + seed)
    deg = np.random.default_rng(730 + seed).integers(pmin, pmax + 1, _n_elem(ref))
    print(f"[hp random n={n} degrees {pmin}..{pmax} refined {int(ref.sum())}]", flush=True)
    Q = W.hp_state(n, ref, deg, _smooth, L=L)
    Q = Q * (1 + 0.01 * np.random.default_rng(seed).standard_normal(Q.shape))
    ora = RefinedMeshDG(n, ref, deg, L=L)
    v = dgm.VariableDegree(n, deg, L=L, refine=ref)
    assert v.E == ora.E and v.num_dof() == ora.num_dof()
    assert v.offsets == [int(x) for x in ora.off]
    Rg = _host(v.rhs(_dev(Q)))
    Ro = ora.rhs(Q)
    err = _err(ora, Q, Rg, Ro)
    print("scaled error per field", err)
    assert np.all(err <= TOL), err


def test_refined_steps_vs_oracle(dgm):
    import torch
    n, L = (4, 3, 3), (1.0, 1.1, 0.9)
    ref = W.random_refinement(n, 0.4, 740)
    deg = np.random.default_rng(741).integers(1, 5, _n_elem(ref))
    print("[hp steps]", flush=True)
    Q0 = W.hp_state(n, ref, deg, _smooth, L=L)
    ora = RefinedMeshDG(n, ref, deg, L=L)
    dt = ora.dt_cfl(Q0, 0.3)
    v = dgm.VariableDegree(n, deg, L=L, refine=ref)
    Q = _dev(Q0)
    res = torch.zeros_like(Q)
    v.step(Q, res, dt, nsteps=3)
    Qo = lserk.integrate(Q0, dt, 3, ora.rhs)
    m = np.abs(Qo).max(axis=1)
    scale = np.array([m[0], m[1:4].max(), m[1:4].max(), m[1:4].max(), m[4]])
    rate_scale = np.abs(ora.rhs(Q0)).max(axis=1) + hp_summand_scale(ora, Q0)
    # 15 stages, each adding at most TOL * dt * rate_scale and two roundings
    bar = 15 * (2 * np.finfo(float).eps * scale + TOL * dt * rate_scale)
    dq = np.abs(_host(Q) - Qo).max(axis=1)
    print("state error per field", dq, "bar", bar)
    assert np.all(dq <= bar)


def test_conservation_across_hanging_faces(dgm):
    """The nodal-rule integrals of the rate vanish: both sides of every
    hanging sub-face use the same flux values and weights."""
    n, L = (5, 4, 3), (1.0, 0.8, 1.2)
    ref = W.random_refinement(n, 0.4, 750)
    deg = np.random.default_rng(751).integers(0, 7, _n_elem(ref))
    Q = W.hp_state(n, ref, deg, _smooth, L=L)
    ora = RefinedMeshDG(n, ref, deg, L=L)
    v = dgm.VariableDegree(n, deg, L=L, refine=ref)
    Rg = _host(v.rhs(_dev(Q)))
    tot = ora.integrals(Rg)
    sc = ora.integrals(np.abs(Rg))
    print("integrals of the rate", tot / sc)
    assert np.all(np.abs(tot) <= 1e-13 * sc)


@pytest.mark.parametrize("n,ref", [((1, 1, 1), [1]), ((2, 1, 1), [1, 0]), ((1, 2, 1), [0, 1]), ((1, 1, 2), [1, 1]),
                                   ((2, 2, 1), [1, 0, 0, 1]), ((3, 1, 1), [1, 0, 1])])
def test_degenerate_meshes_vs_oracle(dgm, n, ref):
    """Meshes one to three cells across: a refined cell whose children meet
    each other across the periodic boundary, a coarse cell whose two faces
    along a direction both hang on the same refined cell."""
    L = (0.7, 1.1, 0.9)
    ref3 = np.array(ref).reshape(n[2], n[1], n[0])
    deg = np.random.default_rng(760 + sum(n)).integers(0, 6, _n_elem(ref3))
    print(f"[hp degenerate n={n} refine {ref}]", flush=True)
    Q = W.hp_state(n, ref3, deg, _smooth, L=L)
    ora = RefinedMeshDG(n, ref3, deg, L=L)
    v = dgm.VariableDegree(n, deg, L=L, refine=ref3)
    Rg = _host(v.rhs(_dev(Q)))
    Ro = ora.rhs(Q)
    err = _err(ora, Q, Rg, Ro)
    print("scaled error per field", err)
    assert np.all(err <= TOL), err
    tot = ora.integrals(Rg)
    assert np.all(np.abs(tot) <= 1e-13 * ora.integrals(np.abs(Rg)))


def _cell_patch(ref, deg, cfirst, off, Q, c, n):
    """3x3x3 periodic patch of cells centred on cell c: its refinement,
    its elements' degrees and state (patch element order)."""
    nx, ny, nz = n
    cx, cy, cz = c % nx, (c // nx) % ny, c // (nx * ny)
    pref = np.zeros((3, 3, 3), dtype=np.int64)
    pdeg, blocks = [], []
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                g = ((cz + kz - 1) % nz) * nx * ny + ((cy + ky - 1) % ny) * nx + (cx + kx - 1) % nx
                pref[kz, ky, kx] = ref[g]
                for e in range(cfirst[g], cfirst[g + 1]):
                    pdeg.append(deg[e])
                    blocks.append(Q[:, off[e]:off[e + 1]])
    return pref, np.array(pdeg), np.ascontiguousarray(np.concatenate(blocks, axis=1))


def test_tgv40_hp_sampled(dgm):
    """The benchmark workload (40^3 cells, those of enstrophy indicator
    >= 0.7 refined, degrees 3..5 from the indicator, Taylor-Green vortex at
    Mach 0.1): the rate of the elements of 40 sampled cells, each against
    the oracle on the 3x3x3 periodic patch of cells around it (an element's
    rate depends only on it and its face neighbours), 16 of them next to a
    refinement jump, 8 inside refined regions, 16 elsewhere."""
    n = (40, 40, 40)
    L = (2 * np.pi,) * 3
    ref3, deg = W.tgv_refined_mesh(n)
    ref = ref3.reshape(-1)
    cfirst = np.concatenate([[0], np.cumsum(np.where(ref == 1, 8, 1))])
    off = W.varp_offsets(deg)
    print("[hp tgv40 sampled]", flush=True)
    Q = W.hp_state(n, ref3, deg, W.tgv_primitives, L=L)
    v = dgm.VariableDegree(n, deg, L=L, refine=ref3)
    Rg = _host(v.rhs(_dev(Q)))
    rng = np.random.default_rng(770)
    jump = np.zeros(ref3.shape, dtype=bool)
    for ax in range(3):
        for sh in (1, -1):
            jump |= ref3 != np.roll(ref3, sh, axis=ax)
    jump = jump.reshape(-1)
    cells = np.concatenate([rng.choice(np.flatnonzero(jump), 16, replace=False),
                            rng.choice(np.flatnonzero(~jump & (ref == 1)), 8, replace=False),
                            rng.choice(np.flatnonzero(~jump & (ref == 0)), 16, replace=False)])
    h = np.array(L) / np.array(n)
    worst = np.zeros(5)
    for c in cells:
        pref, pdeg, pQ = _cell_patch(ref, deg, cfirst, off, Q, int(c), n)
        ora = RefinedMeshDG((3, 3, 3), pref, pdeg, L=tuple(3 * h))
        Ro = ora.rhs(pQ)
        mine = range(ora.first[13], ora.first[14])
        for k, e in zip(mine, range(cfirst[c], cfirst[c + 1])):
            worst = np.maximum(worst, _err(ora, pQ, Rg[:, off[e]:off[e + 1]], ora.element(Ro, k), [k]))
    print("worst scaled error per field", worst)
    assert np.all(worst <= TOL), worst


def test_timing_names_the_hanging_kernel(dgm):
    n = (3, 2, 2)
    ref = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0]).reshape(2, 2, 3)
    deg = np.random.default_rng(780).integers(1, 4, _n_elem(ref))
    v = dgm.VariableDegree(n, deg, refine=ref)
    Q = _dev(W.hp_state(n, ref, deg, _smooth))
    v.set_timing(True)
    v.rhs(Q)
    t = v.timing_read()
    assert t["hanging"][1] == 1
    assert all(k == "hanging" or k == "mortar" or k[1] == 0 for k in t)


def test_argument_checks_refined(dgm):
    with pytest.raises(dgm.DGError, match="refinement 2"):
        dgm.VariableDegree((2, 1, 1), [1] * 9, refine=[2, 0])
    with pytest.raises(ValueError, match="degrees for 9 elements"):
        dgm.VariableDegree((2, 1, 1), [1, 1], refine=[1, 0])
    with pytest.raises(dgm.DGError, match="degree 8"):
        dgm.VariableDegree((2, 1, 1), [1] * 8 + [8], refine=[1, 0])
    v = dgm.VariableDegree((2, 1, 1), [0] * 8 + [2], refine=[1, 0])
    assert v.E == 9 and v.num_dof() == 8 + 27


@pytest.mark.parametrize("refined,pmin,pmax", [(False, 1, 5), (True, 1, 5), (False, 0, 7), (True, 0, 7)])
def test_stage_traces_equal_traces_from_the_state(dgm, refined, pmin, pmax):
    """Within one call the face kernels read the traces that the previous
    stage's kernels wrote; the first stage of a call forms them from the
    state.  Three steps in one call and three calls of one step therefore
    take the two routes at the starts of steps 2 and 3, and must agree bit
    for bit (state and residual)."""
    import torch
    n, L = (4, 3, 3), (1.0, 0.9, 1.1)
    ref = W.random_refinement(n, 0.4, 790) if refined else np.zeros((n[2], n[1], n[0]), dtype=np.int64)
    deg = np.random.default_rng(791 + pmax).integers(pmin, pmax + 1, _n_elem(ref))
    print(f"[hp traces refined={refined} degrees {pmin}..{pmax}]", flush=True)
    Q0 = W.hp_state(n, ref, deg, _smooth, L=L)
    v = dgm.VariableDegree(n, deg, L=L, refine=ref)
    dt = RefinedMeshDG(n, ref, deg, L=L).dt_cfl(Q0, 0.3)
    Qa, Qb = _dev(Q0), _dev(Q0)
    ra, rb = torch.zeros_like(Qa), torch.zeros_like(Qb)
    v.step(Qa, ra, dt, nsteps=3)
    for _ in range(3):
        v.step(Qb, rb, dt, nsteps=1)
    assert torch.equal(Qa, Qb) and torch.equal(ra, rb)
