"""Viscous (Navier-Stokes, BR1) terms on the GPU against the oracle's
``NavierStokesDG``: the right-hand side element by element for p = 0..7 on
ragged anisotropic meshes, LSERK45 steps, the Taylor-Green vortex at
Re = 1600 on the 48^3 p=4 mesh on sampled elements (5x5x5 periodic patches),
the inviscid rate formed in the viscous-flux launch against its own launch,
conservation over steps, and the calls that the viscous terms do not cover."""

import ctypes
import math

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.viscous import NavierStokesDG
from tests.parity import TOL, patch_rhs_viscous, summand_scale, visc_summand_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _scaled_error(ns, Q, Rg, Ro):
    d = np.abs(Rg - Ro).reshape(5, -1).max(axis=1)
    ref = np.abs(Ro).reshape(5, -1).max(axis=1)
    return d / (ref + summand_scale(ns, Q) + visc_summand_scale(ns, Q))


@pytest.mark.parametrize("p,n", [(0, (4, 3, 5)), (1, (5, 3, 4)), (2, (4, 5, 3)), (3, (3, 4, 5)), (4, (4, 3, 3)),
                                 (5, (3, 2, 3)), (6, (2, 3, 2)), (7, (2, 2, 3))])
def test_viscous_rhs_vs_oracle(dgm, p, n):
    L = (1.0, 0.8, 1.3)
    mu, pr = 0.02, 0.72
    print(f"[visc rhs p={p} n={n}]", flush=True)
    Q = W.random_smooth(n, p, seed=200 + p, L=L, noise=0.03)
    ns = NavierStokesDG(n, p, L=L, mu=mu, prandtl=pr)
    s = dgm.Solver(n, p, L=L, mu=mu, prandtl=pr)
    Rg = _host(s.rhs(_dev(Q)))
    Ro = ns.rhs(Q)
    err = _scaled_error(ns, Q, Rg, Ro)
    print("scaled error per field", err)
    assert np.all(err <= TOL), err
    # the viscous part is not negligible in these states
    Rv = ns.rhs_viscous(Q)
    assert np.max(np.abs(Rv[1:])) >= 1e-3 * np.max(np.abs(Ro[1:]))


@pytest.mark.parametrize("p", [1, 3, 4])
def test_viscous_steps_vs_oracle(dgm, p):
    n, L = (4, 3, 3), (1.0, 1.1, 0.9)
    mu, pr = 0.05, 0.7
    print(f"[visc steps p={p}]", flush=True)
    Q0 = W.random_smooth(n, p, seed=210 + p, L=L, noise=0.02)
    ns = NavierStokesDG(n, p, L=L, mu=mu, prandtl=pr)
    dt = ns.dt_cfl(Q0, 0.3)
    s = dgm.Solver(n, p, L=L, mu=mu, prandtl=pr)
    Q = _dev(Q0)
    import torch
    res = torch.zeros_like(Q)
    s.step(Q, res, dt, nsteps=3)
    Qo = lserk.integrate(Q0, dt, 3, ns.rhs)
    Qg = _host(Q)
    m = np.abs(Qo).reshape(5, -1).max(axis=1)
    scale = np.array([m[0], m[1:4].max(), m[1:4].max(), m[1:4].max(), m[4]])
    dq = np.abs(Qg - Qo).reshape(5, -1).max(axis=1)
    # per stage: the rounding of the update (2 ulp of the state) plus dt
    # times a rate difference of 1e-12 of the rate's summand scale; 15 stages
    R0 = ns.rhs(Q0)
    rate_scale = np.abs(R0).reshape(5, -1).max(axis=1) + summand_scale(ns, Q0) + visc_summand_scale(ns, Q0)
    bar = 15 * (2 * np.finfo(float).eps * scale + TOL * dt * rate_scale)
    print("state error / bar", dq / bar)
    assert np.all(dq <= bar)
    # graph replay falls back to direct launches and gives the same bits
    Qb = _dev(Q0)
    rb = torch.zeros_like(Qb)
    s.step(Qb, rb, dt, nsteps=3, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(Qb, Q)


@pytest.mark.parametrize("p,n", [(0, (3, 2, 4)), (1, (4, 3, 2)), (2, (3, 4, 2)), (3, (3, 4, 5)), (4, (4, 3, 3)),
                                 (5, (3, 2, 3)), (6, (2, 3, 2)), (7, (2, 2, 3))])
def test_fused_inviscid_rate_equals_its_own_launch(dgm, p, n):
    """The inviscid rate formed inside the viscous-flux launch against the
    neighbour-read kernel's launch of its own: the same bits, for the
    right-hand side and over steps."""
    import torch
    L = (1.0, 1.2, 0.8)
    print(f"[visc fused p={p} n={n}]", flush=True)
    Q0 = W.random_smooth(n, p, seed=260 + p, L=L, noise=0.03)
    fused = dgm.Solver(n, p, L=L, mu=0.03, prandtl=0.7)
    split = dgm.Solver(n, p, L=L, mu=0.03, prandtl=0.7)
    split.set_option(dgm.DG_OPT_VISC_FUSED, 0)
    assert fused.options()["visc_fused"] == 1 and split.options()["visc_fused"] == 0
    Q = _dev(Q0)
    assert torch.equal(fused.rhs(Q), split.rhs(Q))
    Qa, Qb = _dev(Q0), _dev(Q0)
    ra, rb = torch.zeros_like(Qa), torch.zeros_like(Qb)
    fused.step(Qa, ra, 1e-4, nsteps=2)
    split.step(Qb, rb, 1e-4, nsteps=2)
    torch.cuda.synchronize()
    assert torch.equal(Qa, Qb) and torch.equal(ra, rb)


def test_viscous_conservation_over_steps(dgm):
    import torch
    n, p, L = (5, 4, 3), 3, (1.0, 1.0, 1.0)
    Q0 = W.random_smooth(n, p, seed=230, L=L, noise=0.02)
    s = dgm.Solver(n, p, L=L, mu=0.05)
    Q = _dev(Q0)
    res = torch.zeros_like(Q)
    I0 = s.integrals(Q)
    s.step(Q, res, 2e-4, nsteps=10)
    I1 = s.integrals(Q)
    scale = np.array([abs(I0[0])] * 4 + [abs(I0[4])])
    assert np.all(np.abs(I1[:5] - I0[:5]) <= 1e-13 * scale + 1e-13 * abs(I0[0]))


def test_tgv_re1600_48cubed_sampled_elements(dgm):
    """The viscous Taylor-Green vortex (Mach 0.1, Re = 1600: mu = 1/1600,
    Pr = 0.71) on the 48^3 p=4 mesh: the GPU right-hand side at sampled
    elements against the oracle on 5x5x5 periodic patches."""
    n, p, L = (48, 48, 48), 4, (2 * math.pi,) * 3
    mu, pr = 1.0 / 1600.0, 0.71
    print("[visc tgv 48^3 p=4 Re 1600, sampled]", flush=True)
    Q = W.tgv(48, 4)
    s = dgm.Solver(n, p, L=L, mu=mu, prandtl=pr)
    Rg = _host(s.rhs(_dev(Q)))
    rng = np.random.default_rng(1600)
    elems = [tuple(int(v) for v in rng.integers(0, 48, size=3)) for _ in range(5)] + [(0, 0, 0), (47, 47, 47)]
    ref = patch_rhs_viscous(n, p, L, Q, elems, mu, pr)
    ns_small = NavierStokesDG((5, 5, 5), p, L=tuple(5 * np.array(L) / 48), mu=mu, prandtl=pr)
    for (ex, ey, ez), Ro in ref.items():
        xs = [(ex + o) % 48 for o in range(-2, 3)]
        ys = [(ey + o) % 48 for o in range(-2, 3)]
        zs = [(ez + o) % 48 for o in range(-2, 3)]
        patch = np.ascontiguousarray(Q[:, zs][:, :, ys][:, :, :, xs])
        got = Rg[:, ez, ey, ex]
        d = np.abs(got - Ro).reshape(5, -1).max(axis=1)
        S = summand_scale(ns_small, patch) + visc_summand_scale(ns_small, patch)
        err = d / (np.abs(Ro).reshape(5, -1).max(axis=1) + S)
        assert np.all(err <= TOL), ((ex, ey, ez), err)


def test_fp32_form_with_viscosity(dgm):
    """The FP32 form's inviscid contractions with FP64 viscous terms: the
    right-hand side stays within a stated bound of the FP64 form's."""
    n, p, L = (4, 3, 5), 3, (1.0, 0.8, 1.3)
    Q = _dev(W.random_smooth(n, p, seed=240, L=L, noise=0.02))
    R64 = _host(dgm.Solver(n, p, L=L, mu=0.02).rhs(Q))
    R32 = _host(dgm.Solver(n, p, L=L, mu=0.02, precision=dgm.DG_FP32_MFMA).rhs(Q))
    rel = np.abs(R32 - R64).reshape(5, -1).max(axis=1) / np.abs(R64).reshape(5, -1).max(axis=1)
    print("fp32 form vs fp64, viscous rhs, relative per field", rel)
    assert np.all(rel <= 1e-4)


def test_viscosity_settings_and_unsupported_calls(dgm):
    import torch
    n, p = (3, 3, 2), 2
    Q0 = W.random_smooth(n, p, seed=250, noise=0.02)
    plain = dgm.Solver(n, p)
    zero = dgm.Solver(n, p, mu=0.0)
    Q = _dev(Q0)
    assert torch.equal(plain.rhs(Q), zero.rhs(Q))
    visc = dgm.Solver(n, p, mu=0.1)
    with pytest.raises(dgm.DGError):
        visc.rhs_vjp(Q, torch.ones_like(Q))
    lib = dgm._lib
    res = torch.zeros_like(Q)
    assert lib.dg_rk_steps_noalloc(visc.ctx, Q.data_ptr(), res.data_ptr(), ctypes.c_double(1e-3), 1) == \
        dgm.DG_EUNSUPPORTED
    for bad in [(-1.0, 0.7), (0.1, 0.0), (float("nan"), 0.7)]:
        with pytest.raises(dgm.DGError):
            dgm.dg_set_viscosity(visc.ctx, *bad)
    # switching the viscosity off again gives the Euler rate
    visc.set_viscosity(0.0)
    assert torch.equal(visc.rhs(Q), plain.rhs(Q))
