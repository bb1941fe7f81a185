"""The kinetic-energy-preserving split form (DG_VOLUME_KEP) on the GPU
against the oracle's ``SplitFormDG``: the right-hand side element by element
for p = 0..7 on ragged anisotropic meshes, three LSERK45 steps, with the
viscous terms, the 48^3 p=4 Taylor-Green vortex on sampled elements (3x3x3
periodic patches), conservation, and the settings it does not combine with."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.splitform import SplitFormDG
from oracle.viscous import NavierStokesDG
from tests.parity import TOL, patch_rhs, split_summand_scale, visc_summand_scale

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


def _err(ora, Q, Rg, Ro, extra=0.0):
    d = np.abs(Rg - Ro).reshape(5, -1).max(axis=1)
    return d / (np.abs(Ro).reshape(5, -1).max(axis=1) + split_summand_scale(ora, Q) + extra)


@pytest.mark.parametrize("p,n", [(0, (4, 3, 5)), (1, (5, 3, 4)), (2, (4, 5, 3)), (3, (3, 4, 5)), (4, (4, 3, 3)),
                                 (5, (3, 2, 3)), (6, (2, 3, 2)), (7, (2, 2, 3))])
def test_split_rhs_vs_oracle(dgm, p, n):
    L = (1.0, 0.8, 1.3)
    print(f"[split rhs p={p} n={n}]", flush=True)
    Q = W.random_smooth(n, p, seed=300 + p, L=L, noise=0.03)
    ora = SplitFormDG(n, p, L=L)
    s = dgm.Solver(n, p, L=L, volume_form=dgm.DG_VOLUME_KEP)
    Rg = _host(s.rhs(_dev(Q)))
    Ro = ora.rhs(Q)
    err = _err(ora, Q, Rg, Ro)
    print("scaled error per field", err)
    assert np.all(err <= TOL), err
    # it is not the standard form
    std = _host(dgm.Solver(n, p, L=L).rhs(_dev(Q)))
    if p > 0:
        assert np.max(np.abs(std - Rg)) > 1e3 * np.max(np.abs(Rg - Ro))


@pytest.mark.parametrize("p", [1, 3, 4])
def test_split_steps_vs_oracle(dgm, p):
    import torch
    n, L = (4, 3, 3), (1.0, 1.1, 0.9)
    print(f"[split steps p={p}]", flush=True)
    Q0 = W.random_smooth(n, p, seed=310 + p, L=L, noise=0.02)
    ora = SplitFormDG(n, p, L=L)
    dt = ora.dt_cfl(Q0, 0.3)
    s = dgm.Solver(n, p, L=L, volume_form=dgm.DG_VOLUME_KEP)
    Q = _dev(Q0)
    res = torch.zeros_like(Q)
    s.step(Q, res, dt, nsteps=3)
    Qo = lserk.integrate(Q0, dt, 3, ora.rhs)
    m = np.abs(Qo).reshape(5, -1).max(axis=1)
    scale = np.array([m[0], m[1:4].max(), m[1:4].max(), m[1:4].max(), m[4]])
    R0 = ora.rhs(Q0)
    rate_scale = np.abs(R0).reshape(5, -1).max(axis=1) + split_summand_scale(ora, Q0)
    bar = 15 * (2 * np.finfo(float).eps * scale + TOL * dt * rate_scale)
    dq = np.abs(_host(Q) - Qo).reshape(5, -1).max(axis=1)
    print("state error / bar", dq / bar)
    assert np.all(dq <= bar)
    Qb = _dev(Q0)
    rb = torch.zeros_like(Qb)
    s.step(Qb, rb, dt, nsteps=3, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(Qb, Q)


def test_split_with_viscosity_vs_oracle(dgm):
    n, p, L = (4, 3, 3), 3, (1.0, 0.8, 1.3)
    mu, pr = 0.02, 0.72
    Q = W.random_smooth(n, p, seed=320, L=L, noise=0.02)
    sp = SplitFormDG(n, p, L=L)
    ns = NavierStokesDG(n, p, L=L, mu=mu, prandtl=pr)
    Ro = sp.rhs(Q) + ns.rhs_viscous(Q)
    s = dgm.Solver(n, p, L=L, mu=mu, prandtl=pr, volume_form=dgm.DG_VOLUME_KEP)
    Rg = _host(s.rhs(_dev(Q)))
    err = _err(sp, Q, Rg, Ro, visc_summand_scale(ns, Q))
    assert np.all(err <= TOL), err


def test_split_conservation_over_steps(dgm):
    import torch
    n, p, L = (5, 4, 3), 3, (1.0, 1.0, 1.0)
    Q0 = W.random_smooth(n, p, seed=330, L=L, noise=0.02)
    s = dgm.Solver(n, p, L=L, volume_form=dgm.DG_VOLUME_KEP)
    Q = _dev(Q0)
    res = torch.zeros_like(Q)
    I0 = s.integrals(Q)
    s.step(Q, res, 2e-4, nsteps=10)
    I1 = s.integrals(Q)
    scale = np.array([abs(I0[0])] * 4 + [abs(I0[4])])
    assert np.all(np.abs(I1[:5] - I0[:5]) <= 1e-13 * scale + 1e-13 * abs(I0[0]))


def test_split_tgv48_p4_sampled_elements(dgm):
    n, p, L = (48, 48, 48), 4, (2 * math.pi,) * 3
    print("[split tgv 48^3 p=4, sampled]", flush=True)
    Q = W.tgv(48, 4)
    s = dgm.Solver(n, p, L=L, volume_form=dgm.DG_VOLUME_KEP)
    Rg = _host(s.rhs(_dev(Q)))
    rng = np.random.default_rng(4848)
    elems = [tuple(int(v) for v in rng.integers(0, 48, size=3)) for _ in range(8)] + [(0, 0, 0), (47, 47, 47)]
    ref = patch_rhs(n, p, L, Q, elems, make=SplitFormDG)
    small = SplitFormDG((3, 3, 3), p, L=tuple(3 * np.array(L) / 48))
    for (ex, ey, ez), Ro in ref.items():
        patch = np.ascontiguousarray(Q[:, [(ez + o) % 48 for o in (-1, 0, 1)]][:, :, [(ey + o) % 48 for o in (-1, 0, 1)]]
                                     [:, :, :, [(ex + o) % 48 for o in (-1, 0, 1)]])
        err = _err(small, patch, Rg[:, ez, ey, ex], Ro)
        assert np.all(err <= TOL), ((ex, ey, ez), err)


def test_split_settings(dgm):
    import torch
    n, p = (3, 3, 2), 2
    Q = _dev(W.random_smooth(n, p, seed=340, noise=0.02))
    s = dgm.Solver(n, p, volume_form=dgm.DG_VOLUME_KEP)
    with pytest.raises(dgm.DGError):
        dgm.dg_set_precision(s.ctx, dgm.DG_FP32_MFMA)
    with pytest.raises(dgm.DGError):
        s.rhs_vjp(Q, torch.ones_like(Q))
    with pytest.raises(dgm.DGError):
        dgm.dg_set_volume_form(s.ctx, 7)
    f32 = dgm.Solver(n, p, precision=dgm.DG_FP32_MFMA)
    with pytest.raises(dgm.DGError):
        dgm.dg_set_volume_form(f32.ctx, dgm.DG_VOLUME_KEP)
    # back to the standard form: the standard rate
    dgm.dg_set_volume_form(s.ctx, dgm.DG_VOLUME_STANDARD)
    assert torch.equal(s.rhs(Q), dgm.Solver(n, p).rhs(Q))
