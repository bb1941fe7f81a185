"""FP32 matrix-core form (contractions on FP32 deviations, FP64 anchors,
LF, lift and RK) against the FP64 oracle and the FP64 GPU path.  The paper
has no FP32 data, so these bars are our own statement of the FP32
error (summand-scaled, as for FP64), not a parity claim."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.dg import DG
from tests.parity import rhs_errors, summand_scale

pytestmark = pytest.mark.gpu

TOL32 = 2e-6   # summand-scaled bar for the FP32 contractions


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


@pytest.mark.parametrize("p", range(1, 8))
def test_fp32_rhs_all_degrees(dgm, p):
    n, L = (3, 2, 5), (1.0, 1.3, 0.7)
    print(f"[fp32 rhs p={p}]", flush=True)
    Q = W.random_smooth(n, p, seed=80 + p, L=L, noise=0.05)
    ora = DG(n, p, L=L)
    Ro = ora.rhs(Q)
    s = dgm.Solver(n, p, L=L, precision=dgm.DG_FP32_MFMA)
    Rg = _host(s.rhs(_dev(Q)))
    plain, scaled = rhs_errors(ora, Q, Rg, Ro)
    print("fp32 plain", plain, "scaled", scaled)
    assert np.all(scaled <= TOL32)


def test_fp32_p0_unsupported(dgm):
    s = dgm.dg_create(2, 2, 2, 0, 1.4)
    try:
        with pytest.raises(dgm.DGError):
            dgm.dg_set_precision(s, dgm.DG_FP32_MFMA)
    finally:
        dgm.dg_destroy(s)


def test_fp32_tgv_low_mach(dgm):
    """Low Mach (p0 = 71): the anchor removes the constant pressure from the
    FP32 contractions, so the error stays at the scale of the variation."""
    L = (2 * math.pi,) * 3
    n, p = (8, 8, 8), 4
    Q = W.tgv(8, 4)
    ora = DG(n, p, L=L)
    Ro = ora.rhs(Q)
    s = dgm.Solver(n, p, L=L, precision=dgm.DG_FP32_MFMA)
    Rg = _host(s.rhs(_dev(Q)))
    d = np.abs(Rg - Ro).reshape(5, -1).max(axis=1)
    ref = np.abs(Ro).reshape(5, -1).max(axis=1)
    S = summand_scale(ora, Q)
    print("fp32 tgv: error / summand scale", d / S, "error / |R|", d / ref)
    # FP32 rounding acts on the flux deviations; the energy flux (E + p) u
    # has no large constant part, so its error is ~1e-7 of the summand scale
    assert np.all(d <= TOL32 * S)


def test_fp32_density_wave_c1_trajectory(dgm):
    """First workload, 20 steps: FP32 form against the oracle's FP64 run."""
    import torch
    n, p = 4, 1
    Q0 = W.density_wave(n, p)
    ora = DG((n, n, n), p)
    dt = ora.dt_cfl(Q0, 0.3)
    s = dgm.Solver((n, n, n), p, precision=dgm.DG_FP32_MFMA)
    Qg = _dev(Q0)
    rg = torch.zeros_like(Qg)
    s.step(Qg, rg, dt, nsteps=20)
    Qo = lserk.integrate(Q0, dt, 20, ora.rhs)
    err = np.linalg.norm((_host(Qg) - Qo).ravel()) / np.linalg.norm(Qo.ravel())
    chg = np.linalg.norm((_host(Qg) - Qo).ravel()) / np.linalg.norm((Qo - Q0).ravel())
    print(f"fp32 c1 L2 rel err {err:.3e}, relative to the change {chg:.3e}")
    assert err <= 1e-7 and chg <= 1e-5


def test_fp32_conservation(dgm):
    """Both sides of a face rebuild the trace from the same FP32 deviation and
    FP64 anchor, so the face flux cancels exactly; the volume term's FP32
    table rounding acts only on flux deviations."""
    import torch
    L = (2 * math.pi,) * 3
    n, p = (6, 6, 6), 3
    s = dgm.Solver(n, p, L=L, precision=dgm.DG_FP32_MFMA)
    Q = W.tgv(6, 3)
    R = s.rhs(_dev(Q))
    ints = s.integrals(R)
    vol = (2 * math.pi) ** 3
    S = summand_scale(DG(n, p, L=L), Q)
    for f in range(5):
        assert abs(ints[f]) <= 1e-9 * vol * S[f], (f, ints[f])
    Qd = _dev(Q)
    r = torch.zeros_like(Qd)
    I0 = s.integrals(Qd)
    s.step(Qd, r, 0.3 * s.dt_cfl(Qd, 1.0), nsteps=10)
    I1 = s.integrals(Qd)
    # The face fluxes cancel exactly; the FP32 column sums of the volume
    # contraction vanish only to FP32 rounding of the flux deviations, so
    # mass and energy drift at ~1e-11 over these steps (FP64 form: 1e-15).
    print("fp32 drift", (I1[0] - I0[0]) / I0[0], (I1[4] - I0[4]) / I0[4])
    assert abs(I1[0] - I0[0]) <= 1e-9 * I0[0]
    assert abs(I1[4] - I0[4]) <= 1e-9 * I0[4]


def test_fp32_steps_bitwise_equal_repeated_step(dgm):
    import torch
    n, p = (5, 3, 4), 4
    s = dgm.Solver(n, p, precision=dgm.DG_FP32_MFMA)
    Q0 = _dev(W.random_smooth(n, p, seed=7, noise=0.02))
    dt = 0.2 * s.dt_cfl(Q0, 1.0)
    Qa, ra = Q0.clone(), torch.zeros_like(Q0)
    Qb, rb = Q0.clone(), torch.zeros_like(Q0)
    s.step(Qa, ra, dt, nsteps=3)
    for _ in range(3):
        s.step(Qb, rb, dt)
    torch.cuda.synchronize()
    assert torch.equal(Qa, Qb)


def test_fp32_vs_fp64_tgv32_full_size(dgm):
    """Second workload at full size for 10 steps: L2 difference between the
    FP32 and FP64 GPU forms (the FP64 form equals the oracle to 1e-12)."""
    import torch
    L = (2 * math.pi,) * 3
    Q0 = _dev(W.tgv(32, 3))
    s64 = dgm.Solver((32,) * 3, 3, L=L)
    s32 = dgm.Solver((32,) * 3, 3, L=L, precision=dgm.DG_FP32_MFMA)
    dt = s64.dt_cfl(Q0, 0.3)
    Qa, ra = Q0.clone(), torch.zeros_like(Q0)
    Qb, rb = Q0.clone(), torch.zeros_like(Q0)
    s64.step(Qa, ra, dt, nsteps=10)
    s32.step(Qb, rb, dt, nsteps=10)
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(Qb - Qa) / torch.linalg.vector_norm(Qa))
    chg = float(torch.linalg.vector_norm(Qb - Qa) / torch.linalg.vector_norm(Qa - Q0))
    print(f"fp32 vs fp64, 10 steps of TGV 32^3 p=3: rel {err:.3e}, rel to change {chg:.3e}")
    assert err <= 1e-8 and chg <= 1e-4
