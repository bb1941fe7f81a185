"""GPU parity of the FP64 hot path against the oracle, through the C ABI.

Bar: per field, |R_gpu - R_oracle|_inf <= 1e-12 (|R_oracle|_inf + S_f),
S_f the summand scale of the contraction (cancellation scale, see
tests/parity.py); states with O(1) right-hand sides also meet the plain
relative bar |dR|_inf <= 1e-12 |R_oracle|_inf."""

import math

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle import lserk
from tests.parity import TOL, patch_rhs, rhs_errors, summand_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _solver(dgm, n, p, L):
    return dgm.Solver(n, p, L=L)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("p", range(0, 8))
def test_rhs_random_state_all_degrees(dgm, p):
    """Anisotropic mesh and box, discontinuous smooth random state; the
    element count (30) leaves a ragged last workgroup for most degrees."""
    n, L = (3, 2, 5), (1.0, 1.3, 0.7)
    print(f"[rhs random p={p} n={n}]", flush=True)
    Q = W.random_smooth(n, p, seed=20 + p, L=L, noise=0.05)
    ora = DG(n, p, L=L)
    Ro = ora.rhs(Q)
    s = _solver(dgm, n, p, L)
    Rg = _host(s.rhs(_dev(Q)))
    plain, scaled = rhs_errors(ora, Q, Rg, Ro)
    print("plain", plain, "scaled", scaled)
    assert np.all(scaled <= TOL)
    assert np.all(plain <= TOL)


@pytest.mark.parametrize("n,p", [((1, 1, 1), 1), ((1, 1, 1), 3), ((2, 1, 3), 2), ((7, 5, 3), 4),
                                 ((5, 3, 1), 3), ((1, 9, 2), 5)])
def test_rhs_edge_meshes(dgm, n, p):
    """Self-neighbour (1 element per direction), two-element periodicity and
    ragged element counts."""
    L = (0.9, 1.1, 1.0)
    print(f"[rhs edge p={p} n={n}]", flush=True)
    Q = W.random_smooth(n, p, seed=31, L=L, noise=0.1)
    ora = DG(n, p, L=L)
    Ro = ora.rhs(Q)
    Rg = _host(_solver(dgm, n, p, L).rhs(_dev(Q)))
    plain, scaled = rhs_errors(ora, Q, Rg, Ro)
    assert np.all(scaled <= TOL) and np.all(plain <= TOL), (plain, scaled)


def test_rhs_density_wave_c1(dgm):
    """First workload: 4^3 elements, p = 1, rho = 1 + 0.2 sin(2 pi (x+y+z))."""
    Q = W.density_wave(4, 1)
    ora = DG((4, 4, 4), 1)
    Ro = ora.rhs(Q)
    Rg = _host(_solver(dgm, (4, 4, 4), 1, (1.0, 1.0, 1.0)).rhs(_dev(Q)))
    plain, scaled = rhs_errors(ora, Q, Rg, Ro)
    assert np.all(plain <= TOL), plain


def test_rhs_tgv_c2_full_size(dgm):
    """Second workload at its full size: TGV 32^3 elements, p = 3, Mach 0.1.
    Low Mach: the right-hand side is a difference of summands ~p0 = 71, so
    momentum and energy are judged on the summand-scaled bar."""
    print("[rhs tgv 32^3 p=3]", flush=True)
    L = (2 * math.pi,) * 3
    Q = W.tgv(32, 3)
    ora = DG((32, 32, 32), 3, L=L)
    Ro = ora.rhs(Q)
    Rg = _host(_solver(dgm, (32, 32, 32), 3, L).rhs(_dev(Q)))
    plain, scaled = rhs_errors(ora, Q, Rg, Ro)
    print("plain", plain, "scaled", scaled)
    assert np.all(scaled <= TOL)


def test_rhs_tgv_c3_full_size_sampled(dgm):
    """Third workload at its full size (TGV 48^3, p = 4, 13.8M nodes) in the
    launch configuration the benchmark times: sampled elements against the
    oracle evaluated on the 3x3x3 periodic patch around each."""
    import torch
    print("[rhs tgv 48^3 p=4 sampled]", flush=True)
    n, p, L = (48, 48, 48), 4, (2 * math.pi,) * 3
    Q = W.tgv(48, 4)
    s = _solver(dgm, n, p, L)
    Rg = _host(s.rhs(_dev(Q)))
    rng = np.random.default_rng(48)
    elems = [(0, 0, 0), (47, 47, 47), (47, 0, 23)] + [tuple(int(v) for v in rng.integers(0, 48, 3))
                                                      for _ in range(9)]
    ref = patch_rhs(n, p, L, Q, elems)
    small = DG((3, 3, 3), p, L=tuple(3 * np.array(L) / 48))
    for (ex, ey, ez), Ro in ref.items():
        got = Rg[:, ez, ey, ex]
        d = np.abs(got - Ro).reshape(5, -1).max(axis=1)
        S = summand_scale(small, Q[:, ez, ey, ex])
        assert np.all(d <= TOL * (np.abs(Ro).reshape(5, -1).max(axis=1) + S)), ((ex, ey, ez), d, S)
    del Rg
    torch.cuda.empty_cache()


def test_free_stream_and_conservation_full_size(dgm):
    """Properties that hold at any size: a uniform state has zero right-hand
    side, and sum_e J w R = 0 for every field (periodic conservation)."""
    import torch
    n, p, L = (48, 48, 48), 4, (2 * math.pi,) * 3
    s = _solver(dgm, n, p, L)
    Q = W.uniform_state(48, 4, 1.1, (0.3, -0.4, 0.2), 71.4)
    R = s.rhs(_dev(Q))
    torch.cuda.synchronize()
    S = summand_scale(DG(n, p, L=L), Q[:, :1, :1, :1])
    assert np.all(R.abs().reshape(5, -1).max(dim=1).values.cpu().numpy() <= 1e-13 * S)
    Q = W.tgv(48, 4)
    Qd = _dev(Q)
    R = s.rhs(Qd)
    ints = s.integrals(R)   # sum J w R_f (the KE entry is not used)
    # Exact in exact arithmetic; in FP64 the rounding of the 1-D tables acts
    # on fluxes of size ~p0, so the bound is relative to the summand scale
    # integrated over the domain (a wrong face weight or neighbour would give
    # errors of order one times the same scale).
    vol = (2 * math.pi) ** 3
    S = summand_scale(DG(n, p, L=L), Q)
    for f in range(5):
        assert abs(ints[f]) <= 1e-13 * vol * S[f], (f, ints[f], vol * S[f])


def test_rhs_deterministic(dgm):
    import torch
    n, p = (6, 5, 4), 3
    Q = _dev(W.random_smooth(n, p, seed=5, noise=0.05))
    s = _solver(dgm, n, p, (1.0, 1.0, 1.0))
    a = s.rhs(Q).clone()
    b = s.rhs(Q)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_translation_equivariance_bitwise(dgm):
    import torch
    n, p = (6, 4, 5), 3
    Q = W.random_smooth(n, p, seed=6, noise=0.05)
    s = _solver(dgm, n, p, (1.0, 1.0, 1.0))
    R = _host(s.rhs(_dev(Q)))
    for ax in (1, 2, 3):
        Rs = _host(s.rhs(_dev(np.roll(Q, 1, axis=ax))))
        assert np.array_equal(Rs, np.roll(R, 1, axis=ax))
