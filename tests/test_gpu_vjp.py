"""GPU adjoint (vector-Jacobian product) of the right-hand side against the
oracle's complex-step derivatives, and the checkpointed gradient through
LSERK45 steps against stored oracle values and central differences."""

import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, lserk
from oracle.dg import DG

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "adjoint_c5.json")


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


@pytest.mark.parametrize("n,p", [((2, 2, 2), 1), ((1, 2, 1), 2), ((2, 1, 1), 3), ((1, 1, 1), 4)])
def test_vjp_equals_dense_jacobian_transpose(dgm, n, p):
    """Tiny meshes: the full Jacobian column by column (complex step), then
    J^T v compared element by element."""
    print(f"[vjp dense n={n} p={p}]", flush=True)
    Q = W.random_smooth(n, p, seed=50 + p, noise=0.05)
    ora = DG(n, p)
    rng = np.random.default_rng(p)
    V = rng.standard_normal(Q.shape)
    ref = adjoint.vjp_dense(ora, Q, V)
    s = dgm.Solver(n, p)
    got = _host(s.rhs_vjp(_dev(Q), _dev(V)))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6, 7])
def test_vjp_dot_product_identity(dgm, p):
    """<J u, v> with J u from the oracle's complex step equals <u, J^T v>
    from the GPU adjoint, on a mesh with ragged workgroups."""
    n, L = (5, 3, 4), (1.0, 0.8, 1.3)
    print(f"[vjp dot p={p}]", flush=True)
    Q = W.random_smooth(n, p, seed=60 + p, L=L, noise=0.05)
    ora = DG(n, p, L=L)
    s = dgm.Solver(n, p, L=L)
    rng = np.random.default_rng(70 + p)
    for _ in range(3):
        U = rng.standard_normal(Q.shape)
        V = rng.standard_normal(Q.shape)
        ju = adjoint.jvp(ora, Q, U)
        jtv = _host(s.rhs_vjp(_dev(Q), _dev(V)))
        lhs = float(np.dot(ju.ravel(), V.ravel()))
        rhs = float(np.dot(U.ravel(), jtv.ravel()))
        scale = float(np.abs(ju).ravel() @ np.abs(V).ravel())
        assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)


def test_autograd_function(dgm):
    import torch
    n, p = (3, 2, 2), 2
    s = dgm.Solver(n, p)
    Q = _dev(W.random_smooth(n, p, seed=3, noise=0.05)).requires_grad_(True)
    V = _dev(np.random.default_rng(0).standard_normal(Q.shape))
    R = dgm.RHS.apply(Q, s)
    (R * V).sum().backward()
    ref = s.rhs_vjp(Q.detach(), V)
    torch.cuda.synchronize()
    assert torch.equal(Q.grad, ref)
    assert torch.equal(R.detach(), s.rhs(Q.detach()))


def test_reverse_stage_dot_product(dgm):
    """One LSERK45 stage (Q, res) -> (Q', res') and its reverse through
    dg_rk_stage_vjp satisfy <dOut, gOut> = <dIn, gIn>, with the tangent map
    from the oracle's complex step of its own stage."""
    n, p = (3, 3, 2), 3
    Q = W.random_smooth(n, p, seed=8, noise=0.02)
    res0 = 1e-3 * W.random_smooth(n, p, seed=9)
    ora = DG(n, p)
    dt = 0.2 * ora.dt_cfl(Q, 1.0)
    rng = np.random.default_rng(10)
    s = dgm.Solver(n, p)
    for st in range(5):
        dQ, dr = rng.standard_normal(Q.shape), rng.standard_normal(Q.shape)
        gQo, gro = rng.standard_normal(Q.shape), rng.standard_normal(Q.shape)
        h = 1e-30
        Qc = Q + 1j * h * dQ
        rc = res0 + 1j * h * dr
        lserk.stage(st, Qc, rc, dt, ora.rhs)
        tQ, tr = np.imag(Qc) / h, np.imag(rc) / h
        lhs = np.dot(tQ.ravel(), gQo.ravel()) + np.dot(tr.ravel(), gro.ravel())
        gQ, gr = _dev(gQo), _dev(gro)
        dgm.dg_rk_stage_vjp(s.ctx, st, _dev(Q), gQ, gr, dt)
        rhs = np.dot(dQ.ravel(), _host(gQ).ravel()) + np.dot(dr.ravel(), _host(gr).ravel())
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(gQo) * np.linalg.norm(dQ)), (st, lhs, rhs)


def _c5_setup(dgm):
    g = json.load(open(GOLD))
    L = (2 * math.pi,) * 3
    Q0 = W.perturbed_tgv(g["n"], g["p"], seed=g["seed"], amp=g["amp"], L=L)
    s = dgm.Solver((g["n"],) * 3, g["p"], L=L)
    return g, Q0, s


@pytest.mark.skipif(not os.path.exists(GOLD), reason="golden file not generated")
def test_c5_gradient_vs_oracle_complex_step(dgm):
    """Adjoint workload: gradient of KE after 40 steps (checkpoint every 8)
    dotted with seeded directions equals the oracle's complex-step
    directional derivatives."""
    import torch
    g, Q0, s = _c5_setup(dgm)
    dt = g["dt"]
    grad, Qf = dgm.rk_gradient(s, _dev(Q0), dt, g["steps"], dgm.kinetic_energy_grad(s), every=8)
    ints = s.integrals(Qf)
    assert abs(ints[5] - g["ke_final"]) <= 1e-12 * abs(g["ke_final"])
    dirs = W.gaussian_directions(Q0, len(g["directional_derivatives"]), seed0=g["direction_seed0"])
    G = _host(grad)
    for U, ref in zip(dirs, g["directional_derivatives"]):
        got = float(np.dot(G.ravel(), U.ravel()))
        assert abs(got - ref) <= 1e-11 * np.linalg.norm(G), (got, ref)


@pytest.mark.skipif(not os.path.exists(GOLD), reason="golden file not generated")
def test_c5_gradient_vs_central_differences_64_directions(dgm):
    """Central differences (h = 1e-6) of the GPU forward on 64 seeded
    directions.  Bound: FD truncation plus roundoff eps |KE| / h."""
    import torch
    g, Q0, s = _c5_setup(dgm)
    dt = g["dt"]
    Qd = _dev(Q0)
    grad, _ = dgm.rk_gradient(s, Qd, dt, g["steps"], dgm.kinetic_energy_grad(s), every=8)
    G = _host(grad)
    h = 1e-6

    def ke(Qs):
        Q = Qs.clone()
        r = torch.zeros_like(Q)
        s.step(Q, r, dt, nsteps=g["steps"])
        return s.integrals(Q)[5]
    dirs = W.gaussian_directions(Q0, 64, seed0=g["direction_seed0"])
    worst = 0.0
    for U in dirs:
        Ud = _dev(U)
        fd = (ke(Qd + h * Ud) - ke(Qd - h * Ud)) / (2 * h)
        ad = float(np.dot(G.ravel(), U.ravel()))
        floor = 20 * np.finfo(float).eps * abs(g["ke_final"]) / h
        assert abs(fd - ad) <= floor + 1e-6 * abs(ad), (fd, ad, floor)
        worst = max(worst, abs(fd - ad))
    print("worst |fd - adjoint|", worst)


@pytest.mark.parametrize("p", [1, 3, 4])
def test_kinetic_energy_grad_vs_oracle_complex_step(dgm, p):
    """dg_kinetic_energy_grad dotted with seeded directions equals the
    complex-step derivative of the oracle's kinetic-energy integral; the
    energy field has zero gradient."""
    n, L = (3, 4, 2), (1.0, 0.7, 1.2)
    Q = W.random_smooth(n, p, seed=80 + p, L=L, noise=0.05)
    ora = DG(n, p, L=L)
    s = dgm.Solver(n, p, L=L)
    G = _host(dgm.kinetic_energy_grad(s)(_dev(Q)))
    assert np.all(G[4] == 0.0)
    rng = np.random.default_rng(90 + p)
    h = 1e-30
    for _ in range(4):
        V = rng.standard_normal(Q.shape)
        ref = ora.integrals(Q + 1j * h * V)[5].imag / h
        got = float(np.dot(G.ravel(), V.ravel()))
        assert abs(got - ref) <= 1e-13 * np.linalg.norm(G) * np.linalg.norm(V), (got, ref)


def test_checkpointing_interval_does_not_change_gradient(dgm):
    import torch
    n, p = (4, 4, 4), 2
    L = (2 * math.pi,) * 3
    s = dgm.Solver(n, p, L=L)
    Q0 = _dev(W.perturbed_tgv(4, 2, seed=3, L=L))
    dt = 0.3 * s.dt_cfl(Q0, 1.0)
    fg = dgm.kinetic_energy_grad(s)
    g1, _ = dgm.rk_gradient(s, Q0, dt, 12, fg, every=1)
    g8, _ = dgm.rk_gradient(s, Q0, dt, 12, fg, every=8)
    g12, _ = dgm.rk_gradient(s, Q0, dt, 12, fg, every=12)
    torch.cuda.synchronize()
    assert torch.equal(g1, g8) and torch.equal(g8, g12)


@pytest.mark.parametrize("p,n", [(1, (7, 5, 3)), (2, (9, 2, 5)), (3, (6, 5, 7)), (4, (5, 3, 4)), (5, (3, 4, 5)),
                                 (6, (2, 3, 3)), (7, (1, 2, 3))])
def test_vjp_exchange_schemes_and_orders_bitwise_equal(dgm, p, n):
    """The neighbour-read adjoint (one launch) equals the trace-buffer adjoint
    (trace launches + VJP launch) bit for bit, for every visiting order, on
    ragged meshes (short row blocks, a one-element row)."""
    import torch
    print(f"[vjp schemes p={p} n={n}]", flush=True)
    Q = _dev(W.random_smooth(n, p, seed=130 + p, noise=0.05))
    V = torch.randn_like(Q)
    outs = []
    for exch, order, px, pz, remap in [(dgm.DG_EXCHANGE_TRACES, dgm.DG_ORDER_LINEAR, 0, 1, 0),
                                       (dgm.DG_EXCHANGE_NEIGHBOUR, dgm.DG_ORDER_LINEAR, 0, 1, 0),
                                       (dgm.DG_EXCHANGE_NEIGHBOUR, dgm.DG_ORDER_PENCIL, 3, 2, 1),
                                       (dgm.DG_EXCHANGE_NEIGHBOUR, dgm.DG_ORDER_PENCIL, 0, 40, 0)]:
        s = dgm.Solver(n, p)
        s.set_option(dgm.DG_OPT_EXCHANGE, exch)
        s.set_option(dgm.DG_OPT_ORDER, order)
        s.set_option(dgm.DG_OPT_PENCIL_X, px)
        s.set_option(dgm.DG_OPT_PENCIL_Z, pz)
        s.set_option(dgm.DG_OPT_XCD_REMAP, remap)
        outs.append(s.rhs_vjp(Q, V))
        torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(outs[0], o)
