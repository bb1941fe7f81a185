"""Batched multi-mesh path: every mesh of a batch reproduces the single-mesh
entry points bit for bit (same per-element arithmetic), graph replays equal
eager launches, the tile choice does not change results, and sampled meshes
match the oracle."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.dg import DG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _specs(count, seed, nmin, nmax):
    return W.batch_specs(count=count, seed=seed, nmin=nmin, nmax=nmax)


def _setup(dgm, specs, precision=None, tiles=None):
    import torch
    prec = dgm.DG_FP64 if precision is None else precision
    b = dgm.Batch([(s["n"],) * 3 for s in specs], [s["p"] for s in specs], [s["L"] for s in specs],
                  precision=prec, tiles=tiles)
    states = [W.batch_state(s) for s in specs]
    Q = b.pack([torch.from_numpy(x) for x in states])
    return b, states, Q


def _dts(specs, states):
    return [0.3 * DG((s["n"],) * 3, s["p"], L=s["L"]).dt_cfl(x, 1.0) for s, x in zip(specs, states)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_rhs_and_steps_equal_single_mesh(dgm, prec):
    import torch
    specs = _specs(14, 7, 2, 5)
    mode = dgm.DG_FP64 if prec == "fp64" else dgm.DG_FP32_MFMA
    print(f"[batch {prec}] degrees", [s["p"] for s in specs], flush=True)
    b, states, Q = _setup(dgm, specs, mode)
    R = b.rhs(Q)
    dts = _dts(specs, states)
    b.set_dt(dts)
    Qs = Q.clone()
    res = torch.zeros_like(Qs)
    b.step(Qs, res, nsteps=3)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        single = dgm.Solver((s["n"],) * 3, s["p"], L=s["L"], precision=mode)
        Qi = torch.from_numpy(states[i]).cuda()
        assert torch.equal(b.view(R, i), single.rhs(Qi)), i
        ri = torch.zeros_like(Qi)
        single.step(Qi, ri, dts[i], nsteps=3)
        torch.cuda.synchronize()
        assert torch.equal(b.view(Qs, i), Qi), i
        assert torch.equal(b.view(res, i), ri), i


def test_batch_graph_replays_equal_eager(dgm):
    """Graph replays of the five stage launches, interleaved with eager work
    and synchronisation, give bitwise the eager result at every check."""
    import torch
    specs = _specs(10, 11, 2, 5)
    b, states, Q0 = _setup(dgm, specs)
    b.set_dt(_dts(specs, states))
    Qa, ra = Q0.clone(), torch.zeros_like(Q0)
    Qb, rb = Q0.clone(), torch.zeros_like(Q0)
    for rep in range(4):
        b.step(Qa, ra, nsteps=1 + rep, graph=False)
        junk = (Qb * 2.0).sum()      # unrelated eager work between replays
        torch.cuda.synchronize()
        b.step(Qb, rb, nsteps=1 + rep, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(Qa, Qb), rep
        assert torch.isfinite(junk)


def test_batch_tiles_do_not_change_results(dgm):
    import torch
    specs = _specs(12, 13, 2, 4)
    b1, states, Q = _setup(dgm, specs)
    tiles = {p: dgm.dg_batch_tile_options(p)[0] for p in range(1, 6)}
    b2, _, _ = _setup(dgm, specs, tiles=tiles)
    dts = _dts(specs, states)
    b1.set_dt(dts)
    b2.set_dt(dts)
    Qa, ra = Q.clone(), torch.zeros_like(Q)
    Qb, rb = Q.clone(), torch.zeros_like(Q)
    b1.step(Qa, ra, nsteps=2)
    b2.step(Qb, rb, nsteps=2, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(Qa, Qb)


def test_batch_sampled_meshes_vs_oracle(dgm):
    import torch
    specs = _specs(8, 17, 2, 3)
    b, states, Q = _setup(dgm, specs)
    dts = _dts(specs, states)
    b.set_dt(dts)
    Qs, res = Q.clone(), torch.zeros_like(Q)
    b.step(Qs, res, nsteps=2)
    torch.cuda.synchronize()
    for i in (0, 3, 5, 7):
        s = specs[i]
        ora = DG((s["n"],) * 3, s["p"], L=s["L"])
        Qo = lserk.integrate(states[i], dts[i], 2, ora.rhs)
        got = b.view(Qs, i).cpu().numpy()
        d = np.abs(got - Qo).reshape(5, -1).max(axis=1)
        assert np.all(d <= 1e-12 * np.abs(Qo).reshape(5, -1).max(axis=1)), (i, d)


def test_batch_errors(dgm):
    with pytest.raises(dgm.DGError):
        dgm.dg_batch_create([(2, 2, 2)], [0], [(1.0, 1.0, 1.0)])     # p = 0 not batched
    with pytest.raises(dgm.DGError):
        dgm.dg_batch_create([(2, 2, 2)], [6], [(1.0, 1.0, 1.0)])
    b = dgm.dg_batch_create([(2, 2, 2)], [2], [(1.0, 1.0, 1.0)])
    try:
        with pytest.raises(dgm.DGError):
            dgm.dg_batch_set_tile(b, 2, 5)     # not a built tile
        import torch
        Q = torch.zeros(5 * 8 * 27, dtype=torch.float64, device="cuda")
        with pytest.raises(dgm.DGError):
            dgm.dg_batch_rk_steps(b, Q, Q.clone(), 1)     # no workspace yet
    finally:
        dgm.dg_batch_destroy(b)


def test_batch_visiting_orders_bitwise_equal(dgm):
    """Every work-list order (row or pencil order inside a mesh, XCD split
    on or off, ragged pencils) and both launch forms (one persistent launch,
    one launch per degree) give bitwise the same steps."""
    import torch
    specs = _specs(12, 19, 2, 7)
    b, states, Q0 = _setup(dgm, specs)
    b.set_dt(_dts(specs, states))
    ref = None
    P, D = dgm.DG_BATCH_PERSISTENT, dgm.DG_BATCH_PER_DEGREE
    for launch, xcd, order, px, pz in [(P, 0, dgm.DG_ORDER_LINEAR, 0, 1), (P, 1, dgm.DG_ORDER_LINEAR, 0, 1),
                                       (P, 0, dgm.DG_ORDER_PENCIL, 3, 2), (P, 1, dgm.DG_ORDER_PENCIL, 16, 8),
                                       (P, 1, dgm.DG_ORDER_PENCIL, 5, 3), (D, 0, dgm.DG_ORDER_LINEAR, 0, 1),
                                       (D, 1, dgm.DG_ORDER_LINEAR, 0, 1), (D, 1, dgm.DG_ORDER_PENCIL, 5, 3)]:
        b.set_option(dgm.DG_OPT_BATCH_LAUNCH, launch)
        b.set_option(dgm.DG_OPT_XCD_REMAP, xcd)
        b.set_option(dgm.DG_OPT_ORDER, order)
        b.set_option(dgm.DG_OPT_PENCIL_X, px)
        b.set_option(dgm.DG_OPT_PENCIL_Z, pz)
        assert b.options()["xcd_remap"] == xcd and b.options()["pencil_z"] == pz
        Q, r = Q0.clone(), torch.zeros_like(Q0)
        b.step(Q, r, nsteps=2, graph=True)
        torch.cuda.synchronize()
        if ref is None:
            ref = Q
        assert torch.equal(Q, ref), (launch, xcd, order, px, pz)
