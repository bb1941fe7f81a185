"""The batched workload at its real size: 512 independent meshes from seed
15698 (n^3 elements with n in 6..24, p in 1..5; 205 M nodes, 934,075 work
items), advanced by one launch per degree and RK stage (the default), and
by the persistent launch whose grid holds only the resident workgroups, so
that every workgroup walks about 1,200 items of mixed (degree, tile)
variants through one shared-memory buffer.

Checked here, in both the FP64 and the FP32 matrix-core form, on the
default launch form:
  - 20 sampled meshes (four per degree: the largest n, the smallest n and two
    seeded picks) bitwise against single-mesh contexts on the same state and
    dt: one right-hand side and two graph-replayed steps (state and residual);
  - the smallest mesh of every degree (n = 6) against the oracle after the two
    steps, whole mesh (FP64: 1e-12 of the state per field; the FP32 form's
    L2 error is printed per degree and held to a stated bound);
  - the two largest p = 5 meshes (24^3) against the oracle on sampled
    elements of the batched right-hand side (3x3x3 periodic patches);
and the persistent launch bitwise equal to it over the whole batch
(right-hand side, state and residual).
"""

import numpy as np
import pytest

import workloads as W
from oracle import lserk
from oracle.dg import DG
from tests.parity import TOL, patch_rhs, rhs_errors

pytestmark = pytest.mark.gpu

STEPS = 2


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _samples(specs):
    rng = np.random.default_rng(1569)
    picks = []
    for p in range(1, 6):
        idx = [i for i, s in enumerate(specs) if s["p"] == p]
        by_n = sorted(idx, key=lambda i: (specs[i]["n"], i))
        chosen = [by_n[-1], by_n[0]]
        rest = [i for i in idx if i not in chosen]
        chosen += [int(v) for v in rng.choice(rest, size=2, replace=False)]
        picks += chosen
    return picks


@pytest.fixture(scope="module")
def c4(dgm):
    """Batch, initial state on the GPU, per-mesh dt (CFL 0.3 from the oracle's
    wave rate) and host copies of the sampled meshes' initial states."""
    import torch
    specs = W.batch_specs(count=512, seed=15698)
    b = dgm.Batch([(s["n"],) * 3 for s in specs], [s["p"] for s in specs], [s["L"] for s in specs])
    Q0 = b.empty()
    dts = []
    for i, s in enumerate(specs):
        x = W.batch_state(s)
        dts.append(DG((s["n"],) * 3, s["p"], L=s["L"]).dt_cfl(x, 0.3))
        b.view(Q0, i).copy_(torch.from_numpy(x))
    b.set_dt(dts)
    torch.cuda.synchronize()
    picks = _samples(specs)
    tile = {p: b.tiles.get(p, dgm.dg_batch_tile_options(p)[-1]) for p in range(1, 6)}
    nitems = sum(s["n"] ** 2 * -(-s["n"] // tile[s["p"]]) for s in specs)
    print(f"[c4] {len(specs)} meshes, {b.total // 5} nodes, tiles {tile}, work items {nitems}, "
          f"sampled meshes {picks}", flush=True)
    return dict(b=b, specs=specs, Q0=Q0, dts=dts, picks=picks)


def _run(dgm, c4, mode):
    import torch
    b = c4["b"]
    dgm.dg_batch_set_precision(b.b, mode)
    R = b.rhs(c4["Q0"])
    Q = c4["Q0"].clone()
    res = torch.zeros_like(Q)
    b.step(Q, res, nsteps=STEPS, graph=True)
    torch.cuda.synchronize()
    return R, Q, res


def _bitwise_vs_single(dgm, c4, mode, R, Q, res):
    import torch
    b, specs = c4["b"], c4["specs"]
    for i in c4["picks"]:
        s = specs[i]
        single = dgm.Solver((s["n"],) * 3, s["p"], L=s["L"], precision=mode)
        Qi = b.view(c4["Q0"], i).clone()
        assert torch.equal(b.view(R, i), single.rhs(Qi)), ("rhs", i)
        ri = torch.zeros_like(Qi)
        single.step(Qi, ri, c4["dts"][i], nsteps=STEPS)
        torch.cuda.synchronize()
        assert torch.equal(b.view(Q, i), Qi), ("state", i)
        assert torch.equal(b.view(res, i), ri), ("residual", i)
        del single


def _oracle_small(c4, Q, p):
    """(GPU state, oracle state, initial state) of the smallest mesh of
    degree p after STEPS steps."""
    b, specs = c4["b"], c4["specs"]
    i = min((j for j, s in enumerate(specs) if s["p"] == p), key=lambda j: (specs[j]["n"], j))
    s = specs[i]
    x0 = b.view(c4["Q0"], i).cpu().numpy()
    ora = DG((s["n"],) * 3, s["p"], L=s["L"])
    Qo = lserk.integrate(x0, c4["dts"][i], STEPS, ora.rhs)
    return i, b.view(Q, i).cpu().numpy(), Qo, x0


@pytest.mark.timeout(400)
def test_c4_fp64_batch(dgm, c4):
    R, Q, res = _run(dgm, c4, dgm.DG_FP64)
    _bitwise_vs_single(dgm, c4, dgm.DG_FP64, R, Q, res)
    for p in range(1, 6):
        i, got, Qo, _ = _oracle_small(c4, Q, p)
        d = np.abs(got - Qo).reshape(5, -1).max(axis=1)
        m = np.abs(Qo).reshape(5, -1).max(axis=1)
        # momentum components against the momentum vector's size: a TGV has
        # w = 0, so rho w alone stays near zero and its own maximum says
        # nothing about the rounding of the other components it mixes with
        ref = np.array([m[0], m[1:4].max(), m[1:4].max(), m[1:4].max(), m[4]])
        print(f"[c4 fp64] mesh {i} p={p} n={c4['specs'][i]['n']}: state-relative error per field {d / ref}",
              flush=True)
        assert np.all(d <= TOL * ref), (i, d / ref)
    specs, b = c4["specs"], c4["b"]
    big = sorted((j for j, s in enumerate(specs) if s["p"] == 5), key=lambda j: (specs[j]["n"], j))[-2:]
    rng = np.random.default_rng(24)
    for i in big:
        s = specs[i]
        n3 = (s["n"],) * 3
        x0 = b.view(c4["Q0"], i).cpu().numpy()
        Rg = b.view(R, i).cpu().numpy()
        elems = [tuple(int(v) for v in rng.integers(0, s["n"], size=3)) for _ in range(6)]
        elems.append((s["n"] - 1, s["n"] - 1, s["n"] - 1))
        ref = patch_rhs(n3, s["p"], s["L"], x0, elems)
        dg_small = DG((3, 3, 3), s["p"], L=tuple(3 * np.array(s["L"]) / s["n"]))
        for (ex, ey, ez), Ro in ref.items():
            got = Rg[:, ez, ey, ex]
            patch = x0[:, [(ez + o) % s["n"] for o in (-1, 0, 1)]][:, :, [(ey + o) % s["n"] for o in (-1, 0, 1)]][
                :, :, :, [(ex + o) % s["n"] for o in (-1, 0, 1)]]
            _, scaled = rhs_errors(dg_small, patch[:, 1:2, 1:2, 1:2], got[:, None, None, None],
                                   Ro[:, None, None, None])
            assert np.all(scaled <= TOL), (i, (ex, ey, ez), scaled)
        print(f"[c4 fp64] mesh {i} ({s['kind']}, n={s['n']}, p=5): batched RHS = oracle on {len(ref)} "
              "sampled elements", flush=True)


# The FP32 form's error against the oracle after two steps of the smallest
# mesh of each degree, relative to the oracle state (L2 over all nodes and
# fields).  Stated bound, not a parity claim: the contractions round to FP32
# (unit roundoff 6e-8) on deviations from a per-element FP64 anchor.
FP32_STATE_BOUND = 1e-8


@pytest.mark.timeout(400)
def test_c4_fp32_batch(dgm, c4):
    R, Q, res = _run(dgm, c4, dgm.DG_FP32_MFMA)
    try:
        _bitwise_vs_single(dgm, c4, dgm.DG_FP32_MFMA, R, Q, res)
        for p in range(1, 6):
            i, got, Qo, x0 = _oracle_small(c4, Q, p)
            e_state = np.linalg.norm(got - Qo) / np.linalg.norm(Qo)
            e_change = np.linalg.norm(got - Qo) / np.linalg.norm(Qo - x0)
            print(f"[c4 fp32] p={p} (mesh {i}, n={c4['specs'][i]['n']}): L2 error vs oracle "
                  f"{e_state:.3e} of the state, {e_change:.3e} of the {STEPS}-step change", flush=True)
            assert e_state <= FP32_STATE_BOUND, (p, e_state)
    finally:
        dgm.dg_batch_set_precision(c4["b"].b, dgm.DG_FP64)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c4_persistent_launch_equals_per_degree(dgm, c4, prec):
    """The same batch run as one persistent launch per stage
    (DG_BATCH_PERSISTENT, XCD split on and off) gives bitwise the default
    per-degree launches' right-hand side, state and residual over the whole
    batch, as does the per-degree form with the XCD remap."""
    import torch
    mode = dgm.DG_FP64 if prec == "fp64" else dgm.DG_FP32_MFMA
    b = c4["b"]
    assert b.options()["batch_launch"] == dgm.DG_BATCH_PER_DEGREE
    try:
        R0, Q0, r0 = _run(dgm, c4, mode)
        for launch, xcd in ((dgm.DG_BATCH_PERSISTENT, 0), (dgm.DG_BATCH_PERSISTENT, 1),
                            (dgm.DG_BATCH_PER_DEGREE, 1)):
            b.set_option(dgm.DG_OPT_BATCH_LAUNCH, launch)
            b.set_option(dgm.DG_OPT_XCD_REMAP, xcd)
            R, Q, res = _run(dgm, c4, mode)
            same = (torch.equal(R, R0), torch.equal(Q, Q0), torch.equal(res, r0))
            print(f"[c4 {prec}] launch form {launch}, xcd {xcd}: bitwise {same}", flush=True)
            assert all(same)
            del R, Q, res
    finally:
        b.set_option(dgm.DG_OPT_BATCH_LAUNCH, dgm.DG_BATCH_PER_DEGREE)
        b.set_option(dgm.DG_OPT_XCD_REMAP, 0)
        dgm.dg_batch_set_precision(b.b, dgm.DG_FP64)
