"""dg_rk_steps_noalloc, the entry point for callers that cannot allocate:
called through the C ABI on contexts that have no workspace, its result
equals dg_rk_steps' on a workspace context bit for bit, on two calls in a
row (the second on a smaller mesh, so the shared static buffer still holds
the first call's larger state), in both precisions, with odd and even step
counts (an odd count ends with the copy back out of the static buffer)."""

import ctypes
import math

import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _bare_ctx(dgm, n, p, L, precision):
    """A context with no workspace set."""
    ctx = dgm.dg_create(*n, p, 1.4)
    dgm.dg_set_domain(ctx, *L)
    dgm.dg_set_precision(ctx, precision)
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_rk_steps_on_two_calls(dgm, prec):
    import torch
    mode = dgm.DG_FP64 if prec == "fp64" else dgm.DG_FP32_MFMA
    lib = dgm._lib
    cases = [((24, 20, 22), 3, 3, (2 * math.pi,) * 3, "tgv"),      # 3 steps: ends in the static buffer
             ((7, 5, 6), 4, 2, (1.0, 0.8, 1.3), "random")]          # smaller state, 2 steps
    for n, p, nsteps, L, kind in cases:
        print(f"[noalloc {prec}] mesh {n} p={p}, {nsteps} steps", flush=True)
        Q0 = W.tgv(n, p, L=L) if kind == "tgv" else W.random_smooth(n, p, seed=7, L=L, noise=0.02)
        ref = dgm.Solver(n, p, L=L, precision=mode)
        Qa = torch.from_numpy(Q0).cuda()
        dt = 0.3 * ref.dt_cfl(Qa, 1.0)
        ra = torch.zeros_like(Qa)
        ref.step(Qa, ra, dt, nsteps=nsteps)
        ctx = _bare_ctx(dgm, n, p, L, mode)
        try:
            Qb = torch.from_numpy(Q0).cuda()
            rb = torch.zeros_like(Qb)
            dgm.dg_set_stream(ctx, None)
            rc = lib.dg_rk_steps_noalloc(ctx, Qb.data_ptr(), rb.data_ptr(), ctypes.c_double(dt), nsteps)
            assert rc == dgm.DG_OK, dgm.dg_last_error()
            torch.cuda.synchronize()
            assert torch.equal(Qa, Qb)
            assert torch.equal(ra, rb)
        finally:
            dgm.dg_destroy(ctx)


def test_noalloc_rejects_states_beyond_its_buffer(dgm):
    """Validation before any launch: the fake device addresses below are
    never dereferenced."""
    lib = dgm._lib
    ctx = _bare_ctx(dgm, (64, 64, 64), 3, (1.0, 1.0, 1.0), dgm.DG_FP64)   # 671 MB of state
    try:
        assert 5 * 64 ** 3 * 64 * 8 > dgm.DG_NOALLOC_MAX_BYTES
        rc = lib.dg_rk_steps_noalloc(ctx, 0x10000000, 0x90000000, ctypes.c_double(1e-3), 1)
        assert rc == dgm.DG_EUNSUPPORTED
        assert "static buffer" in dgm.dg_last_error()
        assert lib.dg_rk_steps_noalloc(ctx, 0x10000000, 0x90000000, ctypes.c_double(1e-3), -1) == dgm.DG_EINVAL
        assert lib.dg_rk_steps_noalloc(ctx, None, 0x90000000, ctypes.c_double(1e-3), 1) == dgm.DG_EINVAL
    finally:
        dgm.dg_destroy(ctx)
