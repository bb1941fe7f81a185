"""The reciprocal and square root inside the flux kernels (1/rho at every node
and face point, the sound speed of the Lax-Friedrichs wave speed) against the
correctly rounded IEEE division and square root that numpy computes on the
host, on seeded inputs spanning the state's range."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgm():
    from paper_2006_15698_amd import dg
    return dg


def _ulps(a, b):
    """Distance in units in the last place between positive doubles."""
    return np.abs(a.view(np.int64) - b.view(np.int64))


def test_recip_sqrt_equal_correctly_rounded(dgm):
    import torch
    rng = np.random.default_rng(2026)
    n = 1 << 22
    x = np.exp2(rng.uniform(-12.0, 12.0, n))              # log-uniform in [2^-12, 2^12]
    x[:4096] = 1.0 + rng.uniform(-1e-3, 1e-3, 4096)       # near 1 (densities)
    x[4096:4096 + 25] = np.exp2(np.arange(-12, 13))        # exact powers of two
    x[8192:8192 + 4096] = rng.uniform(60.0, 120.0, 4096)   # gamma p / rho at Mach 0.1
    xd = torch.from_numpy(x).cuda()
    r = torch.empty_like(xd)
    s = torch.empty_like(xd)
    dgm.dg_recip_sqrt(xd, r, s)
    torch.cuda.synchronize()
    rg, sg = r.cpu().numpy(), s.cpu().numpy()
    ur, us = _ulps(rg, 1.0 / x), _ulps(sg, np.sqrt(x))
    print(f"recip: {np.count_nonzero(ur)} of {n} differ (max {ur.max()} ulp); "
          f"sqrt: {np.count_nonzero(us)} differ (max {us.max()} ulp)")
    assert ur.max() == 0 and us.max() == 0


def test_sqrt_of_zero(dgm):
    import torch
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    r = torch.empty_like(x)
    s = torch.empty_like(x)
    dgm.dg_recip_sqrt(x, r, s)
    torch.cuda.synchronize()
    assert torch.all(s == 0.0)
