"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle (a flipped sign, a
transposed operand, a wrong neighbour direction, a dropped term, a wrong
metric or coefficient) and runs the oracle's pin tests against the copy:
at least one pin must fail.  An unmodified copy must pass them all (so a
failure is the planted mistake's, not the harness's).  Everything runs on
the CPU, in subprocesses, on temporary copies; the repository's oracle is
never changed."""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["test_oracle_quadrature.py", "test_oracle_euler.py", "test_oracle_dg.py", "test_oracle_lserk.py",
             "test_oracle_adjoint.py", "test_oracle_viscous.py", "test_oracle_splitform.py", "test_oracle_varp.py",
             "test_oracle_hp.py"]

# (oracle file, exact text, replacement, what the mistake is)
MUTATIONS = [
    ("euler.py", "return 0.5 * (fm + fp) - 0.5 * lam", "return 0.5 * (fm + fp) + 0.5 * lam",
     "sign of the Lax-Friedrichs dissipation"),
    ("euler.py", "lam = _max(lam_m, lam_p)", "lam = np.minimum(lam_m, lam_p)", "min instead of max wave speed"),
    ("euler.py", "out[1 + d] = out[1 + d] + p", "out[1 + d] = out[1 + d]", "pressure dropped from the momentum flux"),
    ("euler.py", "(q[4] + p) * ud", "q[4] * ud", "pressure work dropped from the energy flux"),
    ("euler.py", "return (gamma - 1.0) * (en - 0.5", "return (gamma - 1.0) * (en - 1.0",
     "kinetic-energy factor in the pressure"),
    ("dg.py", "V += (Fd.reshape(-1, N3) @ self.Grad[d])", "V += (Fd.reshape(-1, N3) @ self.Grad[d].T)",
     "transposed volume operator"),
    ("dg.py", "q_nbr = np.roll(q, -1, axis=ax)", "q_nbr = np.roll(q, 1, axis=ax)", "wrong neighbour direction"),
    ("dg.py", "q_minus = (flat @ Bp.T)", "q_minus = (flat @ Bm.T)", "trace taken on the wrong face"),
    ("dg.py", "S -= np.roll(contrib, 1, axis=ax)", "S -= np.roll(contrib, -1, axis=ax)",
     "face flux lifted into the wrong element"),
    ("dg.py", "self.Jf = np.array([hy * hz / 4.0, hx * hz / 4.0, hx * hy / 4.0])",
     "self.Jf = np.array([hx * hz / 4.0, hy * hz / 4.0, hx * hy / 4.0])", "face Jacobians swapped"),
    ("dg.py", "* (2.0 / self.h[d])\n", "* (2.0 / self.h[0])\n", "metric of the x direction used for all"),
    ("dg.py", "return 3 - d", "return 1 + d", "x and z axes of the element array swapped"),
    ("dg.py", "(V - S).reshape(-1, N3).T", "(V + S).reshape(-1, N3).T", "sign of the surface term"),
    ("dg.py", "ke = np.einsum(\"et,t->\", 0.5 *", "ke = np.einsum(\"et,t->\", 1.0 *", "kinetic-energy integral factor"),
    ("dg.py", "r = sum((np.abs(q[1 + d] / q[0]) + c) / self.h[d]", "r = sum((np.abs(q[1 + d] / q[0]) + c) / self.h[0]",
     "wave rate uses one mesh spacing"),
    ("lserk.py", "Fraction(-2404267990393, 2016746695238)", "Fraction(-2404267990393, 2016746695239)",
     "one Runge-Kutta coefficient off in the last digit"),
    ("quadrature.py", "weights = 2.0 * vecs[0, :] ** 2", "weights = 2.0 * vecs[0, :] ** 2 * (1 + 1e-9)",
     "quadrature weights off by 1e-9"),
    ("viscous.py", "tau = tau - (2.0 / 3.0) * self.mu * div", "tau = tau - (1.0 / 3.0) * self.mu * div",
     "wrong bulk-viscosity factor"),
    ("viscous.py", "tau = self.mu * (grad_u[d, k] + grad_u[k, d])", "tau = self.mu * (grad_u[d, k] + grad_u[d, k])",
     "velocity gradient not symmetrised"),
    ("viscous.py", "mean = 0.5 * (own + nbr)", "mean = own", "one-sided instead of central face value"),
    ("viscous.py", "nbr = (np.roll(X, -1, axis=ax)", "nbr = (np.roll(X, 1, axis=ax)", "wrong neighbour in the lifting"),
    ("viscous.py", "en = self.kappa * theta[d, 3]", "en = 0.0 * theta[d, 3]", "heat flux dropped"),
    ("viscous.py", "/ (self.gamma - 1.0)) / self.prandtl", "/ (self.gamma - 1.0)) * self.prandtl",
     "conductivity multiplied by the Prandtl number"),
    ("viscous.py", "out = np.linalg.solve(self.M, (S - V)", "out = np.linalg.solve(self.M, (V - S)",
     "sign of the weak derivative"),
    ("viscous.py", "en = en + vel[k] * tau", "en = en", "viscous work dropped from the energy flux"),
    ("splitform.py", "m = mass * (0.5 * (ua[k] + ub[k]))", "m = 0.5 * (qa[1 + k] + qb[1 + k]) * ud",
     "momentum mean taken of rho u instead of the product of means"),
    ("splitform.py", "out.append(mass * (0.5 * (ea + eb)) + pm * ud)", "out.append(mass * (0.5 * (ea + eb)))",
     "pressure work dropped from the two-point energy flux"),
    ("splitform.py", "Qn[N:, :N] = -0.5 * self.B1 @ self.E1", "Qn[N:, :N] = 0.5 * self.B1 @ self.E1",
     "sign of the face-row coupling block"),
    ("splitform.py", "r = r + np.einsum(\"fi,f,...f->...i\", self.E1, np.diag(self.B1), corr)",
     "r = r - np.einsum(\"fi,f,...f->...i\", self.E1, np.diag(self.B1), corr)", "sign of the interface correction"),
    ("splitform.py", "nbr_plus = np.roll(t_plus, 1, axis=ax)", "nbr_plus = np.roll(t_plus, -1, axis=ax)",
     "wrong neighbour on the -d face"),
    ("varp.py", "m = max(p, pn)", "m = min(p, pn)", "mortar rule of the lower degree"),
    ("varp.py", "qp = self.element(Q, nb) @ Bm_nbr.T", "qp = q @ Bm_own.T", "own trace used for the neighbour's"),
    ("varp.py", "S[:, snb] -= fstar @ Bm_nbr", "S[:, snb] += fstar @ Bm_nbr", "sign of the neighbour's face term"),
    ("varp.py", "wf, Bm_own = self._mortar(d, 1, p, m)", "wf, Bm_own = self._mortar(d, -1, p, m)",
     "own trace taken on the wrong face"),
    ("varp.py", "return w[lo] * w[hi], basis3d", "return w[lo] * w[lo], basis3d", "mortar weights of one axis twice"),
    ("hp.py", "small = a if self.size[a][t[0]] <= self.size[b][t[0]] else b",
     "small = a if self.size[a][t[0]] >= self.size[b][t[0]] else b", "mortar on the larger face"),
    ("hp.py", "ra[:, d], rb[:, d] = 1.0, -1.0", "ra[:, d], rb[:, d] = 1.0, 1.0", "neighbour's trace on its far face"),
    ("hp.py", "kk[t[0]], kk[t[1]] = k1, k2", "kk[t[0]], kk[t[1]] = k1, k1", "one quarter of a hanging face twice"),
    ("hp.py", "S[:, self.off[b]:self.off[b + 1]] -= fstar @ Bb", "S[:, self.off[b]:self.off[b + 1]] += fstar @ Bb",
     "sign of the neighbour's face term"),
    ("hp.py", "area = self.size[small][t[0]] * self.size[small][t[1]] / 4.0",
     "area = self.hc[t[0]] * self.hc[t[1]] / 4.0", "the cell's face area for every sub-face"),
    ("hp.py", "                    kk[d] = 0\n", "                    kk[d] = 1\n", "wrong child across a cell face"),
]


def _copy_tree(dst):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "workloads"), os.path.join(dst, "workloads"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    for f in ["conftest.py", "parity.py", "__init__.py"] + PIN_TESTS:
        src = os.path.join(ROOT, "tests", f)
        if os.path.exists(src):
            shutil.copy(src, os.path.join(dst, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"),
                    ignore=shutil.ignore_patterns("*.npz", "__pycache__"))


def _run_pins(dst, first=None):
    """All pins, stopping at the first failure; the mutated module's own
    pin file (test_oracle_<module>.py) first, so that a caught mistake
    stops early."""
    order = sorted(PIN_TESTS, key=lambda f: f != first)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + \
          [os.path.join("tests", f) for f in order]
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2")
    return subprocess.run(cmd, cwd=dst, capture_output=True, text=True, timeout=600, env=env)


def _case(tmp, k, mutation):
    dst = os.path.join(tmp, f"case{k}")
    _copy_tree(dst)
    first = None
    if mutation is not None:
        fname, old, new, _ = mutation
        path = os.path.join(dst, "oracle", fname)
        src = open(path).read()
        assert src.count(old) == 1, f"mutation anchor not found once in {fname}: {old!r}"
        open(path, "w").write(src.replace(old, new))
        first = "test_oracle_" + fname
    return _run_pins(dst, first)


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    cases = [None] + MUTATIONS
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda kc: _case(str(tmp_path), kc[0], kc[1]), enumerate(cases)))
    control = results[0]
    assert control.returncode == 0, "unmodified oracle copy fails its pins:\n" + control.stdout[-2000:]
    missed = []
    for mut, res in zip(MUTATIONS, results[1:]):
        tail = res.stdout.strip().splitlines()[-1] if res.stdout.strip() else ""
        # a pin must fail (exit status 1 with a failure), not the run break (collection error, 2+)
        if res.returncode != 1 or "failed" not in tail:
            missed.append((mut[3], res.returncode, tail))
    assert not missed, f"planted mistakes not caught by any pin: {missed}"
