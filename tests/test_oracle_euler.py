"""Pins of the oracle's pointwise physics (Section II-A, Eqs. (2)-(3)) and of
its local Lax-Friedrichs flux (Section II-B)."""

import json
import os

import numpy as np
import pytest

from oracle.euler import flux, lax_friedrichs, pressure, sound_speed

GOLD = os.path.join(os.path.dirname(__file__), "golden", "euler_pointwise.json")


def _load():
    with open(GOLD) as f:
        return json.load(f)


def test_hand_worked_states():
    g = _load()
    for st in g["states"]:
        q = np.array(st["Q"])
        assert abs(pressure(q, g["gamma"]) - st["p"]) < 1e-14
        assert abs(sound_speed(q, g["gamma"]) ** 2 - st["c2"]) < 1e-14
        for d in range(3):
            assert np.max(np.abs(flux(q, d, g["gamma"]) - np.array(st["F"][d]))) < 1e-14


def test_hand_worked_lf():
    g = _load()
    byname = {s["name"]: np.array(s["Q"]) for s in g["states"]}
    for ex in g["lf_examples"]:
        fs = lax_friedrichs(byname[ex["left"]], byname[ex["right"]], ex["d"], g["gamma"])
        assert np.max(np.abs(fs - np.array(ex["Fstar"]))) < 1e-14


def _random_states(rng, m):
    rho = rng.uniform(0.5, 2.0, m)
    u = rng.uniform(-1.5, 1.5, (3, m))
    p = rng.uniform(0.3, 3.0, m)
    en = p / 0.4 + 0.5 * rho * (u ** 2).sum(0)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2], en])


@pytest.mark.parametrize("d", [0, 1, 2])
def test_lf_consistency_and_conservation(d):
    rng = np.random.default_rng(d)
    qa = _random_states(rng, 64)
    qb = _random_states(rng, 64)
    # consistency: F*(Q, Q) = F^d(Q)
    assert np.max(np.abs(lax_friedrichs(qa, qa, d, 1.4) - flux(qa, d, 1.4))) < 1e-14
    # conservation under reflection of axis d (M flips momentum d):
    # F*(QL, QR) = -M F*(M QR, M QL)
    M = np.ones((5, 1))
    M[1 + d] = -1.0
    lhs = lax_friedrichs(qa, qb, d, 1.4)
    rhs = -M * lax_friedrichs(M * qb, M * qa, d, 1.4)
    assert np.max(np.abs(lhs - rhs)) < 1e-13
