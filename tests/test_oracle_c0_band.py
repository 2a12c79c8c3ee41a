"""Plausibility band of the 48^3 sphere case (D = 8, kappa 2, g 1e-5,
tau 0.6; the plain method of Sec. 2 with the force read on the surface 3
cells out).  Not parity (that is GPU against the oracle): a check that the
oracle's coupled run lands where Stokes settling puts it.

Stokes speed of the sphere under the body acceleration g acting on its mass
kappa V against 6 pi nu R v:  v_S = (2/9) kappa R^2 g / nu = 2.13e-3.  In the
periodic array of the 48^3 box (solid fraction phi = V / 48^3 = 0.0024) the
drag is larger by Hasimoto's K(phi) = 1 / (1 - 1.7601 phi^(1/3) + phi -
1.5593 phi^2) = 1.31, so the terminal speed is v_S / K.  From rest the sphere
accelerates (monotonically over the first 200 steps) and stays below
v_S / K; after 2000 steps (about ten
viscous times R^2 / nu) the drag is within a few per cent of the weight."""
import math
import os

import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "sphere48_fp64_trajectory.txt")


def _band(case, body):
    R = 4.0
    nu = (case["tau"] - 0.5) / 3.0
    g = case["gravity"]
    kappa = body["kappa"]
    v_s = 2.0 / 9.0 * kappa * R * R * g / nu
    V = 4.0 / 3.0 * math.pi * R ** 3
    phi = V / (case["nx"] * case["ny"] * case["nz"])
    K = 1.0 / (1.0 - 1.7601 * phi ** (1.0 / 3.0) + phi - 1.5593 * phi * phi)
    return v_s, K, kappa * V * g


def test_stokes_band_numbers():
    case, body = W.case_sphere48()
    v_s, K, weight = _band(case, body)
    assert v_s == pytest.approx(2.13e-3, rel=2e-3)
    assert K == pytest.approx(1.31, abs=0.01)


@pytest.mark.slow
def test_first_200_steps_accelerate_inside_the_band(orc):
    case, body = W.case_sphere48()
    v_s, K, weight = _band(case, body)
    s = orc.OracleSim(case, body)
    v, F = [], []
    for _ in range(200):
        s.step(1)
        b = s.body_state()
        v.append(-b["v"][2])
        F.append(b["F"][2])
    v, F = np.array(v), np.array(F)
    assert np.all(np.diff(v) > 0)                 # falls faster every step
    assert 0.0 < v[-1] < v_s / K
    assert np.all(F[1:] > 0) and np.all(F < weight)   # the fluid holds the sphere back, less than its weight
    # the stored 2000-step run (the same oracle) continues it
    gold = np.loadtxt(GOLDEN)
    assert np.allclose(gold[:200, 12], -v, rtol=1e-12, atol=0)


def test_stored_run_approaches_the_terminal_state():
    case, body = W.case_sphere48()
    v_s, K, weight = _band(case, body)
    gold = np.loadtxt(GOLDEN)
    v, F = -gold[:, 12], gold[:, 3]
    # acoustic waves of the closed box ripple v_z by ~1e-4 relative after
    # ~500 steps; the mean over 200-step windows still grows
    means = [v[a:a + 200].mean() for a in (100, 500, 900, 1300, 1800)]
    assert np.all(np.diff(means) > 0) and v.max() < v_s / K
    assert 0.95 < F[-1] / weight < 1.0
    assert 0.6 < v[-1] / (v_s / K) < 1.0
