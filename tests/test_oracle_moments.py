"""Pins of moment storage's premise against the oracle (App. A, Sec. 2.2): a
regularized post-collision state is fully determined by ten of its own
moments -- rho, rho u and the off-equilibrium stress Q = Pi(C) - Pi(f0(p, u))
-- through f0(p, u) + f1(Q, u), since f1 is linear in its stress.  A forced
cell adds only the equilibrium shift: C_h = f0(p, u + tau h) + f1(Q, u), and
in the momentum-exact variant less w_i xi_i . (tau - 1) rho h / cs^2.  All
from the oracle's own collision, to rounding."""
import numpy as np
import pytest

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def lat(orc):
    xi, w = orc.lattice()
    return xi.astype(float), w


def moments(x, f):
    rho = f.sum()
    j = x.T @ f
    Pi = np.einsum("ia,ib,i->ab", x, x, f)
    return rho, j, Pi


def cells(w, n=40, seed=27):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield w * (1.0 + 0.05 * rng.normal(size=27)), 0.55 + 0.9 * rng.random(), rng.normal(size=3) * 1e-3


def test_collided_state_is_rebuilt_from_ten_moments(orc, lat):
    x, w = lat
    worst = 0.0
    for f, tau, _ in cells(w):
        C = orc.collide_cell(f, None, tau)
        rho, j, Pi = moments(x, C)
        u = j / rho
        p = CS2 * (rho - 1.0)
        Q = Pi - moments(x, orc.feq(p, u))[2]
        R = orc.feq(p, u) + orc.fneq(Q, u)
        worst = max(worst, np.abs(R - C).max())
        # the collision keeps mass and momentum: the same rho, u as f
        r0, j0, _ = moments(x, f)
        assert rho == pytest.approx(r0, abs=1e-14) and np.allclose(j, j0, atol=1e-15)
    assert worst < 1e-15


@pytest.mark.parametrize("forcing", [0, 1])
def test_forced_state_is_the_moments_plus_the_equilibrium_shift(orc, lat, forcing):
    x, w = lat
    worst = 0.0
    for f, tau, h in cells(w, seed=28 + forcing):
        C = orc.collide_cell(f, None, tau)
        Ch = orc.collide_cell(f, h, tau, forcing=forcing)
        rho, j, Pi = moments(x, C)
        u = j / rho
        p = CS2 * (rho - 1.0)
        Q = Pi - moments(x, orc.feq(p, u))[2]
        R = orc.feq(p, u + tau * h) + orc.fneq(Q, u)
        if forcing == 1:
            R -= w * (x @ ((tau - 1.0) * rho * h)) / CS2
        worst = max(worst, np.abs(R - Ch).max())
        assert np.abs(Ch - C).max() > 1e-6   # the force does change the state
    assert worst < 1e-15
