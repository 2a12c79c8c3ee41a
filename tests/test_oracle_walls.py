"""Pins of the oracle's moving no-slip wall (bounce-back plus the wall's
momentum, the shear flow of the rotation case of Sec. 3.1): plane Couette
flow between walls halfway outside the first and last rows, moving at -U and
+U, is exactly linear at steady state, u_x(z) = U (2 (z + 1/2) / nz - 1),
with uniform density, for both collision models and any tau; a resting wall
gives the plain bounce-back; and the wall term enters with the sign of the
wall's motion."""
import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W

XI = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)], float)


def couette(orc, nz, U, tau, collision, steps):
    g = np.broadcast_to(W.D3Q27_W, (nz, 3, 3, 27)).copy()
    for _ in range(steps):
        g = orc.stream_grid(orc.collide_grid(g, tau, 0, collision=collision), W.BC_NOSLIP, W.BC_NOSLIP, (-U, U))
    rho = g.sum(-1)
    return (g @ XI)[..., 0] / rho, rho


@pytest.mark.parametrize("tau,collision", [(0.6, 0), (0.6, 1), (1.4, 0)])
def test_couette_profile_is_exact(orc, tau, collision):
    nz, U = 12, 0.01
    ux, rho = couette(orc, nz, U, tau, collision, 14000 if tau < 1 else 4000)
    exact = U * (2 * (np.arange(nz) + 0.5) / nz - 1)
    assert np.abs(ux - exact[:, None, None]).max() < 1e-9 * U
    assert np.abs(rho - 1).max() < 1e-9


def test_resting_wall_is_plain_bounce_back(orc):
    rng = np.random.default_rng(4)
    C = W.D3Q27_W * (1 + 0.05 * rng.normal(size=(6, 3, 4, 27)))
    a = orc.stream_grid(C, W.BC_NOSLIP, W.BC_NOSLIP)
    b = orc.stream_grid(C, W.BC_NOSLIP, W.BC_NOSLIP, (0.0, 0.0))
    assert np.array_equal(a, b)
    # bottom row, direction (+1, 0, +1) comes back from (-1, 0, -1) of the same cell
    i, o = 9 * 2 + 3 * 1 + 2, 9 * 0 + 3 * 1 + 0
    assert a[0, 1, 2, i] == C[0, 1, 2, o]
    m = orc.stream_grid(C, W.BC_NOSLIP, W.BC_NOSLIP, (0.02, 0.0))
    assert m[0, 1, 2, i] - C[0, 1, 2, o] == pytest.approx(6 * W.D3Q27_W[i] * 0.02, rel=1e-12)
    assert np.array_equal(m[1:], a[1:])
