"""Pins of the D3Q19 comparison lattice of the oracle (oracle/orc19.c)
against what the lattice and the Hermite construction fix: isotropy of the
weights, the equilibrium's moments (exact to second order; the supported
third moments; the lattice's own aliasing of xi_x^3 to xi_x), the moments of
the regularized non-equilibrium part (second moment P1, the recursion at
third order), conservation through a collision, the rest state as a fixed
point, and the Taylor-Green decay rate against nu = cs^2 (tau - 1/2) for both
collision models."""
import math

import numpy as np
import pytest

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def lat(orc):
    return orc.lattice19()


def moments(xi, f):
    x = xi.astype(float)
    return f.sum(), x.T @ f, np.einsum("ia,ib,i->ab", x, x, f)


def test_lattice_isotropy(lat):
    xi, w = lat
    x = xi.astype(float)
    assert len({tuple(v) for v in xi}) == 19 and (np.abs(xi).sum(1) <= 2).all()
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(x.T @ w, 0, atol=1e-16)
    assert np.allclose(np.einsum("ia,ib,i->ab", x, x, w), CS2 * np.eye(3), atol=1e-16)
    assert np.einsum("i,i->", w, x[:, 0] ** 4) == pytest.approx(3 * CS2 ** 2, abs=1e-16)
    assert np.einsum("i,i->", w, x[:, 0] ** 2 * x[:, 1] ** 2) == pytest.approx(CS2 ** 2, abs=1e-16)


def test_equilibrium_moments(orc, lat):
    xi, _ = lat
    x = xi.astype(float)
    rho, u = 1.07, np.array([0.06, -0.04, 0.03])
    f0 = orc.feq19(rho, u)
    m0, m1, m2 = moments(xi, f0)
    assert m0 == pytest.approx(rho, abs=1e-15)
    assert np.allclose(m1, rho * u, atol=1e-16)
    assert np.allclose(m2, rho * (np.outer(u, u) + CS2 * np.eye(3)), atol=1e-16)
    # the third moments the lattice carries, on the orthogonal combinations
    # H_xxy +- H_yzz (H_abc = xi_a xi_b xi_c - cs^2 (...)): exact
    hxxy = x[:, 0] ** 2 * x[:, 1] - CS2 * x[:, 1]
    hyzz = x[:, 1] * x[:, 2] ** 2 - CS2 * x[:, 1]
    axxy, ayzz = rho * u[0] ** 2 * u[1], rho * u[1] * u[2] ** 2
    assert ((hxxy + hyzz) * f0).sum() == pytest.approx(axxy + ayzz, abs=1e-17)
    assert ((hxxy - hyzz) * f0).sum() == pytest.approx(axxy - ayzz, abs=1e-17)
    # one it cannot carry: xi_x^3 = xi_x on this lattice, so the moment is rho u_x
    assert (x[:, 0] ** 3 * f0).sum() == pytest.approx(rho * u[0], abs=1e-16)


def test_regularized_nonequilibrium_moments(orc, lat):
    xi, _ = lat
    x = xi.astype(float)
    rng = np.random.default_rng(19)
    A = rng.normal(size=(3, 3)) * 1e-3
    P1 = A + A.T
    u = np.array([0.05, 0.02, -0.03])
    f1 = orc.f1_19(P1, u)
    m0, m1, m2 = moments(xi, f1)
    assert abs(m0) < 1e-17 and np.allclose(m1, 0, atol=1e-17)
    assert np.allclose(m2, P1, atol=1e-17)
    # third order from the recursion: a1_xxy = 2 P1_xy u_x + P1_xx u_y,
    # a1_yzz = 2 P1_yz u_z + P1_zz u_y, on the combinations
    hxxy = x[:, 0] ** 2 * x[:, 1] - CS2 * x[:, 1]
    hyzz = x[:, 1] * x[:, 2] ** 2 - CS2 * x[:, 1]
    axxy = 2 * P1[0, 1] * u[0] + P1[0, 0] * u[1]
    ayzz = 2 * P1[1, 2] * u[2] + P1[2, 2] * u[1]
    assert ((hxxy + hyzz) * f1).sum() == pytest.approx(axxy + ayzz, abs=1e-18)
    assert ((hxxy - hyzz) * f1).sum() == pytest.approx(axxy - ayzz, abs=1e-18)


@pytest.mark.parametrize("collision", [0, 1])
def test_collision_conserves_and_relaxes_the_stress(orc, lat, collision):
    xi, w = lat
    rng = np.random.default_rng(7 + collision)
    rho, u = 1.02, np.array([0.03, -0.05, 0.04])
    f = orc.feq19(rho, u) + 1e-3 * w * rng.normal(size=19)
    tau = 0.63
    C = orc.collide19(f, tau, collision)
    r0, j0, _ = moments(xi, f)
    r1, j1, m2 = moments(xi, C)
    assert r1 == pytest.approx(r0, abs=1e-15) and np.allclose(j1, j0, atol=1e-16)
    uu = j0 / r0
    Pf = moments(xi, f)[2]
    P1 = Pf - r0 * (np.outer(uu, uu) + CS2 * np.eye(3))
    assert np.allclose(m2, r0 * (np.outer(uu, uu) + CS2 * np.eye(3)) + (1 - 1 / tau) * P1, atol=1e-15)


def test_rest_state_is_a_fixed_point(orc, lat):
    _, w = lat
    f = np.broadcast_to(w, (4, 5, 6, 19)).copy()
    for collision in (0, 1):
        g = orc.run19(f, 0.55, 5, collision)
        assert np.abs(g - f).max() < 1e-15


def tgv_viscosity19(orc, N, tau, collision, U0=0.01, t1=20):
    """Decay rate of a 2-D Taylor-Green vortex in an N x N x 1 periodic box,
    u ~ exp(-2 nu k^2 t), returned as a viscosity."""
    xi, _ = orc.lattice19()
    k = 2 * math.pi / N
    nu = CS2 * (tau - 0.5)
    t2 = t1 + int(0.5 / (2 * nu * k * k))
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ux = U0 * np.sin(k * x) * np.cos(k * y)
    uy = -U0 * np.cos(k * x) * np.sin(k * y)
    p = -U0 ** 2 / 4 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    f = np.zeros((1, N, N, 19))
    for j in range(N):
        for i in range(N):
            f[0, j, i] = orc.feq19(1.0 + p[j, i] / CS2, [ux[j, i], uy[j, i], 0.0])

    def amp(g):
        rho = g.sum(-1)
        jx = (g * xi[:, 0]).sum(-1) / rho
        return np.abs(np.fft.fft2(jx[0])[1, 1])

    g1 = orc.run19(f, tau, t1, collision)
    g2 = orc.run19(g1, tau, t2 - t1, collision)
    return -math.log(amp(g2) / amp(g1)) / (t2 - t1) / (2 * k * k)


@pytest.mark.parametrize("collision", [0, 1])
def test_taylor_green_viscosity(orc, collision):
    tau = 0.8
    nu = CS2 * (tau - 0.5)
    e32 = abs(tgv_viscosity19(orc, 32, tau, collision) / nu - 1)
    e64 = abs(tgv_viscosity19(orc, 64, tau, collision) / nu - 1)
    assert e64 < 2e-3
    assert e64 < e32 / 2.5       # second order in space


def test_streaming_moves_each_population_along_its_velocity(orc, lat):
    xi, _ = lat
    nz, ny, nx = 5, 6, 7
    f = np.zeros((nz, ny, nx, 19))
    z, y, x = 0, 5, 3
    f[z, y, x, :] = 1.0 + np.arange(19)
    g = orc.stream19(f)
    assert g.sum() == pytest.approx(f.sum())
    for i in range(19):
        t = ((z + xi[i, 2]) % nz, (y + xi[i, 1]) % ny, (x + xi[i, 0]) % nx)
        assert g[t + (i,)] == 1.0 + i


def test_grid_step_is_collide_then_stream(orc, lat):
    _, w = lat
    rng = np.random.default_rng(3)
    f = w * (1.0 + 0.02 * rng.normal(size=(4, 5, 6, 19)))
    for collision in (0, 1):
        g = orc.stream19(orc.collide_grid19(f, 0.7, collision))
        assert np.array_equal(g, orc.run19(f, 0.7, 1, collision))
        assert np.array_equal(orc.collide_grid19(f, 0.7, collision)[2, 3, 1], orc.collide19(f[2, 3, 1], 0.7, collision))
