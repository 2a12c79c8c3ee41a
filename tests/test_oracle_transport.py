"""Pins of the oracle's streaming, weight function, interpolation and
spreading (Sec. 2.1 evolution rule, Sec. 2.2) against library routines and
the defining properties of Peskin's four-point kernel."""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_grid(rng, shape, nc):
    return rng.standard_normal(shape + (nc,))


def test_periodic_stream_is_numpy_roll(orc):
    """f_i(x) = C_i(x - xi_i) on a periodic box equals np.roll by +xi_i."""
    rng = np.random.default_rng(1)
    xi, _ = orc.lattice()
    C = rand_grid(rng, (5, 6, 7), 27)
    f = orc.stream_grid(C)
    for i in range(27):
        ref = np.roll(C[..., i], shift=(xi[i, 2], xi[i, 1], xi[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(f[..., i], ref)


def ghost_stream(C, xi, mode):
    """Reference: pad one ghost slab below and above in z, filled by the wall
    rule, then pull with np.roll; freeslip ghosts mirror xi_z, noslip ghosts
    hold the reversed population of the wall cell."""
    nz, ny, nx, _ = C.shape
    f = np.empty_like(C)
    for i in range(27):
        ex, ey, ez = xi[i]
        G = np.zeros((nz + 2, ny, nx))
        G[1:-1] = C[..., i]
        if mode == "freeslip":
            im = 9 * (-ez + 1) + 3 * (ey + 1) + (ex + 1)
            G[0] = C[0, ..., im]
            G[-1] = C[-1, ..., im]
        else:
            # a ghost at x - xi must deliver C_opp(i)(x): shift the wall slab by -xi in x,y
            G[0] = np.roll(C[0, ..., 26 - i], shift=(-ey, -ex), axis=(0, 1))
            G[-1] = np.roll(C[-1, ..., 26 - i], shift=(-ey, -ex), axis=(0, 1))
        R = np.roll(G, shift=(ez, ey, ex), axis=(0, 1, 2))
        f[..., i] = R[1:-1]
    return f


@pytest.mark.parametrize("mode,bc", [("freeslip", 1), ("noslip", 2)])
def test_wall_stream_matches_ghost_construction(orc, mode, bc):
    rng = np.random.default_rng(2)
    xi, _ = orc.lattice()
    C = rand_grid(rng, (6, 5, 4), 27)
    f = orc.stream_grid(C, bc, bc)
    assert np.array_equal(f, ghost_stream(C, xi, mode))


@pytest.mark.parametrize("bc", [1, 2])
def test_wall_stream_conserves_mass(orc, bc):
    rng = np.random.default_rng(3)
    C = rand_grid(rng, (6, 5, 4), 27)
    f = orc.stream_grid(C, bc, bc)
    assert abs(f.sum() - C.sum()) < 1e-10


def test_freeslip_reverses_only_normal_momentum_at_walls(orc):
    """Specular walls keep the tangential momentum of the whole box."""
    rng = np.random.default_rng(4)
    xi, _ = orc.lattice()
    C = rand_grid(rng, (6, 5, 4), 27)
    f = orc.stream_grid(C, 1, 1)
    assert np.allclose((f @ xi[:, :2]).sum((0, 1, 2)), (C @ xi[:, :2]).sum((0, 1, 2)))


def test_weight_function_golden(orc):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "peskin4_kernel.txt")) if l[0] != "#"]
    for r, v in rows:
        assert abs(orc.phi(float(r)) - float(v)) < 1e-15


@pytest.mark.parametrize("r", np.linspace(0.0, 1.0, 41))
def test_weight_function_moment_conditions(orc, r):
    """Peskin's four-point kernel is defined by: partition of unity, zero
    first moment, even and odd node sums of 1/2 each, and sum of squares 3/8."""
    js = np.arange(-3, 5)
    ph = np.array([orc.phi(r - j) for j in js])
    assert abs(ph.sum() - 1) < 1e-15
    assert abs(((r - js) * ph).sum()) < 1e-15
    assert abs(ph[js % 2 == 0].sum() - 0.5) < 1e-15
    assert abs((ph ** 2).sum() - 3.0 / 8.0) < 1e-15
    assert (ph >= 0).all()


def test_interpolation_exact_for_linear_fields(orc):
    rng = np.random.default_rng(5)
    nz, ny, nx = 10, 12, 14
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a = rng.standard_normal(4)
    field = (a[0] + a[1] * x + a[2] * y + a[3] * z)[..., None]
    X = np.column_stack([rng.uniform(3, nx - 4, 50), rng.uniform(3, ny - 4, 50), rng.uniform(2, nz - 3, 50)])
    out = orc.interp(field, X)[:, 0]
    assert np.allclose(out, a[0] + X @ a[1:], atol=1e-12)


def test_spread_conserves_force_and_moment_and_is_adjoint(orc):
    rng = np.random.default_rng(6)
    shape = (10, 11, 12)
    nz, ny, nx = shape
    M = 40
    X = np.column_stack([rng.uniform(3, nx - 4, M), rng.uniform(3, ny - 4, M), rng.uniform(2, nz - 3, M)])
    h = rng.standard_normal((M, 3))
    dS = rng.uniform(0.3, 0.7, M)
    H = orc.spread(shape, X, h, dS)
    assert np.allclose(H.sum((0, 1, 2)), (h * dS[:, None]).sum(0), atol=1e-13)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x, y, z], -1).astype(float)
    torque_grid = np.cross(pos, H).sum((0, 1, 2))
    torque_mark = np.cross(X, h * dS[:, None]).sum(0)
    assert np.allclose(torque_grid, torque_mark, atol=1e-11)
    u = rng.standard_normal(shape + (3,))
    lhs = (orc.interp(u, X) * h * dS[:, None]).sum()
    rhs = (u * H).sum()
    assert abs(lhs - rhs) < 1e-12


def test_stencil_wraps_laterally_and_refuses_vertical_exit(orc):
    rng = np.random.default_rng(7)
    shape = (8, 8, 8)
    u = rng.standard_normal(shape + (3,))
    X = np.array([[0.3, 7.6, 4.0]])
    # wrap-around equals interpolation in a rolled field
    ref = orc.interp(np.roll(u, shift=(0, -4, 4), axis=(0, 1, 2)), X + np.array([[4.0, -4.0, 0.0]]))
    assert np.allclose(orc.interp(u, X), ref, atol=1e-14)
    with pytest.raises(ValueError):
        orc.interp(u, np.array([[4.0, 4.0, 0.5]]))


@pytest.mark.parametrize("nz,sponge,tau0", [(40, 8, 0.55), (768, 61, 0.53048), (64, 2, 2.0)])
def test_sponge_profile(orc, nz, sponge, tau0):
    """Sec. 2.5: tau rises linearly inside the top zone to reach 1 on the top
    boundary; below the zone it is tau0 (continuous at the zone start)."""
    taus = np.array([orc.tau_at(nz, tau0, sponge, z) for z in range(nz)])
    zs = nz - sponge
    assert np.all(taus[: zs + 1] == tau0)
    assert abs(taus[-1] - 1.0) < 1e-15
    assert np.allclose(np.diff(taus[zs:], 2), 0, atol=1e-15)


def test_collision_grid_uses_sponge(orc):
    rng = np.random.default_rng(8)
    _, w = orc.lattice()
    f = w * (1 + 0.03 * rng.standard_normal((12, 3, 3, 27)))
    C = orc.collide_grid(f, 0.6, 5)
    for z in range(12):
        tau = orc.tau_at(12, 0.6, 5, z)
        assert np.allclose(C[z, 1, 2], orc.collide_cell(f[z, 1, 2], None, tau), atol=1e-16)
