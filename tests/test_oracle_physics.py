"""Physics pins of the oracle's whole time step: Taylor-Green decay against
the Navier-Stokes solution with nu = cs^2 (tau - 1/2) (Sec. 2.1), channel
flow under a uniform immersed force (Sec. 2.2 forced rule), exact mass
conservation of the coupled step, and translation invariance of the
falling-frame window (Sec. 2.5)."""
import math

import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W

CS2 = 1.0 / 3.0


def tgv_viscosity(orc, N, tau, U0=0.01, t1=20):
    """Decay rate of a 2-D Taylor-Green vortex, u ~ exp(-2 nu k^2 t), on an
    N x N periodic box (one cell deep), returned as a viscosity."""
    xi, _ = orc.lattice()
    k = 2 * math.pi / N
    nu = (tau - 0.5) / 3
    t2 = t1 + int(0.5 / (2 * nu * k * k))
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ux = U0 * np.sin(k * x) * np.cos(k * y)
    uy = -U0 * np.cos(k * x) * np.sin(k * y)
    p = -U0 ** 2 / 4 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    f = np.zeros((1, N, N, 27))
    for j in range(N):
        for i in range(N):
            f[0, j, i] = orc.feq(p[j, i], [ux[j, i], uy[j, i], 0.0])
    E = {}
    for s in range(t2 + 1):
        if s in (t1, t2):
            u = (f @ xi[:, :2].astype(float)) / f.sum(-1)[..., None]
            E[s] = (u ** 2).sum()
        f = orc.stream_grid(orc.collide_grid(f, tau))
    return math.log(E[t1] / E[t2]) / (t2 - t1) / (4 * k * k), nu


def test_taylor_green_decay_second_order(orc):
    r16, nu = tgv_viscosity(orc, 16, 0.8)
    r32, _ = tgv_viscosity(orc, 32, 0.8)
    e16, e32 = abs(r16 / nu - 1), abs(r32 / nu - 1)
    assert e16 < 2e-3 and e32 < 5e-4
    assert e16 / e32 > 3.0          # second-order convergence


@pytest.mark.parametrize("tau", [0.6, 0.8])
def test_channel_flow_under_uniform_immersed_force(orc, tau):
    """Steady flow between no-slip walls driven by a uniform h.  The forced
    rule evaluates f^(0) at u + tau h while f^(1) carries no momentum, so each
    step injects tau rho h: the profile is a parabola of curvature -tau h / nu
    (a reading of Sec. 2.2; with h alone the curvature would be off by tau).
    The wall slip of the halfway bounce-back shows up as a uniform offset."""
    xi, w = orc.lattice()
    nz, g = 16, 1e-6
    nu = (tau - 0.5) / 3
    f = np.tile(w, (nz, 1, 1, 1))
    H = np.zeros((nz, 1, 1, 3))
    H[..., 0] = g
    steps = int(25 * nz * nz / (math.pi ** 2 * nu))
    for _ in range(steps):
        f = orc.stream_grid(orc.collide_grid(f, tau, 0, H), 2, 2)
    u = ((f @ xi[:, 0]) / f.sum(-1)).ravel()
    curv = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.allclose(curv, -tau * g / nu, rtol=1e-7)
    z = np.arange(nz)
    par = tau * g / (2 * nu) * (z + 0.5) * (nz - 0.5 - z)
    off = u - par
    assert np.ptp(off) < 1e-7 * par.max()
    assert abs(off.mean()) < 3 * g


@pytest.mark.parametrize("tau", [0.6, 0.8])
def test_channel_flow_momentum_exact_variant(orc, tau):
    """With the momentum-exact variant a uniform h is a body force of density
    rho h per step: the steady profile is the plane Poiseuille parabola of
    curvature -h / nu, whatever tau."""
    xi, w = orc.lattice()
    nz, g = 16, 1e-6
    nu = (tau - 0.5) / 3
    f = np.tile(w, (nz, 1, 1, 1))
    H = np.zeros((nz, 1, 1, 3))
    H[..., 0] = g
    steps = int(25 * nz * nz / (math.pi ** 2 * nu))
    for _ in range(steps):
        f = orc.stream_grid(orc.collide_grid(f, tau, 0, H, forcing=1), 2, 2)
    u = ((f @ xi[:, 0]) / f.sum(-1)).ravel()
    curv = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.allclose(curv, -g / nu, rtol=1e-7)


@pytest.mark.parametrize("offset", [0.0, 3.0])
def test_stress_integral_of_linear_pressure_is_enclosed_volume(orc, offset):
    """A fluid at rest with density linear in z has sigma = -p I, p = cs^2
    (rho - 1), up to O(alpha^2) after one stream.  By the divergence theorem
    the stress integral over a closed surface is then -grad p times the
    enclosed volume: 4/3 pi R^3 at the markers, 4/3 pi (R + delta)^3 on the
    parallel surface of the force-surface variant; the torque vanishes."""
    _, w = orc.lattice()
    n, nz, R, alpha = 32, 40, 5.0, 1e-6
    zc = (nz - 1) / 2
    case = W.make_case(n, n, nz, 0.8, W.BC_FREESLIP, W.BC_FREESLIP, 0, 0.0)
    body = W.sphere_fibonacci_body(R, 2000, 2.0, [(n - 1) / 2, (n - 1) / 2, zc], force_offset=offset)
    o = orc.OracleSim(case, body)
    rho = 1.0 + alpha * (np.arange(nz) - zc)
    o.set_populations(np.broadcast_to(rho[:, None, None, None] * w, (nz, n, n, 27)))
    o.step(1)
    st = o.body_state()
    expect = -CS2 * alpha * 4.0 / 3.0 * math.pi * (R + offset) ** 3
    assert abs(st["F"][2] - expect) < 2e-3 * abs(expect)
    assert np.max(np.abs(st["F"][:2])) < 1e-3 * abs(expect)
    assert np.max(np.abs(st["T"])) < 1e-3 * abs(expect) * R
    assert abs(st["F_pressure"][2] - expect) < 2e-3 * abs(expect)


@pytest.mark.parametrize("forcing", [0, 1])
def test_pressure_top_hydrostatic_column(orc, forcing):
    """Constant-pressure top (density 1 on the halfway plane above the top
    row) over a no-slip bottom, uniform downward h: the steady column is
    hydrostatic, rho - 1 = 3 a (nz - 1/2 - z) with a = tau g for the forced
    rule as printed (each step adds tau rho h) and a = g for the
    momentum-exact variant."""
    xi, w = orc.lattice()
    nz, tau, g = 12, 0.8, 1e-5
    f = np.tile(w, (nz, 1, 1, 1))
    H = np.zeros((nz, 1, 1, 3))
    H[..., 2] = -g
    for _ in range(6000):
        f = orc.stream_grid(orc.collide_grid(f, tau, 0, H, forcing=forcing), orc.BC_NOSLIP, orc.BC_PRESSURE)
    rho = f.sum(-1).ravel()
    a = tau * g if forcing == 0 else g
    expect = 3 * a * (nz - 0.5 - np.arange(nz))
    assert np.max(np.abs((rho - 1) - expect)) < 1e-3 * expect.max()


def test_pressure_top_drains_to_unit_density(orc):
    """A closed column at rest with density 1.01 and a constant-pressure top
    loses its excess mass through the top: the density relaxes to 1
    everywhere (with walls on both ends the mass would stay)."""
    xi, w = orc.lattice()
    nz, tau = 12, 0.8
    f = np.tile(1.01 * w, (nz, 1, 1, 1))
    m0 = f.sum() - nz
    for _ in range(8000):
        f = orc.stream_grid(orc.collide_grid(f, tau, 0), orc.BC_NOSLIP, orc.BC_PRESSURE)
    assert np.max(np.abs(f.sum(-1) - 1.0)) < 1e-4 * m0 / nz
    g = np.tile(1.01 * w, (nz, 1, 1, 1))
    for _ in range(200):
        g = orc.stream_grid(orc.collide_grid(g, tau, 0), orc.BC_NOSLIP, orc.BC_NOSLIP)
    assert abs(g.sum() - nz - m0) < 1e-12


def small_case(nz=32, h_end=0.0, bc=W.BC_FREESLIP, markers=200, R=3.0, zc=None, gravity=1e-5, sponge=0):
    n = 20
    zc = (nz - 1) / 2 if zc is None else zc
    case = W.make_case(n, n, nz, 0.7, bc, bc, sponge, gravity, h_ini=zc, h_end=h_end)
    body = W.sphere_fibonacci_body(R, markers, 2.0, [(n - 1) / 2, (n - 1) / 2, zc])
    return case, body


def test_coupled_step_conserves_mass(orc):
    case, body = small_case()
    s = orc.OracleSim(case, body)
    m0 = s.populations().sum()
    s.step(12)
    assert abs(s.populations().sum() - m0) < 1e-9
    st = s.body_state()
    assert st["v"][2] < 0 and st["F"][2] > 0          # falling, fluid pushes back


def test_window_shift_is_a_translation(orc):
    """With z periodic and the top slabs still exactly at rest, the re-injected
    run equals the plain run rolled up by Delta, and the body is Delta higher."""
    zc = 12.0
    caseA, body = small_case(nz=48, h_end=zc - 1e-6, bc=W.BC_PERIODIC, zc=zc, gravity=4e-5)
    caseA["h_ini"] = zc + 8.0          # Delta = 8
    caseB, _ = small_case(nz=48, h_end=0.0, bc=W.BC_PERIODIC, zc=zc, gravity=4e-5)
    A = orc.OracleSim(caseA, body)
    B = orc.OracleSim(caseB, body)
    A.step(6)
    B.step(6)
    assert A.body_state()["shifts"] == 1
    assert B.body_state()["shifts"] == 0
    dz = 8
    CA, CB = A.post_collision(), B.post_collision()
    assert np.allclose(CA, np.roll(CB, dz, axis=0), rtol=0, atol=1e-14)
    A.step(4)
    B.step(4)
    CA, CB = A.post_collision(), B.post_collision()
    assert np.allclose(CA, np.roll(CB, dz, axis=0), rtol=0, atol=1e-13)
    sa, sb = A.body_state(), B.body_state()
    assert np.allclose(sa["r"], sb["r"] + np.array([0, 0, dz]), atol=1e-12)
    assert np.allclose(sa["F"], sb["F"], rtol=1e-9, atol=1e-16)
    assert np.allclose(sa["T"], sb["T"], rtol=1e-6, atol=1e-15)


def test_window_shift_resets_bottom_and_keeps_content(orc):
    case, body = small_case(nz=40, h_end=19.5 - 1e-6, zc=19.5)
    case["h_ini"] = 25.5                       # Delta = 6
    s = orc.OracleSim(case, body)
    s.step(1)
    before_f = s.populations()
    before_h = s.immersed_force()
    assert s.body_state()["pending_shift"] == 6
    C = s.post_collision()
    _, w = orc.lattice()
    assert np.array_equal(C[:6], np.broadcast_to(w, C[:6].shape))
    ref = np.zeros_like(before_f)
    for z in range(40):
        for y in range(20):
            for x in range(20):
                ref[z, y, x] = orc.collide_cell(before_f[z, y, x], before_h[z, y, x], 0.7)
    assert np.allclose(C[6:], ref[:-6], rtol=0, atol=1e-16)


def test_spin_down_of_rotating_sphere(orc):
    """A sphere spinning in quiescent fluid must be slowed by the fluid
    (torque opposite to w): this pins the orientation of the torque sum,
    T = sum dS (X_k - C_m) x (sigma n)."""
    case, body = small_case(gravity=0.0, markers=300, R=4.0)
    body["w0"] = np.array([0.0, 0.0, 2e-3])
    s = orc.OracleSim(case, body)
    s.step(10)
    st = s.body_state()
    assert st["T"][2] < 0
    assert st["w"][2] < 2e-3
