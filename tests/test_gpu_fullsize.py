"""Parity at the full size of the scale workload (256 x 256 x 768, the
benchmark's configuration and launch schedule).

1. Lattice kernel, one step from an analytic initial state written straight
   into the FP32 population buffer: sampled cells (random interior cells and
   cells of the top and bottom wall rows) against the oracle's collision of
   the pulled populations, computed cell by cell.
2. The coupled step: the lattice Boltzmann update is local (a population
   moves one cell per step), so after n steps from rest everything within a
   box of margin > n cells around the particle's region is identical in any
   domain that contains that box.  The oracle runs the same body on such a
   crop; force, torque, body state and the populations near the body must
   match the full-size GPU run."""
import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W
from tests.gpu_util import max_rel, oracle_to_soa, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2408_15115_amd import turret
    return turret


def analytic_deviation(i, x, y, z, nx, ny, nz, w):
    """g_i = 0.01 w_i (cos(kx x + a_i) + cos(ky y + b_i) + cos(kz z + c_i)),
    evaluated at integer coordinates (broadcastable arrays)."""
    a, b, c = 0.7 * i, 1.3 * i + 0.2, 0.4 * i - 1.0
    return w[i] * 0.01 * (np.cos(2 * np.pi * 3 * x / nx + a) + np.cos(2 * np.pi * 2 * y / ny + b) +
                          np.cos(2 * np.pi * 5 * z / nz + c))


def current_state(S, torch, nx, ny, nz):
    """FP32 deviations of the current buffer as a device view (27, nz, ny, nx);
    valid for one case whose ring origin is 0."""
    cur = S.bufs[0] if S.current_buffer() == S.bufs[0].data_ptr() else S.bufs[1]
    plane = S.plane_stride(0)
    return cur.view(torch.float32)[:27 * plane].view(27, plane)[:, :nx * ny * nz].view(27, nz, ny, nx)


def test_lattice_step_at_full_size_sampled(T, orc):
    import torch
    case, _ = W.case_ellipsoid_tall()
    nx, ny, nz = case["nx"], case["ny"], case["nz"]
    tau, sponge = case["tau"], case["sponge"]
    xi, w = orc.lattice()
    say("full-size lattice parity: writing the analytic state")
    S = T.Solver([case], None, stream=torch.cuda.Stream())
    plane = S.plane_stride(0)
    assert S.pop_offset(0) == 0 and plane >= nx * ny * nz
    pop = S.bufs[0] if S.current_buffer() == S.bufs[0].data_ptr() else S.bufs[1]
    view = pop.view(torch.float32)
    X = np.arange(nx, dtype=np.float64)[None, None, :]
    Y = np.arange(ny, dtype=np.float64)[None, :, None]
    Z = np.arange(nz, dtype=np.float64)[:, None, None]
    for i in range(27):
        g = analytic_deviation(i, X, Y, Z, nx, ny, nz, w).astype(np.float32)
        view[i * plane:i * plane + nx * ny * nz].copy_(torch.from_numpy(np.ascontiguousarray(g).ravel()))
    torch.cuda.synchronize()
    S.lbm_step()
    torch.cuda.synchronize()
    out = current_state(S, torch, nx, ny, nz)
    rng = np.random.default_rng(42)
    cells = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(600)]
    cells += [(int(rng.integers(nx)), int(rng.integers(ny)), z) for z in (0, nz - 1) for _ in range(100)]
    cells += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, nz - 2), (nx - 1, 0, 1)]
    cx = torch.tensor([c[0] for c in cells], device="cuda")
    cy = torch.tensor([c[1] for c in cells], device="cuda")
    cz = torch.tensor([c[2] for c in cells], device="cuda")
    got = out[:, cz, cy, cx].double().cpu().numpy().T + w   # (cells, 27)
    worst = 0.0
    for k, (x, y, z) in enumerate(cells):
        f_in = np.empty(27)
        for i in range(27):
            sx, sy, sz = (x - xi[i, 0]) % nx, (y - xi[i, 1]) % ny, z - xi[i, 2]
            j = i
            if sz < 0 or sz >= nz:      # free-slip: mirrored population of the lateral neighbour
                sz = z
                j = 9 * (-xi[i, 2] + 1) + 3 * (xi[i, 1] + 1) + (xi[i, 0] + 1)
            g = np.float32(analytic_deviation(j, np.float64(sx), np.float64(sy), np.float64(sz), nx, ny, nz, w))
            f_in[i] = w[j] + float(g)
        ref = orc.collide_cell(f_in, None, orc.tau_at(nz, tau, sponge, z))
        worst = max(worst, max_rel(got[k], ref))
    say(f"  sampled cells {len(cells)}: max rel err {worst:.3e}")
    assert worst < 1e-5
    S.close()


def test_coupled_steps_at_full_size_match_cropped_oracle(T, orc):
    import torch
    case, body = W.case_ellipsoid_tall()
    steps = 8
    say("full-size coupled parity: 256x256x768, 12252 markers")
    S = T.Solver([case], [body], stream=torch.cuda.Stream())
    S.run(steps)
    st = S.body_state()
    # crop: the region of the body plus a margin larger than the light cone
    rb = float(np.linalg.norm(body["x_body"], axis=1).max())
    half = int(np.ceil(rb)) + 4 + steps + 4
    r0 = np.asarray(body["r0"])
    lo = np.floor(r0).astype(int) - half
    n = 2 * half + 2
    crop = dict(case)
    crop.update(nx=n, ny=n, nz=n, bc_zlo=W.BC_PERIODIC, bc_zhi=W.BC_PERIODIC, sponge=0, h_ini=0.0, h_end=0.0)
    cb = dict(body)
    cb["r0"] = r0 - lo
    o = orc.OracleSim(crop, cb)
    o.step(steps)
    ost = o.body_state()
    Fs = np.linalg.norm(ost["F"])
    say(f"  |F| {Fs:.3e}; F err {np.max(np.abs(st['F'] - ost['F'])) / Fs:.3e}")
    assert np.max(np.abs(st["F"] - ost["F"])) < 1e-4 * Fs
    assert np.max(np.abs(st["T"] - ost["T"])) < 1e-4 * Fs * rb
    assert np.allclose(st["r"], ost["r"] + lo, atol=1e-10)
    assert np.allclose(st["v"], ost["v"], rtol=1e-6, atol=1e-14)
    # populations in the inner box (light cone of the body region) at full size
    inner = slice(steps + 2, n - steps - 2)
    ref = oracle_to_soa(o.post_collision())[:, inner, inner, inner]
    gz = slice(lo[2] + steps + 2, lo[2] + n - steps - 2)
    gy = slice(lo[1] + steps + 2, lo[1] + n - steps - 2)
    gx = slice(lo[0] + steps + 2, lo[0] + n - steps - 2)
    nx, ny, nz = case["nx"], case["ny"], case["nz"]
    _, w = orc.lattice()
    f = current_state(S, torch, nx, ny, nz)[:, gz, gy, gx].double().cpu().numpy() + w[:, None, None, None]
    assert st["z0"] == 0
    err = max_rel(f, ref)
    say(f"  populations near the body: max rel err {err:.3e}")
    assert err < 1e-5
    S.close()
