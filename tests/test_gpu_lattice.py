"""GPU parity of the fused stream + recursive-regularized collision kernel
against the FP64 oracle (Sec. 2.1, App. A), element by element, in FP32
storage: relative error on f below 1e-5 after one and after many steps, on
ragged boxes spanning several tiles, with periodic, free-slip and no-slip z
walls and a sponge."""
import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W
from tests.gpu_util import max_rel, oracle_to_soa, say

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2408_15115_amd import turret
    return turret


CASES = [
    # nx, ny, nz, tau, bc, sponge
    (8, 9, 10, 0.6, W.BC_PERIODIC, 0),
    (16, 12, 11, 0.8, W.BC_FREESLIP, 0),
    (12, 10, 14, 0.55, W.BC_NOSLIP, 0),
    (64, 8, 9, 1.3, W.BC_FREESLIP, 4),
    (33, 17, 19, 0.51, W.BC_NOSLIP, 6),
    # the paper's domain: no-slip bottom, constant-pressure top, sponge
    (20, 12, 16, 0.7, (W.BC_NOSLIP, W.BC_PRESSURE), 5),
    (12, 9, 13, 0.9, (W.BC_PRESSURE, W.BC_FREESLIP), 0),
]


def run_pair(T, orc, nx, ny, nz, tau, bc, sponge, steps, seed, storage="f32", amp=0.05, collision=0,
             u_wall=(0.0, 0.0)):
    lo, hi = bc if isinstance(bc, tuple) else (bc, bc)
    case = W.make_case(nx, ny, nz, tau, lo, hi, sponge, u_wall=u_wall)
    f0 = W.random_populations(seed, nx, ny, nz, amp=amp)
    say(f"lattice parity nx={nx} ny={ny} nz={nz} tau={tau} bc={bc} sponge={sponge} steps={steps} {storage} "
        f"collision={collision}")
    S = T.Solver([case], storage=storage, collision=collision)
    S.set_populations(oracle_to_soa(f0))
    for _ in range(steps):
        S.lbm_step()
    gpu = S.populations()
    # the library keeps post-collision states: its input is C_0, so the
    # oracle streams it first, then alternates collide/stream
    f = orc.stream_grid(f0, lo, hi, u_wall)
    for s in range(steps):
        C = orc.collide_grid(f, tau, sponge, collision=collision)
        if s + 1 < steps:
            f = orc.stream_grid(C, lo, hi, u_wall)
    S.close()
    return gpu, oracle_to_soa(C)


@pytest.mark.parametrize("nx,ny,nz,tau,bc,sponge", CASES)
def test_one_step_matches_oracle(T, orc, nx, ny, nz, tau, bc, sponge):
    gpu, ref = run_pair(T, orc, nx, ny, nz, tau, bc, sponge, 1, seed=nx * 7 + nz)
    assert max_rel(gpu, ref) < TOL_F32


@pytest.mark.parametrize("nx,ny,nz,tau,bc,sponge", CASES[1:4] + CASES[5:6])
def test_many_steps_match_oracle(T, orc, nx, ny, nz, tau, bc, sponge):
    gpu, ref = run_pair(T, orc, nx, ny, nz, tau, bc, sponge, 25, seed=nx + ny, amp=0.02)
    assert max_rel(gpu, ref) < TOL_F32


@pytest.mark.parametrize("nx,ny,nz,tau,bc,sponge,steps", [(16, 12, 11, 0.8, W.BC_FREESLIP, 0, 1),
                                                          (20, 12, 16, 0.7, (W.BC_NOSLIP, W.BC_PRESSURE), 5, 20)])
def test_bgk_comparison_collision_matches_oracle(T, orc, nx, ny, nz, tau, bc, sponge, steps):
    gpu, ref = run_pair(T, orc, nx, ny, nz, tau, bc, sponge, steps, seed=5 + nx, amp=0.02, collision=1)
    assert max_rel(gpu, ref) < TOL_F32
    rr, _ = run_pair(T, orc, nx, ny, nz, tau, bc, sponge, steps, seed=5 + nx, amp=0.02)
    assert max_rel(gpu, rr) > 1e-6


@pytest.mark.parametrize("lo,hi", [(W.BC_FREESLIP, W.BC_FREESLIP), (W.BC_NOSLIP, W.BC_PRESSURE)])
def test_rest_state_stays_exactly_at_rest(T, lo, hi):
    case = W.make_case(16, 16, 16, 0.6, lo, hi, 5)
    S = T.Solver([case])
    S.run(10)
    f = S.populations()
    assert np.array_equal(f, np.broadcast_to(W.D3Q27_W[:, None, None, None], f.shape))


def test_mass_is_conserved(T):
    nx, ny, nz = 24, 20, 18
    for bc in (W.BC_PERIODIC, W.BC_FREESLIP, W.BC_NOSLIP):
        case = W.make_case(nx, ny, nz, 0.7, bc, bc, 0)
        f0 = W.random_populations(3, nx, ny, nz, amp=0.05)
        S = T.Solver([case])
        S.set_populations(oracle_to_soa(f0))
        m0 = S.populations().sum()
        for _ in range(30):
            S.lbm_step()
        assert abs(S.populations().sum() - m0) / m0 < 1e-6
        S.close()


@pytest.mark.parametrize("block,schedule", [(64, 0), (128, 1), (256, 2)])
def test_schedules_are_bitwise_identical(T, block, schedule):
    nx, ny, nz = 40, 24, 20
    case = W.make_case(nx, ny, nz, 0.6, W.BC_FREESLIP, W.BC_FREESLIP, 3)
    f0 = oracle_to_soa(W.random_populations(5, nx, ny, nz))
    outs = []
    for blk, sch in ((256, 0), (block, schedule)):
        S = T.Solver([case], block=blk, schedule=sch, persist_wgs=37)
        S.set_populations(f0)
        for _ in range(3):
            S.lbm_step()
        outs.append(S.populations())
        S.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("steps,storage,tol", [(1, "f32", TOL_F32), (20, "f32", TOL_F32), (20, "f16", 2e-3)])
def test_moving_walls_match_oracle(T, orc, steps, storage, tol):
    """No-slip walls moving in x (the shear flow of the rotation case)."""
    gpu, ref = run_pair(T, orc, 16, 12, 11, 0.7, W.BC_NOSLIP, 0, steps, seed=13, amp=0.02, storage=storage,
                        u_wall=(-0.03, 0.05))
    assert max_rel(gpu, ref) < tol
