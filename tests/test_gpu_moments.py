"""GPU parity of the moment-storage form of the D3Q27 recursive-regularized
step (App. A: the collided state is a function of rho, u and P1 only)
against the FP64 oracle, element by element on the reconstructed
populations: FP32, boxes with ragged column tiles and several z chunks,
periodic or between free-slip, no-slip (resting or moving) and
constant-pressure walls, with and without a sponge, after one and after
many steps; the
round trip of a regularized state through the ten stored moments; agreement
with population storage on the same state; the rest state; and mass and
momentum conservation."""
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


def regularized_state(orc, seed, nx, ny, nz, tau, sponge, amp):
    """A post-collision state of the regularized collision: the collision of a
    smooth random near-rest field."""
    return orc.collide_grid(W.random_populations(seed, nx, ny, nz, amp=amp), tau, sponge)


def run_pair(T, orc, nx, ny, nz, tau, sponge, steps, seed, amp=0.05, bc=(W.BC_PERIODIC, W.BC_PERIODIC),
             u_wall=(0.0, 0.0)):
    case = W.make_case(nx, ny, nz, tau, bc[0], bc[1], sponge, u_wall=u_wall)
    C0 = regularized_state(orc, seed, nx, ny, nz, tau, sponge, amp)
    say(f"moment storage parity nx={nx} ny={ny} nz={nz} tau={tau} sponge={sponge} steps={steps} bc={bc} "
        f"u_wall={u_wall}")
    S = T.Solver([case], storage="mom")
    S.set_populations(oracle_to_soa(C0))
    for _ in range(steps):
        S.lbm_step()
    gpu = S.populations()
    err = S.body_state(0, check=False)["err"]
    S.close()
    assert err == 0
    C = C0
    for _ in range(steps):
        C = orc.collide_grid(orc.stream_grid(C, bc[0], bc[1], u_wall), tau, sponge)
    return gpu, oracle_to_soa(C), C0


CASES = [
    # nx, ny, nz, tau, sponge: tiles are 32 x 5 cells, z chunks 32 planes
    (8, 9, 10, 0.6, 0),
    (20, 14, 40, 0.8, 0),
    (33, 25, 70, 0.51, 0),
    (16, 12, 32, 1.3, 0),
    (24, 13, 48, 0.7, 9),
]


@pytest.mark.parametrize("nx,ny,nz,tau,sponge", CASES)
def test_one_step_matches_oracle(T, orc, nx, ny, nz, tau, sponge):
    gpu, ref, _ = run_pair(T, orc, nx, ny, nz, tau, sponge, 1, seed=nx * 3 + nz)
    assert max_rel(gpu, ref) < TOL_F32


@pytest.mark.parametrize("nx,ny,nz,tau,sponge", [CASES[1], CASES[2], CASES[4]])
def test_many_steps_match_oracle(T, orc, nx, ny, nz, tau, sponge):
    gpu, ref, _ = run_pair(T, orc, nx, ny, nz, tau, sponge, 25, seed=nx + ny, amp=0.02)
    assert max_rel(gpu, ref) < TOL_F32


WALLS = [
    # nx, ny, nz, tau, sponge, (bottom, top), u_wall
    (20, 14, 40, 0.8, 6, (W.BC_FREESLIP, W.BC_FREESLIP), (0.0, 0.0)),
    (33, 12, 37, 0.6, 0, (W.BC_NOSLIP, W.BC_NOSLIP), (-0.03, 0.05)),
    (24, 13, 48, 0.7, 9, (W.BC_NOSLIP, W.BC_PRESSURE), (0.0, 0.0)),   # the paper's domain
    (16, 10, 12, 0.9, 0, (W.BC_PRESSURE, W.BC_FREESLIP), (0.0, 0.0)),
]


@pytest.mark.parametrize("steps", [1, 20])
@pytest.mark.parametrize("nx,ny,nz,tau,sponge,bc,u_wall", WALLS)
def test_walls_match_oracle(T, orc, nx, ny, nz, tau, sponge, bc, u_wall, steps):
    gpu, ref, _ = run_pair(T, orc, nx, ny, nz, tau, sponge, steps, seed=nx + nz, amp=0.02, bc=bc, u_wall=u_wall)
    assert max_rel(gpu, ref) < TOL_F32


def test_round_trip_of_a_regularized_state(T, orc):
    nx, ny, nz, tau = 20, 14, 40, 0.8
    C0 = regularized_state(orc, 11, nx, ny, nz, tau, 0, 0.05)
    S = T.Solver([W.make_case(nx, ny, nz, tau, W.BC_PERIODIC, W.BC_PERIODIC, 0)], storage="mom")
    S.set_populations(oracle_to_soa(C0))
    back = S.populations()
    S.close()
    assert max_rel(back, oracle_to_soa(C0)) < 1e-6


@pytest.mark.parametrize("nx,ny,nz,tau", [(33, 25, 70, 0.55), (96, 40, 100, 0.52)])
def test_matches_population_storage(T, orc, nx, ny, nz, tau):
    case = W.make_case(nx, ny, nz, tau, W.BC_PERIODIC, W.BC_PERIODIC, 0)
    C0 = oracle_to_soa(regularized_state(orc, 5, nx, ny, nz, tau, 0, 0.03))
    out = []
    for storage in ("f32", "mom"):
        S = T.Solver([case], storage=storage)
        S.set_populations(C0)
        S.run(40)
        out.append(S.populations())
        S.close()
    assert max_rel(out[1], out[0]) < TOL_F32


def test_rest_state_and_conservation(T, orc):
    nx, ny, nz, tau = 20, 14, 40, 0.6
    case = W.make_case(nx, ny, nz, tau, W.BC_PERIODIC, W.BC_PERIODIC, 0)
    w = W.D3Q27_W
    S = T.Solver([case], storage="mom")
    rest = np.broadcast_to(w[:, None, None, None], (27, nz, ny, nx)).copy()
    S.set_populations(rest)
    S.run(10)
    assert np.array_equal(S.populations(), rest)
    C0 = oracle_to_soa(regularized_state(orc, 8, nx, ny, nz, tau, 0, 0.05))
    S.set_populations(C0)
    xi = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)], float)
    m0, j0 = C0.sum(), np.tensordot(xi.T, C0, axes=(1, 0)).reshape(3, -1).sum(1)
    S.run(50)
    f = S.populations()
    S.close()
    m1, j1 = f.sum(), np.tensordot(xi.T, f, axes=(1, 0)).reshape(3, -1).sum(1)
    assert abs(m1 - m0) / m0 < 1e-6
    assert np.abs(j1 - j0).max() < 1e-6 * m0 * 0.05
