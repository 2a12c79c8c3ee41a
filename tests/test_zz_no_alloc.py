"""The no-allocation population read (lbm_get_populations_noalloc) against
lbm_get_populations: bit for bit, on two calls in a row through the C ABI,
the second on a smaller case, for moment storage (whose read stages the
rebuilt populations in the library's fixed device scratch) and for FP16
population storage; and the size limit of the scratch."""
import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2408_15115_amd import turret
    return turret


def read_both(T, case, body, storage, steps, f0=None):
    import torch
    S = T.Solver([case], [body] if body is not None else None, storage=storage)
    if f0 is not None:
        S.set_populations(np.ascontiguousarray(np.moveaxis(f0, -1, 0)))
    S.run(steps)
    nx, ny, nz = S.dims[0]
    dev = torch.full((S.q * nx * ny * nz,), float("nan"), dtype=torch.float64, device="cuda")
    S.populations_noalloc(dev)
    S.stream.synchronize()
    got = dev.cpu().numpy().reshape(S.q, nz, ny, nx)
    ref = S.populations()
    shifts = S.body_state()["shifts"] if body is not None else 0
    S.close()
    return got, ref, shifts


@pytest.mark.parametrize("storage", ["mom", "f16"])
def test_noalloc_read_equals_the_allocating_read(T, storage):
    big_case, big_body = W.case_sphere48()
    # a window shift of 6 rows early in the run, so that the ring origin is not 0
    big_case["h_ini"], big_case["h_end"] = 29.5, 23.4999
    small_case = W.make_case(20, 16, 24, 0.7, W.BC_NOSLIP, W.BC_PRESSURE, 5)
    say(f"no-allocation read, {storage}: 48^3 sphere after 30 steps, then a 20x16x24 box after 7 steps")
    got, ref, shifts = read_both(T, big_case, big_body, storage, 30)
    assert shifts == 1
    assert np.array_equal(got, ref)
    f0 = W.random_populations(4, 20, 16, 24, amp=0.05)
    got2, ref2, _ = read_both(T, small_case, None, storage, 7, f0)
    assert np.array_equal(got2, ref2)
    assert np.abs(got2 - W.D3Q27_W[:, None, None, None]).max() > 1e-4     # a state away from rest


def test_noalloc_read_rejects_cases_beyond_the_scratch(T):
    import torch
    case = W.make_case(96, 96, 80, 0.7, W.BC_FREESLIP, W.BC_FREESLIP, 0)   # 737k cells: 80 MB staged
    S = T.Solver([case], storage="mom")
    dev = torch.empty(27 * 96 * 96 * 80, dtype=torch.float64, device="cuda")
    with pytest.raises(T.TurretError) as e:
        S.populations_noalloc(dev)
    assert e.value.code == T.LBM_EINVAL and "scratch" in str(e.value)
    S.close()
