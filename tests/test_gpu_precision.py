"""Precision form: the 48^3 sphere case with populations stored as FP32, FP16
and BF16 deviations f_i - w_i (per-direction power-of-two scale, FP32
arithmetic, FP64 force/torque sums and rigid-body update), compared over 2000
steps with the stored FP64 oracle trajectory
(tests/golden/sphere48_fp64_trajectory.txt, written by
make_sphere48_trajectory.py from the oracle only).  FP16 and BF16 runs keep
the library's full-precision box around the body (the particle region and a
one-cell rim stored in FP32); the FP16 run without it is reported beside.

Reported per storage: drag (F_z) relative error at step 200 and its maximum
over steps 200..2000, the drag averaged over steps 1001..2000, and the
relative error of the settling velocity v_z at step 2000 (the
terminal-velocity proxy of the plain-method case)."""
import json
import os

import numpy as np
import pytest

from paper_2408_15115_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "sphere48_fp64_trajectory.txt")
# result summaries go to $TURRET_RESULTS_DIR when it is set
OUTDIR = os.environ.get("TURRET_RESULTS_DIR")

# Bounds per storage: instantaneous drag error (max over steps 200..2000),
# drag averaged over steps 1001..2000, and v_z at step 2000.  FP32 is held to
# the parity tolerance and FP16 to the 1e-3 target on all three.  BF16 (an
# 8-bit significand) misses the 1e-3 drag target even with the box (the
# oracle's model of BF16 storage with the box reaches 1.7e-2 on the
# instantaneous drag); its bounds state that level.  FP16 without the box
# reaches 1.3e-3 / 9e-6 / 3.2e-4 and is only reported.
BOUND = {"f32": (1e-4, 1e-4, 1e-4), "f16": (1e-3, 1e-3, 1e-3), "bf16": (3e-2, 3e-2, 3e-2)}


@pytest.fixture(scope="module")
def golden():
    return np.loadtxt(GOLDEN)


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2408_15115_amd import turret
    return turret


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "f16-nobox"])
def test_drag_and_settling_velocity_vs_fp64(T, golden, storage):
    case, body = W.case_sphere48()
    steps = int(golden[-1, 0])
    say(f"precision form: sphere48, {storage}, {steps} steps")
    fine = 0 if storage.endswith("nobox") else None
    S = T.Solver([case], [body], storage=storage.split("-")[0], fine_box=fine)
    Fz = np.empty(steps)
    vz = np.empty(steps)
    for n in range(steps):
        S.run(1)
        st = S.body_state()
        Fz[n] = st["F"][2]
        vz[n] = st["v"][2]
    ref_F, ref_v = golden[:, 3], golden[:, 12]
    rel_F = np.abs(Fz - ref_F) / np.abs(ref_F)
    drag200 = float(rel_F[199])
    drag_max = float(rel_F[199:].max())
    drag_avg = float(abs(Fz[1000:].mean() - ref_F[1000:].mean()) / abs(ref_F[1000:].mean()))
    vterm = float(abs(vz[-1] - ref_v[-1]) / abs(ref_v[-1]))
    res = {"storage": storage, "drag_rel_err_step200": drag200, "drag_rel_err_max_200_2000": drag_max,
           "drag_rel_err_mean_1001_2000": drag_avg, "vz_rel_err_step2000": vterm, "Fz_2000": float(Fz[-1]), "vz_2000": float(vz[-1]),
           "ref_Fz_2000": float(ref_F[-1]), "ref_vz_2000": float(ref_v[-1])}
    say("  " + json.dumps(res))
    if OUTDIR:
        os.makedirs(OUTDIR, exist_ok=True)
        with open(os.path.join(OUTDIR, f"precision_{storage}.json"), "w") as f:
            json.dump(res, f)
        np.save(os.path.join(OUTDIR, f"precision_{storage}_Fz_vz.npy"), np.stack([Fz, vz]))
    if storage not in BOUND:
        return
    b_inst, b_avg, b_v = BOUND[storage]
    assert drag_max < b_inst
    assert drag_avg < b_avg
    assert vterm < b_v
