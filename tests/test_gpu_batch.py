"""Batched form: independent cases of uneven boxes and shapes in one context
(one lattice-kernel launch over a shared tile table, batched IBM, per-case
bodies and windows).  Each case of a batch must be bitwise identical to the
same case run alone, under every schedule and tile order; one case matches
the FP64 oracle; a case that blows up is masked without disturbing the
others; the autotuner returns and caches a schedule."""
import os

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


def small_batch():
    """Three cases of different boxes, relaxation times, walls and shapes."""
    c0 = W.make_case(24, 24, 40, 0.7, W.BC_FREESLIP, W.BC_FREESLIP, 4, 2e-5, h_ini=26.0, h_end=20.0 - 1e-6)
    b0 = W.sphere_fibonacci_body(3.0, 200, 2.0, [11.8, 11.3, 20.0])
    V, F = W.ellipsoid_mesh(4.0, 3.0, 2.5, 5)
    c1 = W.make_case(32, 28, 36, 0.56, W.BC_NOSLIP, W.BC_NOSLIP, 0, 3e-5)
    b1 = W.mesh_body(V, F, 5.0, [15.2, 13.7, 18.4], d0=W.rotation_matrix([1.0, 2.0, 0.5], 0.6).T)
    V2, F2 = W.perturbed_sphere_mesh(np.random.default_rng(7), freq=6)
    c2 = W.make_case(20, 22, 48, 1.1, W.BC_FREESLIP, W.BC_FREESLIP, 6, 1e-5)
    b2 = W.mesh_body(V2 * 3.0, F2, 30.0, [9.5, 10.5, 30.0], w0=np.array([0.0, 1e-3, 0.0]))
    return [c0, c1, c2], [b0, b1, b2]


def run_alone(T, case, body, steps):
    S = T.Solver([case], [body])
    S.run(steps)
    out = S.populations(), S.body_state()
    S.close()
    return out


@pytest.fixture(scope="module")
def alone(T):
    cases, bodies = small_batch()
    return [run_alone(T, c, b, 12) for c, b in zip(cases, bodies)]


SCHEDULES = [dict(block=256, schedule=0, tile_order=0), dict(block=64, schedule=1, tile_order=1),
             dict(block=128, schedule=2, persist_wgs=7, tile_order=2),
             dict(block=256, schedule=3, persist_wgs=5, tile_order=1),
             dict(block=128, schedule=4, persist_wgs=6, tile_order=2)]


@pytest.mark.parametrize("sched", SCHEDULES)
def test_batch_case_equals_case_alone(T, alone, sched):
    cases, bodies = small_batch()
    say(f"batch isolation {sched}")
    S = T.Solver(cases, bodies, **sched)
    S.run(12)
    for c in range(3):
        f, st = S.populations(c), S.body_state(c)
        assert np.array_equal(f, alone[c][0]), c
        for k in ("r", "v", "w", "F", "T", "d"):
            assert np.array_equal(st[k], alone[c][1][k]), (c, k)
    assert S.body_state(0)["shifts"] == 1


def test_particle_free_case_in_a_batch(T, alone):
    """A case without a particle beside particle cases: it evolves exactly as
    it does alone, and the particle cases are untouched by it."""
    cases, bodies = small_batch()
    fluid = W.make_case(20, 18, 26, 0.65, W.BC_NOSLIP, W.BC_PRESSURE, 5)
    f0 = np.moveaxis(W.random_populations(21, 20, 18, 26, amp=0.02), -1, 0)
    S = T.Solver(cases + [fluid], bodies + [None])
    S.set_populations(f0, 3)
    S.run(12)
    A = T.Solver([fluid])
    A.set_populations(f0)
    A.run(12)
    assert np.array_equal(S.populations(3), A.populations())
    for c in range(3):
        assert np.array_equal(S.populations(c), alone[c][0]), c
    S.close()
    A.close()


def test_batched_cases_match_oracle(T, orc):
    """Every case of the batch (three boxes, relaxation times, walls and
    shapes, one window shift in case 0) against the oracle run alone."""
    cases, bodies = small_batch()
    S = T.Solver(cases, bodies, schedule=3, persist_wgs=16, tile_order=2)
    S.run(12)
    for c in range(3):
        say(f"batch case {c} vs oracle, 12 steps")
        o = orc.OracleSim(cases[c], bodies[c])
        o.step(12)
        err = max_rel(S.populations(c), oracle_to_soa(o.post_collision()))
        ost, st = o.body_state(), S.body_state(c)
        ferr = np.max(np.abs(st["F"] - ost["F"])) / np.linalg.norm(ost["F"])
        say(f"  populations {err:.2e}, force {ferr:.2e}, shifts {st['shifts']}")
        assert err < 1e-5 and ferr < 1e-4, c
        assert st["shifts"] == ost["shifts"]
        assert np.allclose(st["r"], ost["r"], rtol=0, atol=1e-9)
    S.close()


def test_schedule_switch_on_a_live_context(T, alone):
    cases, bodies = small_batch()
    S = T.Solver(cases, bodies)
    for k in range(12):   # the steps of the runs alone, cycling through every schedule
        S.set_schedule(**SCHEDULES[k % len(SCHEDULES)])
        S.run(1)
    for c in range(3):
        assert np.array_equal(S.populations(c), alone[c][0])


def test_masked_case_does_not_disturb_the_others(T, alone):
    """A NaN planted (from the host) in one case trips the lattice guard; that
    case is frozen and reported, the others run on bitwise unchanged."""
    cases, bodies = small_batch()
    S = T.Solver(cases, bodies, schedule=3, persist_wgs=9)
    f = S.populations(1)
    f[5, 10, 7, 9] = np.nan
    S.set_populations(f, 1)
    S.run(12)
    with pytest.raises(T.TurretError) as e:
        S.body_state(1)
    assert e.value.code == T.LBM_EUNSTABLE
    assert S.body_state(1, check=False)["err"] & 4
    for c in (0, 2):
        assert np.array_equal(S.populations(c), alone[c][0])


def test_autotuner_returns_and_caches(T, tmp_path):
    from paper_2408_15115_amd import autotune
    cases, _ = small_batch()
    path = os.path.join(tmp_path, "tune.json")
    cands = [dict(block=256, schedule=0, persist_wgs=0, tile_order=0),
             dict(block=128, schedule=3, persist_wgs=64, tile_order=2)]
    r1 = autotune.tune(cases, candidates=cands, path=path)
    assert not r1["cached"] and r1["best"] in cands and len(r1["table"]) == 2
    r2 = autotune.tune(cases, candidates=cands, path=path)
    assert r2["cached"] and r2["best"] == r1["best"]


def test_step_tuner_times_whole_steps_and_caches(T, tmp_path):
    """The whole-step selection times coupled steps (lattice kernel, coupling
    beside it, window) for the leading lattice schedules and caches its pick."""
    from paper_2408_15115_amd import autotune
    cases, bodies = small_batch()
    path = os.path.join(tmp_path, "tune.json")
    cands = [dict(block=256, schedule=0, persist_wgs=0, tile_order=0),
             dict(block=256, schedule=3, persist_wgs=64, tile_order=2)]
    r1 = autotune.tune_step(cases, bodies, candidates=cands, path=path, steps=3, warmup=1)
    sched = {k: v for k, v in r1["best"].items() if k != "serial_ibm"}
    assert not r1["cached"] and sched in cands and r1["best"]["serial_ibm"] in (0, 1)
    assert len(r1["table"]) == 3   # both schedules beside, the faster one serial
    assert r1["ms"] > 0 and r1["lattice_ms"] > 0
    r2 = autotune.tune_step(cases, bodies, candidates=cands, path=path, steps=3, warmup=1)
    assert r2["cached"] and r2["best"] == r1["best"]


@pytest.mark.parametrize("sched", [dict(schedule=3, persist_wgs=11), dict(schedule=4, persist_wgs=9)])
def test_fp16_batch_case_equals_case_alone(T, sched):
    """FP16 storage with a full-precision box per body: each case of the
    batch (persistent work-queue schedules) equals the case run alone."""
    cases, bodies = small_batch()
    S = T.Solver(cases, bodies, storage="f16", **sched)
    S.run(12)
    for c in range(3):
        A = T.Solver([cases[c]], [bodies[c]], storage="f16")
        A.run(12)
        assert np.array_equal(S.populations(c), A.populations()), c
        for k in ("r", "v", "w", "F", "T"):
            assert np.array_equal(S.body_state(c)[k], A.body_state()[k]), (c, k)
        A.close()
    S.close()
