"""Host-side checks of the benchmark's command line and the schedule tuner's
candidate set (no GPU)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""   # no JSON line


def test_tuner_candidates_cover_every_lattice_schedule():
    from paper_2408_15115_amd import autotune
    cands = autotune.default_candidates(256)
    assert {c["schedule"] for c in cands} == {0, 1, 2, 3, 4}
    for c in cands:
        assert c["block"] in (64, 128, 256)
        assert c["tile_order"] in (0, 1, 2)
        # persistent schedules get an explicit workgroup count, the others none
        assert (c["persist_wgs"] > 0) == (c["schedule"] >= 2)
    assert len({tuple(sorted(c.items())) for c in cands}) == len(cands)
