"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs its own pins without a report: every array access
of the oracle stays in bounds and no integer overflow, bad shift or
misaligned access happens on the pinned cases.  The long Couette runs are left
out to keep the suite short; they exercise the same wall code as the shorter
wall pins."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.slow
def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc's sanitizer runtimes are not installed")
    so = str(tmp_path / "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "orc.c"), os.path.join(ROOT, "oracle", "orc19.c"),
                           "-o", so, "-lm"])
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=so, OMP_NUM_THREADS="4", LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    # the sanitizer runtime is the one the interpreter has loaded
    probe = "import ctypes; assert hasattr(ctypes.CDLL(None), '__asan_init')"
    assert subprocess.run([sys.executable, "-c", probe], env=env).returncode == 0
    pins = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", "-k", "not couette", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stdout + r.stderr, tail
    assert "AddressSanitizer" not in r.stdout + r.stderr, tail
