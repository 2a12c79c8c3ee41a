"""Mutation check of the oracle's pins.

Each entry plants one plausible mistake in a scratch copy of ``orc.c``
(a coefficient, a sign, an index, a dropped term or step, a wrong loop
bound), builds it, and runs the pin files named for it against that build
through ``ORACLE_LIB_OVERRIDE``.  Every mutant must make at least one pin
fail; the unmodified source must pass the same files.  A surviving mutant
means some part of the oracle is not fixed by anything outside itself."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle", "orc.c")
ORC19 = os.path.join(ROOT, "oracle", "orc19.c")

COLL = "tests/test_oracle_collision.py"
TRAN = "tests/test_oracle_transport.py"
BODY = "tests/test_oracle_body.py"
PHYS = "tests/test_oracle_physics.py"
IBM = "tests/test_oracle_ibm.py"
WALL = "tests/test_oracle_walls.py"
SYM = "tests/test_oracle_symmetry.py"
STOK = "tests/test_oracle_stokes.py"

# (name, text in orc.c, replacement, pin files expected to catch it)
MUTANTS = [
    # forcing loop of Sec. 2.2 (l = 0..4, n cycles)
    ("ibm_drop_l2", "u2[3 * q + a] = S->uu[3 * q + a] + S->h[3 * q + a];",
     "u2[3 * q + a] = S->uu[3 * q + a];", [IBM]),
    ("ibm_three_cycles", "S->cycles = ip[3];", "S->cycles = ip[3] - 1;", [IBM]),
    ("ibm_loop_bound", "for (int c = 1; c <= S->cycles; c++) {", "for (int c = 1; c < S->cycles; c++) {", [IBM]),
    ("ibm_update_sign", "S->hk[3 * k + a] += S->U[3 * k + a] - I[3 * k + a];",
     "S->hk[3 * k + a] -= S->U[3 * k + a] - I[3 * k + a];", [IBM]),
    ("ibm_l0_sign", "S->hk[3 * k + a] = S->U[3 * k + a] - I[3 * k + a];",
     "S->hk[3 * k + a] = I[3 * k + a] - S->U[3 * k + a];", [IBM]),
    ("ibm_no_reset", "memset(S->h, 0, 3 * n * sizeof(double));\n        for (int k = 0; k < M; k++) spread_add",
     "for (int k = 0; k < M; k++) spread_add", [IBM]),
    ("spread_area", "H[3 * cc + d] += h[d] * W * dS;", "H[3 * cc + d] += h[d] * W;", [TRAN, IBM]),
    ("marker_velocity", "S->U[3 * k + a] = S->B.v[a] + wr[a];", "S->U[3 * k + a] = S->B.v[a] - wr[a];", [PHYS]),
    # equilibrium and off-equilibrium of App. A
    ("feq_order5", "case 5: return 1.0 / (4.0 * pow(CS2, 5));", "case 5: return 1.0 / (2.0 * pow(CS2, 5));", [COLL]),
    ("feq_order6", "case 6: return 1.0 / (8.0 * pow(CS2, 6));", "case 6: return 1.0 / (4.0 * pow(CS2, 6));", [COLL]),
    ("feq_mult_xyz", "{3, {X_, Y_, Z_}, 2.0}", "{3, {X_, Y_, Z_}, 1.0}", [COLL]),
    ("hermite_rec", "s -= CS2 * hermite(xi, sub, n - 2);", "s -= hermite(xi, sub, n - 2);", [COLL]),
    ("a1_perm_index", "s += prod * P1[al[(m - 1 + r) % m]][al[n - 1]];",
     "s += prod * P1[al[(m - 1) % m]][al[n - 1]];", [COLL]),
    ("term_asymmetric", "{4, {X_, Y_, Y_, Z_}, 2.0}", "{4, {X_, Y_, Y_, Z_}, 1.0}", [SYM]),
    ("fneq_h2", "double s = h2 / (2.0 * CS2 * CS2);", "double s = h2 / (CS2 * CS2);", [COLL]),
    ("density", "*p = CS2 * (s - RHO0);", "*p = CS2 * s;", [COLL]),
    # collision and stress (Sec. 2.1, 2.2)
    ("missing_tau_shift", "us[d] = u[d] + tau * (h ? h[d] : 0.0);", "us[d] = u[d] + (h ? h[d] : 0.0);", [COLL]),
    ("relax_factor", "out[i] = fs[i] + (1.0 - 1.0 / tau) * f1[i];", "out[i] = fs[i] + (1.0 - 0.5 / tau) * f1[i];",
     [COLL]),
    ("stress_factor", "(1.0 / (2.0 * tau) - 1.0) * P1[a][b]", "(1.0 / tau - 1.0) * P1[a][b]", [COLL]),
    ("sim_pressure", "S->sig[10 * c + 9] = CS2 * (rho - RHO0);", "S->sig[10 * c + 9] = 0.5 * CS2 * (rho - RHO0);",
     [PHYS]),
    # weight function, stencil, streaming, walls
    ("kernel_branch", "return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * r * r));",
     "return 0.125 * (5.0 - 2.0 * a + sqrt(-7.0 + 12.0 * a - 4.0 * r * r));", [TRAN]),
    ("stencil_base", "int b = (int)floor(X[d]) - 1;", "int b = (int)floor(X[d]) - 2;", [TRAN]),
    ("stream_x", "int sx = wrap(x - g_xi[i][0], D->nx);", "int sx = wrap(x + g_xi[i][0], D->nx);", [TRAN]),
    ("freeslip_mirror", "int im = 9 * (-g_xi[i][2] + 1) + 3 * (g_xi[i][1] + 1) + (g_xi[i][0] + 1);",
     "int im = 9 * (-g_xi[i][2] + 1) + 3 * (-g_xi[i][1] + 1) + (g_xi[i][0] + 1);", [TRAN]),
    ("pressure_wall", "f[Q * c + i] = -C[Q * c + (Q - 1 - i)] + 2.0 * g_w[i] * RHO0;",
     "f[Q * c + i] = -C[Q * c + (Q - 1 - i)] + g_w[i] * RHO0;", [PHYS]),
    ("moving_wall", "2.0 * g_w[i] * RHO0 * g_xi[i][0] * uw / CS2", "2.0 * g_w[i] * RHO0 * g_xi[i][0] * uw", [WALL]),
    ("sponge_denominator", "(double)(D->nz - 1 - zs)", "(double)(D->nz - zs)", [TRAN]),
    # force and torque (Sec. 2.2)
    ("torque_order", "cross(rel, s, rs);", "cross(s, rel, rs);", [PHYS]),
    ("force_area", "F[a] += area * s[a];", "F[a] += s[a];", [PHYS]),
    ("force_point", "Y[a] = S->X[3 * k + a] + S->force_offset * nk[a];",
     "Y[a] = S->X[3 * k + a] - S->force_offset * nk[a];", [PHYS]),
    # rigid body (Sec. 2.3)
    ("corrector_half", "mid[d] = 0.5 * (di[d] + dp[d]);", "mid[d] = dp[d];", [BODY]),
    ("M_not_inverse", "matvec(Minv, t2, t3);", "matvec(B->d, t2, t3);", [BODY]),
    ("gravity_sign", "F[2] / kv - B->gravity", "F[2] / kv + B->gravity", [BODY]),
    ("external_torque", "T[0] + B->Text[0]", "T[0] - B->Text[0]", [BODY]),
    # falling-frame window (Sec. 2.5)
    ("window_reset", "dst[Q * c + i] = g_w[i];", "dst[Q * c + i] = 0.0;", [PHYS]),
    ("window_delta", "int dz = (int)lround(S->h_ini - S->h_end);", "int dz = (int)lround(S->h_ini - S->h_end) + 1;",
     [PHYS]),
]


def _build(src_text: str, out_dir: str, name: str) -> str:
    c_path = os.path.join(out_dir, f"orc_{name}.c")
    so_path = os.path.join(out_dir, f"liboracle_{name}.so")
    with open(c_path, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-w", c_path, ORC19, "-o", so_path, "-lm"])
    return so_path


def _run_pins(so_path: str, files: list[str]) -> int:
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=so_path, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
           *files]
    return subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL).returncode


def _pin_files():
    return sorted({f for m in MUTANTS for f in m[3]})


@pytest.mark.slow
def test_mutants_are_distinct_single_edits():
    src = open(ORC).read()
    names = [m[0] for m in MUTANTS]
    assert len(names) == len(set(names))
    for name, old, new, _ in MUTANTS:
        assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once"
        assert old != new


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    src = open(ORC).read()
    control = _build(src, str(tmp_path), "control")
    assert _run_pins(control, _pin_files()) == 0, "the unmodified oracle must pass its pins"

    def one(m):
        name, old, new, files = m
        so = _build(src.replace(old, new), str(tmp_path), name)
        return name, _run_pins(so, files)

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(one, MUTANTS))
    survivors = [n for n, rc in results if rc == 0]
    broken = [(n, rc) for n, rc in results if rc not in (0, 1)]
    assert not broken, f"pin runs that errored instead of failing: {broken}"
    assert not survivors, f"mutants that pass every pin: {survivors}"
