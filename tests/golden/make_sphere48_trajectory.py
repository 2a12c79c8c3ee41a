"""Write the FP64 oracle trajectory of the 48^3 sphere case (the plain-method
case: tau 0.6, 400 Fibonacci markers, kappa 2, g 1e-5, free-slip z walls,
force and torque on the parallel surface 3 cells outside the markers) for
2000 steps.  Calls only the oracle; the stored values are its output.

Usage: python tests/golden/make_sphere48_trajectory.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2408_15115_amd import workloads as W  # noqa: E402

STEPS = 2000
OUT = os.path.join(HERE, "sphere48_fp64_trajectory.txt")


def main():
    case, body = W.case_sphere48()
    s = O.OracleSim(case, body)
    rows = []
    for n in range(1, STEPS + 1):
        s.step(1)
        b = s.body_state()
        rows.append([n, *b["F"], *b["T"], *b["F_pressure"], *b["v"], *b["r"]])
        if n % 200 == 0:
            print(n, b["F"][2], b["v"][2], flush=True)
    hdr = ("FP64 oracle trajectory, 48^3 sphere case (tau 0.6, R 4, 400 Fibonacci markers, kappa 2, "
           f"g 1e-5, free-slip z, force surface {body.get('force_offset', 0.0):g} cells out), "
           "written by make_sphere48_trajectory.py from the oracle only.\n"
           "columns: step Fx Fy Fz Tx Ty Tz Fpx Fpy Fpz vx vy vz rx ry rz")
    np.savetxt(OUT, np.array(rows), header=hdr, fmt="%.17g")


if __name__ == "__main__":
    main()
