"""Writes the stored expected values in this folder.  Calls only oracle/ (and the seeded input
generators); run from the repository root:  python tests/golden/make_golden.py"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    # three CN steps of the plain 1D workload shrunk to 24 points (Sec. 2, Eqs. (2)-(4))
    w = workloads.plain_1d(n=24, dx=0.5, dt=0.05, steps=3)
    psi3 = oracle.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], w["steps"])
    # one explicit solve of a small strictly diagonally dominant system
    a, b, c, d = workloads.random_system(17, 2024, "dd")
    x = oracle.thomas(a, b, c, d)
    out = {
        "cn_plain_1d_24": {"n": 24, "dx": 0.5, "dt": 0.05, "steps": 3,
                           "psi_re": psi3.real.tolist(), "psi_im": psi3.imag.tolist()},
        "solve_dd_17": {"seed": 2024, "x_re": x.real.tolist(), "x_im": x.imag.tolist()},
        "written_by": "tests/golden/make_golden.py (oracle only)",
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
