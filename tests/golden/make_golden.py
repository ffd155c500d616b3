"""Writes the stored oracle values under tests/golden/ (calls only oracle/ and workloads/)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import fg  # noqa: E402


def main():
    a = W.square_coeff(45, d=2, fraction=0.3, inside=10.0, outside=1.0)
    r = fg.solve(a, tol=1e-12, max_iter=2000)
    with open(os.path.join(HERE, "square2d_N45_AH.txt"), "w") as f:
        f.write("# A_H of the 2D square inclusion (N = 45, 10 inside, side sqrt(0.3)),\n")
        f.write("# oracle.fg PCG to 1e-12; written by tests/golden/make_golden.py\n")
        for row in r.A_H:
            f.write(" ".join(f"{v:.17e}" for v in row) + "\n")


if __name__ == "__main__":
    main()
