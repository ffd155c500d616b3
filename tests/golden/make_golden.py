"""Writes the stored oracle values under tests/golden/ (calls only oracle/ and workloads/).

    python tests/golden/make_golden.py [square2d] [ball243]

With no argument every value is written.  The 243^3 ball takes about an
hour of one CPU core (the oracle's full-spectrum PCG on 14.3 M points).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import fg  # noqa: E402


def square2d():
    a = W.square_coeff(45, d=2, fraction=0.3, inside=10.0, outside=1.0)
    r = fg.solve(a, tol=1e-12, max_iter=2000)
    with open(os.path.join(HERE, "square2d_N45_AH.txt"), "w") as f:
        f.write("# A_H of the 2D square inclusion (N = 45, 10 inside, side sqrt(0.3)),\n")
        f.write("# oracle.fg PCG to 1e-12; written by tests/golden/make_golden.py\n")
        for row in r.A_H:
            f.write(" ".join(f"{v:.17e}" for v in row) + "\n")


def ball243():
    # The centred ball is invariant under permutations and reflections of
    # the axes, so A_H = a_H I (eq. homog) and the corrector for E = e1
    # fixes a_H; the oracle solves that one field.
    N = 243
    a = W.ball_coeff(N, radius=0.3, inside=100.0, outside=1.0)
    t0 = time.time()
    r = fg.solve(a, Es=[[1.0, 0.0, 0.0]], tol=1e-10, max_iter=2000)
    dt = time.time() - t0
    with open(os.path.join(HERE, "ball3d_N243_c100_AH.txt"), "w") as f:
        f.write("# a_H = A_H[0][0] of the 3D ball |x| < 0.3 (N = 243, 100 inside, 1 outside),\n")
        f.write("# E = e1; oracle.fg PCG to 1e-10 (%d iterations, %.0f s);\n" % (r.iters[0], dt))
        f.write("# written by tests/golden/make_golden.py\n")
        f.write(f"{r.A_H[0, 0]:.17e}\n")


def main():
    which = sys.argv[1:] or ["square2d", "ball243"]
    for w in which:
        {"square2d": square2d, "ball243": ball243}[w]()


if __name__ == "__main__":
    main()
