"""Writes the oracle regression fixtures in this folder.

Calls only the oracle (and the seeded input generators).  The fixtures
freeze the oracle's FP64 forces on a small seeded ball so that any later
change of its arithmetic shows up as a test failure and must be justified.
Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2107_07166_amd.generators import uniform_ball  # noqa: E402

CASES = [  # (name, n, seed, n_leaf, theta, p, eps, variant)
    ("ball96_p3_standard", 96, 210707166, 4, 0.5, 3, 1e-3, "standard"),
    ("ball96_p3_conserving", 96, 210707166, 4, 0.5, 3, 1e-3, "conserving"),
    ("ball96_p6_conserving", 96, 210707166, 4, 0.7, 6, 0.0, "conserving"),
]


def main():
    for name, n, seed, n_leaf, theta, p, eps, variant in CASES:
        pos, m = uniform_ball(n, seed)
        t = oracle.Tree(pos, m, n_leaf=n_leaf, theta=theta)
        f = t.forces(p, eps, variant)
        hdr = (f"oracle forces (G=1), uniform ball n={n} seed={seed} n_leaf={n_leaf} "
               f"theta={theta} p={p} eps={eps} variant={variant}; "
               f"far pairs={t.n_m2l} near pairs={t.n_p2p}")
        np.savetxt(os.path.join(HERE, name + ".txt"), f, fmt="%.17e", header=hdr)


if __name__ == "__main__":
    main()
