"""Regression of the oracle against fixtures written by tests/golden/make_golden.py.

The fixtures were produced by the oracle itself; they are not an external
pin (the pins live in test_oracle_pins.py and test_oracle_tree.py) but make
any later change of the oracle's arithmetic visible.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import uniform_ball

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,n,seed,n_leaf,theta,p,eps,variant", [
    ("ball96_p3_standard", 96, 210707166, 4, 0.5, 3, 1e-3, "standard"),
    ("ball96_p3_conserving", 96, 210707166, 4, 0.5, 3, 1e-3, "conserving"),
    ("ball96_p6_conserving", 96, 210707166, 4, 0.7, 6, 0.0, "conserving"),
])
def test_oracle_matches_frozen_fixture(name, n, seed, n_leaf, theta, p, eps, variant):
    ref = np.loadtxt(os.path.join(HERE, name + ".txt"))
    pos, m = uniform_ball(n, seed)
    f = oracle.Tree(pos, m, n_leaf=n_leaf, theta=theta).forces(p, eps, variant)
    np.testing.assert_allclose(f, ref, rtol=1e-14, atol=1e-16 * np.abs(ref).max())
