"""MI355X-native torque-free Fast Multipole gravity solver (arXiv:2107.07166).

The solver itself lives in the HIP library built from ``csrc/`` and is reached
through ``paper_2107_07166_amd.api``; importing this package loads nothing.
"""

__all__ = ["api", "generators"]
