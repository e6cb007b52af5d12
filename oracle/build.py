"""Build the oracle shared library (plain C, FP64, no contraction, OpenMP).

TEST INFRASTRUCTURE: compiles oracle.c into liboracle.so next to it.
"""

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent


def build(verbose: bool = False) -> str:
    src = HERE / "oracle.c"
    out = HERE / "liboracle.so"
    tmp = HERE / "liboracle.so.tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", os.fspath(tmp), os.fspath(src), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return os.fspath(out)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
