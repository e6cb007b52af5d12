"""Build libtfmm.so (HIP, gfx950) in-tree.

Compiles every csrc/*.hip translation unit with hipcc for gfx950 into
_build/ and links paper_2107_07166_amd/libtfmm.so.  The expansion operators
are regenerated first (csrc/gen_expansions.py -> csrc/expansions_gen.h).

Flags:
* packed FP32 instructions are disabled for all device code (hipcc's host
  pass warns that it does not know the feature; that is harmless);
* the tree and walk units are compiled without floating-point contraction,
  so the FP64 quantities that decide the node table and the interaction lists
  are reproducible bit for bit.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = ROOT / "_build"
LIB = PKG / "libtfmm.so"

ARCH = os.environ.get("TFMM_OFFLOAD_ARCH", "gfx950")
NO_CONTRACT = {"tree.hip", "walk.hip"}


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libtfmm)")


def _flags(src: Path):
    f = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
         "-Wno-unused-command-line-argument",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         f"-I{ROOT / 'include'}", f"-I{CSRC}"]
    if src.name in NO_CONTRACT:
        f.append("-ffp-contract=off")
    return f


def build(verbose: bool = False, jobs: int | None = None) -> str:
    subprocess.run([sys.executable, str(CSRC / "gen_expansions.py")], check=True,
                   stdout=subprocess.DEVNULL)
    BUILD.mkdir(exist_ok=True)
    hipcc = _hipcc()
    srcs = sorted(CSRC.glob("*.hip"))

    def compile_one(src: Path) -> Path:
        obj = BUILD / (src.stem + ".o")
        cmd = [hipcc, "-c", str(src), "-o", str(obj)] + _flags(src)
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src.name} failed:\n{r.stderr}")
        noise = [ln for ln in r.stderr.splitlines()
                 if ln.strip() and "packed-fp32-ops" not in ln and "target-feature" not in ln]
        if verbose and noise:
            print("\n".join(noise), flush=True)
        return obj

    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", str(tmp)] + [str(o) for o in objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libtfmm.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return str(LIB)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
