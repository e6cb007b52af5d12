"""ctypes declarations of libtfmm's C ABI (include/tfmm.h).

Loading fails loudly when the HIP library has not been built: there is no
CPU fallback anywhere in the solver.
"""

from __future__ import annotations

import ctypes
import os
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libtfmm.so"

OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4
STANDARD, CONSERVING, CONSERVING_R2 = 0, 1, 2
FP64, MIXED32 = 0, 1

STATUS_NAMES = {OK: "TFMM_OK", EINVAL: "TFMM_EINVAL", ENOMEM: "TFMM_ENOMEM",
                EDEVICE: "TFMM_EDEVICE", ESTATE: "TFMM_ESTATE"}

# Every symbol the header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t


class Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("theta", ctypes.c_double), ("softening", ctypes.c_double),
                ("G", ctypes.c_double), ("variant", ctypes.c_int), ("precision", ctypes.c_int),
                ("scalar_degree", ctypes.c_int)]


SIGNATURES = {
    "tfmm_ctx_create": (_int, [_int, _sz, ctypes.POINTER(_vp)]),
    "tfmm_ctx_destroy": (_int, [_vp]),
    "tfmm_last_error": (ctypes.c_char_p, [_vp]),
    "tfmm_ctx_bytes_in_use": (_sz, [_vp]),
    "tfmm_ctx_bytes_held": (_sz, [_vp]),
    "tfmm_ctx_trim": (_int, [_vp]),
    "tfmm_ctx_set_budget": (_int, [_vp, _sz]),
    "tfmm_build_tree": (_int, [_vp, _i64, _vp, _vp, _int, _vp, ctypes.POINTER(_vp)]),
    "tfmm_tree_rebuild": (_int, [_vp, _i64, _vp, _vp, _vp]),
    "tfmm_build_forest": (_int, [_vp, _int, _vp, _vp, _vp, _int, _vp, ctypes.POINTER(_vp)]),
    "tfmm_forest_rebuild": (_int, [_vp, _int, _vp, _vp, _vp, _vp]),
    "tfmm_evaluate_forest": (_int, [_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp]),
    "tfmm_tree_walk": (_int, [_vp, _d, _vp]),
    "tfmm_evaluate_forces": (_int, [_vp, ctypes.POINTER(Params), _vp, _vp, _vp]),
    "tfmm_evaluate_forces_oneshot": (_int, [_vp, _i64, _vp, _vp, _int, ctypes.POINTER(Params), _vp, _vp]),
    "tfmm_leapfrog": (_int, [_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _d, _int, _int, _vp]),
    "tfmm_momentum_diagnostics": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tfmm_momentum_diagnostics_noalloc": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tfmm_tree_info": (_int, [_vp, _vp]),
    "tfmm_tree_export": (_int, [_vp] + [_vp] * 12),
    "tfmm_lists_export": (_int, [_vp, _vp, _vp]),
    "tfmm_tree_destroy": (_int, [_vp]),
    "tfmm_footprint_bytes": (_sz, [_i64, _int, _int, _int]),
    "tfmm_tree_set_timing": (_int, [_vp, _int]),
    "tfmm_tree_phase_times": (_int, [_vp, _vp]),
}

_lib = None


def load(path: os.PathLike | str | None = None):
    """Load libtfmm.so (built by paper_2107_07166_amd/build.py) and declare its ABI."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path is not None else LIB_PATH
    if not p.exists():
        raise RuntimeError(
            f"libtfmm.so not found at {p}: build it first with "
            "`python paper_2107_07166_amd/build.py` (there is no CPU fallback)")
    lib = ctypes.CDLL(str(p))
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class TfmmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
