"""The C-ABI library loads and exports every symbol include/tfmm.h declares.

CPU-only: nothing here launches device work.
"""
import re
from pathlib import Path

import pytest

from paper_2107_07166_amd import _lib

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "tfmm.h"


def _declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfmm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    assert set(_declared()) == set(_lib.SIGNATURES)


@pytest.fixture(scope="module")
def lib():
    if not _lib.LIB_PATH.exists():
        pytest.fail("libtfmm.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_host_only_entry_points(lib):
    # pure host computations and argument checks that never touch a device
    fp = lib.tfmm_footprint_bytes(1 << 20, 4, 64, 1)
    assert fp > (1 << 20) * 100
    assert lib.tfmm_footprint_bytes(0, 4, 64, 1) == 0
    assert lib.tfmm_footprint_bytes(1000, 9, 64, 1) == 0
    assert lib.tfmm_footprint_bytes(2 << 20, 4, 64, 1) > fp
    assert lib.tfmm_tree_info(None, None) == _lib.EINVAL
    assert lib.tfmm_last_error(None) == b"NULL context"
    assert lib.tfmm_ctx_create(0, 0, None) == _lib.EINVAL
    assert lib.tfmm_tree_destroy(None) == _lib.OK
    assert lib.tfmm_ctx_destroy(None) == _lib.OK
    assert lib.tfmm_ctx_bytes_held(None) == 0
    assert lib.tfmm_ctx_trim(None) == _lib.EINVAL
    assert lib.tfmm_ctx_set_budget(None, 0) == _lib.EINVAL
    assert lib.tfmm_build_forest(None, 1, None, None, None, 8, None, None) == _lib.EINVAL
    assert lib.tfmm_forest_rebuild(None, 1, None, None, None, None) == _lib.EINVAL
    assert lib.tfmm_evaluate_forest(None, None, None, None, None, None) == _lib.EINVAL
