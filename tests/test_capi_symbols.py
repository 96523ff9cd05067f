"""The C-ABI library loads (no GPU needed) and exports every function that
include/qtthom.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtthom.h")
LIB = os.path.join(ROOT, "paper_2412_11566_amd", "libqtthom.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|size_t|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path_calls():
    names = declared()
    for n in ("qtt_from_voxels", "sfft_apply", "tt_hadamard", "green_apply", "tt_round",
              "ls_solve", "ls_adjoint", "qtt_batch_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqtthom.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
