"""The C-ABI library loads and exports every entry point that
include/firls.h declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "firls.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|int|size_t|const char\*)\s+(firls_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("firls_create", "firls_solve", "firls_solve_batched", "firls_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1411_5057_amd import firls as F
    if not os.path.exists(F.LIB_PATH):
        pytest.fail("libfirls.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(F.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(declared()) == sorted(F.EXPORTED)


def test_binding_has_no_cpu_fallback():
    """The binding never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_1411_5057_amd", "firls.py")).read()
    assert "oracle" not in src
