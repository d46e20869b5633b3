"""The C-ABI library loads and exports every entry point its header declares
(no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpmc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mpmc_init", "mpmc_free", "mpmc_rhs", "mpmc_rk3_step", "mpmc_adjoint_step",
                     "mpmc_compute_dt", "mpmc_stats"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2504_14063_amd import mpmc
    if not os.path.exists(mpmc.LIB_PATH):
        pytest.skip("libmpmc.so not built")
    lib = ctypes.CDLL(mpmc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_oracle_is_not_linked_by_the_library():
    from paper_2504_14063_amd import mpmc
    if not os.path.exists(mpmc.LIB_PATH):
        pytest.skip("libmpmc.so not built")
    lib = ctypes.CDLL(mpmc.LIB_PATH)
    assert not hasattr(lib, "oracle_rk3_step")
    for f in os.listdir(os.path.join(ROOT, "paper_2504_14063_amd", "csrc")):
        txt = open(os.path.join(ROOT, "paper_2504_14063_amd", "csrc", f)).read()
        assert "oracle" not in txt.lower(), f
