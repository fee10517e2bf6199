"""The C-ABI library loads and exports every entry point the public header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["gsi_create", "gsi_step", "gsi_solve", "gsi_residuals", "gsi_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2306_10379_amd import gsi
    if not os.path.exists(gsi.LIB_PATH):
        pytest.fail("libgsi.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(gsi.LIB_PATH)
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing
    assert sorted(gsi.EXPORTS) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2306_10379_amd import gsi
    saved = gsi._lib
    gsi._lib = None
    try:
        with pytest.raises(RuntimeError):
            gsi.load(str(tmp_path / "missing.so"))
    finally:
        gsi._lib = saved
