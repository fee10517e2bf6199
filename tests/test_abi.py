"""The C-ABI library loads and exports every entry point the public header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for header in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:gsi|fno)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


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
    from paper_2306_10379_amd import fno
    assert sorted(gsi.EXPORTS + fno.EXPORTS) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2306_10379_amd import gsi
    saved = gsi._lib
    gsi._lib = None
    try:
        with pytest.raises(RuntimeError):
            gsi.load(str(tmp_path / "missing.so"))
    finally:
        gsi._lib = saved


def test_network_parameter_count_matches_reference():
    """fno_param_count is host arithmetic (no device call): it must equal the reference's
    count for the documented layout and reject invalid configurations."""
    from oracle import fno_oracle as F
    from paper_2306_10379_amd import fno
    L = fno.load()
    for cfg in [F.Config(), F.Config(N=16, m=6, w=5, L=2, p=4), F.Config(N=32, m=11, w=7, L=0, p=9)]:
        for bf16 in (0, 1):
            c = fno.FnoConfig(cfg.N, cfg.m, cfg.w, cfg.L, cfg.p, 4, bf16)
            assert L.fno_param_count(ctypes.byref(c)) == F.param_count(cfg)
    for bad in [(20, 6, 5, 2, 4, 1), (16, 40, 5, 2, 4, 1), (16, 6, 33, 2, 4, 1), (16, 6, 5, 2, 0, 1),
                (16, 6, 5, 2, 4, 1, 2)]:
        assert L.fno_param_count(ctypes.byref(fno.FnoConfig(*bad))) == -1


def test_ctypes_structs_match_the_header_layout(tmp_path):
    # the ctypes mirrors of the C structs must have the header's sizes and field offsets:
    # a small C program compiled against include/ prints them
    import shutil
    import subprocess
    from paper_2306_10379_amd import fno, gsi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gsi_options": gsi.GsiOptions, "gsi_csr": gsi.GsiCsr, "gsi_stencil": gsi.GsiStencil,
               "gsi_zcsr": gsi.GsiZcsr, "fno_config": fno.FnoConfig}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsi.h"', '#include "fno.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
