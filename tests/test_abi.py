"""The C ABI library loads and exports every function include/*.h declares (CPU only:
no compute call is made)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1606_07652_amd", "lib", "librbffmm.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        for m in re.finditer(r"\b(?:int|const\s+char\s*\*)\s*(rbf_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rbf_fmm_plan", "rbf_fmm_matvec", "rbf_interp_solve", "rbf_fmm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_the_same_functions():
    from paper_1606_07652_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_binding_struct_sizes_match_header():
    """The ctypes structs must match the C layout (sizes computed by the C compiler)."""
    import subprocess
    import tempfile
    from paper_1606_07652_amd import _lib
    src = r'''
#include <stdio.h>
#include "rbf_fmm.h"
int main(void){printf("%zu %zu %zu %zu\n", sizeof(rbf_opts), sizeof(rbf_solve_opts), sizeof(rbf_solve_info), sizeof(rbf_plan_info));return 0;}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(v) for v in subprocess.check_output([exe]).split()]
    assert sizes == [ctypes.sizeof(_lib.RbfOpts), ctypes.sizeof(_lib.RbfSolveOpts),
                     ctypes.sizeof(_lib.RbfSolveInfo), ctypes.sizeof(_lib.RbfPlanInfo)]


def test_product_path_fails_loudly_without_library(monkeypatch):
    from paper_1606_07652_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/librbffmm.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError):
        _lib.load()
