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


STRUCTS = {"rbf_opts": "RbfOpts", "rbf_solve_opts": "RbfSolveOpts", "rbf_solve_info": "RbfSolveInfo",
           "rbf_plan_info": "RbfPlanInfo", "rbf_band_info": "RbfBandInfo", "rbf_batch_info": "RbfBatchInfo", "rbf_train_opts": "RbfTrainOpts",
           "rbf_train_info": "RbfTrainInfo"}


def test_binding_struct_layouts_match_header():
    """Every ctypes struct has the C size and every field the C offset (computed by gcc)."""
    import subprocess
    import tempfile
    from paper_1606_07652_amd import _lib
    lines, expect = [], []
    for cname, pyname in STRUCTS.items():
        st = getattr(_lib, pyname)
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(st))
        for fname, _ in st._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append(getattr(st, fname).offset)
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"rbf_fmm.h\"\nint main(void){" + "".join(lines) + "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    assert got == expect


def test_header_constants_match_binding():
    import subprocess
    import tempfile
    from paper_1606_07652_amd import _lib
    names = ["RBF_PC_BLOCK", "RBF_MLP_IN", "RBF_MLP_HIDDEN", "RBF_MLP_NPARAMS", "RBF_MLP_BF16", "RBF_MLP_F32",
             "RBF_PC_NONE", "RBF_PC_BLOCK_JACOBI", "RBF_PC_LEARNED", "RBF_NPHASES", "RBF_ESTATE"]
    src = "#include <stdio.h>\n#include \"rbf_fmm.h\"\nint main(void){" + "".join(
        f'printf("%ld\\n", (long)({n}));' for n in names) + "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    assert got == [getattr(_lib, n) for n in names]


def test_product_path_fails_loudly_without_library(monkeypatch):
    from paper_1606_07652_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/librbffmm.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError):
        _lib.load()
