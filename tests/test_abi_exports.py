"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^(?:mxl_status|const char \*)\s*(mxl_\w+)\s*\(", txt, re.M))
    return names


def test_header_declares_entry_points():
    d = declared()
    for must in ("mxl_apply", "mxl_apply_adv", "mxl_solve", "mxl_csr_create", "mxl_convert",
                 "mxl_jacobi_generate", "mxl_solver_generate", "mxl_ir_generate"):
        assert must in d


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2006_16852_amd", "libmxl.so"))
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_imports_without_gpu():
    import paper_2006_16852_amd as mxl
    assert mxl.version().startswith("mxl")
