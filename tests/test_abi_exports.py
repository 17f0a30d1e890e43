"""The C-ABI library loads and exports every function include/colsten.h declares.
(No compute call: this runs without a GPU.)"""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(cs_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("cs_grid_create", "cs_grid_destroy", "cs_colour_pass", "cs_gs_sweeps",
                 "cs_jacobi_sweeps", "cs_residual", "cs_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_1810_04033_amd import colsten
    lib = ctypes.CDLL(colsten.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(colsten.exported_symbols()) == _declared()
