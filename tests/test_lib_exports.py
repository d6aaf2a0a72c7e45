"""The C-ABI library loads and exports every function include/sfc.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2508_19891_amd import build_lib, sfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(sfc_[a-z_0-9]+)\s*\(", text, re.M)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    if not os.path.exists(sfc.LIB_PATH):
        build_lib.build()
    L = ctypes.CDLL(sfc.LIB_PATH)
    names = declared_functions()
    assert "sfc_build" in names and "sfc_query_batch" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_declared_symbols():
    assert set(declared_functions()) <= set(sfc.EXPORTS)
