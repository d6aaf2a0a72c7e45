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


def test_options_layout_matches_header():
    """sfc_default_options (host only) fills the binding's struct: every field
    lands where the header puts it, the last one (metric) included."""
    if not os.path.exists(sfc.LIB_PATH):
        build_lib.build()
    L = ctypes.CDLL(sfc.LIB_PATH)
    opt = sfc.Options()
    ctypes.memset(ctypes.byref(opt), 0x5A, ctypes.sizeof(opt))
    L.sfc_default_options(ctypes.byref(opt))
    assert (opt.curve, opt.search, opt.refine, opt.learn_steps) == (sfc.MORTON, sfc.BINARY, 0, -1)
    assert opt.early_term == 0 and opt.metric == sfc.L2
    assert not opt.stream and not opt.alloc_ctx
