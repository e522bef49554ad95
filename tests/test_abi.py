"""The C interface: every function declared in include/schur_refine.h is exported
by the built library and bound by the Python layer (CPU only, no compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "schur_refine.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:int|size_t|void|const char\*)\s+\**\s*(\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("schur_refine", "schur_refine_batched", "schur_refine_dd",
                     "sr_workspace_bytes", "sr_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2203_10879_amd as sr

    if not os.path.exists(sr.SO_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(sr.SO_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(sr.EXPORTS)


def test_host_only_calls_without_gpu():
    import paper_2203_10879_amd as sr

    if not os.path.exists(sr.SO_PATH):
        pytest.skip("library not built")
    assert sr.sr_status_string(0) == "converged"
    assert "breakdown" in sr.sr_status_string(3)
    assert sr.sr_workspace_bytes(1024) > 3 * 16 * 1024 * 1024
    o = sr.SrOpts()
    sr.lib().sr_default_opts(ctypes.byref(o))
    assert o.gemm == 0 and o.compensated == 1 and o.gate_lp_terms == 1
