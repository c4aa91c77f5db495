"""The C-ABI library loads and exports every entry point that include/oefe.h declares.

No GPU calls are made here (loading a HIP shared library does not touch the device).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oefe.h")
LIB = os.path.join(ROOT, "paper_2010_09701_amd", "liboefe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["ham_apply", "chebyshev_filter", "cholgs", "rayleigh_ritz", "band_energy_grad", "lanczos_bounds",
              "oefe_op_create", "oefe_op_destroy", "oefe_work_size"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liboefe.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="liboefe.so not built (run __graft_entry__.build())")
def test_binding_names_match_header():
    from paper_2010_09701_amd import oefe
    assert sorted(oefe.EXPORTED) == declared_functions()
