"""The C ABI: libddml.so loads and exports every entry point include/ddml.h declares.

No compute call is made, so this runs without a GPU.  The Python binding's
export list must match the header as well (it is the names the tests and the
benchmark call through).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddml.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(ddml_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ["ddml_create", "ddml_set_gauge", "ddml_set_domain", "ddml_apply_Dw", "ddml_solve_domain",
              "ddml_propagator_series", "ddml_contract_pp_disconnected", "ddml_contract_nucleon",
              "ddml_apply_boundary", "ddml_factorized_series", "ddml_contract_pion", "ddml_submit"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1601_04587_amd import build, ddml
    if not os.path.exists(ddml.LIB_PATH):
        build.build()
    lib = ctypes.CDLL(ddml.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(ddml.EXPORTS) == declared()
    ddml.load()   # argument types set for every binding
