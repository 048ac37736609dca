"""The C-ABI library loads and exports every function that include/dabs.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dabs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dabs_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_calls():
    names = declared_functions()
    for must in ("dabs_problem_create", "dabs_search", "dabs_batch_search", "dabs_energy",
                 "dabs_solver_create", "dabs_solver_run", "dabs_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2207_03069_amd as dabs
    if not os.path.exists(dabs.LIB_PATH):
        pytest.fail("libdabs.so is not built")
    lib = ctypes.CDLL(dabs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # host-only calls work without a device
    assert dabs.dabs_strerror(dabs.DABS_E_NOT_SYMMETRIC) == "W is not symmetric"
    assert dabs.dabs_max_n(dabs.DABS_W_I16) >= 2048


def test_binding_names_match_header():
    import paper_2207_03069_amd as dabs
    for n in declared_functions():
        assert hasattr(dabs, n), n
