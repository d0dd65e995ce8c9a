"""The C-ABI library loads and exports every function include/orqa.h declares
(no compute call: runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "orqa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2506_13241_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2506_13241_amd import build
        build.build()
    return ctypes.CDLL(P.LIB_PATH)


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ("pauli_sum_create", "apply_rotation_layer", "pauli_sum_truncate", "expectation_z"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    import paper_2506_13241_amd as P
    names = header_functions()
    assert set(names) == set(P.EXPORTED_SYMBOLS)
    for n in names:
        assert hasattr(lib, n), n


def test_binding_refuses_missing_library(tmp_path):
    import paper_2506_13241_amd as P
    saved = P._lib
    try:
        P._lib = None
        with pytest.raises(ImportError):
            P.load_library(str(tmp_path / "missing.so"))
    finally:
        P._lib = saved


def test_invalid_arguments_fail_before_any_device_call(lib):
    import paper_2506_13241_amd as P
    L = P.load_library()
    h = ctypes.c_void_p()
    assert L.pauli_sum_create(0, 1, 0, 0, None, None, 0, None, ctypes.byref(h)) == P.PS_ERR_INVALID
    assert L.pauli_sum_create(5, 33, 0, 0, None, None, 0, None, ctypes.byref(h)) == P.PS_ERR_INVALID
    assert b"n_lanes" in L.ps_last_error()


def test_scorer_and_graph_entry_points_validate_before_device_calls(lib):
    import numpy as np
    import paper_2506_13241_amd as P
    L = P.load_library()
    s = ctypes.c_void_p()
    qm = np.zeros((160, 2), dtype=np.uint64)
    let = np.zeros(160, dtype=np.uint8)
    sc = np.ones(160, dtype=np.float32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    # NULL tables, qubit count out of range, letter out of range
    assert L.ps_scorer_create(127, None, ptr(let), ptr(sc), None, ctypes.byref(s)) == P.PS_ERR_INVALID
    assert L.ps_scorer_create(0, ptr(qm), ptr(let), ptr(sc), None, ctypes.byref(s)) == P.PS_ERR_INVALID
    bad = let.copy()
    bad[7] = 4
    assert L.ps_scorer_create(127, ptr(qm), ptr(bad), ptr(sc), None, ctypes.byref(s)) == P.PS_ERR_INVALID
    assert b"feature 7" in L.ps_last_error()
    # NULL handles
    assert L.ps_scorer_set_params(None, None, 0) == P.PS_ERR_INVALID
    assert L.ps_scorer_get_params(None, None, 0) == P.PS_ERR_INVALID
    assert L.ps_scorer_set_data(None, None, None, 0) == P.PS_ERR_INVALID
    assert L.ps_scorer_forward(None, None, None) == P.PS_ERR_INVALID
    assert L.ps_scorer_loss_grad(None, None, None) == P.PS_ERR_INVALID
    assert L.ps_scorer_adam_step(None, ctypes.c_float(1e-3)) == P.PS_ERR_INVALID
    assert L.ps_scorer_destroy(None) == P.PS_OK
    assert L.pauli_sum_load_scorer(None, None) == P.PS_ERR_INVALID
    assert L.pauli_sum_set_graphs(None, 1) == P.PS_ERR_INVALID
    assert L.pauli_sum_set_timing(None, 1) == P.PS_ERR_INVALID


def test_binding_has_every_entry_point_by_name():
    """The Python binding offers every C entry point under its own name."""
    import paper_2506_13241_amd as P
    assert [n for n in P.EXPORTED_SYMBOLS if not callable(getattr(P, n, None))] == []
