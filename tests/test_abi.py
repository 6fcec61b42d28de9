"""CPU checks of the C ABI: every declared symbol is exported, and invalid
inputs are rejected with the documented error codes before any device work.
A valid problem on a machine without a GPU fails loudly (MWU_ERR_DEVICE)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2307_03307_amd as mwu
from paper_2307_03307_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mwu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mwu_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_status_strings():
    L = _lib.load()
    assert L.mwu_status_string(0) == b"MWU_OK"
    for code, name in _lib.ERRORS.items():
        assert L.mwu_status_string(code).decode() == name


def _code(fn):
    with pytest.raises(mwu.MwuError) as e:
        fn()
    return e.value.code


def test_invalid_graphs_rejected():
    u = np.array([0, 1, 2], np.int32)
    v = np.array([1, 2, 0], np.int32)
    assert _code(lambda: mwu.bmatch(3, [0, 1], [1, 1])) == -5          # self-loop
    assert _code(lambda: mwu.bmatch(3, [0, 1, 0], [1, 2, 1])) == -5    # duplicate edge
    assert _code(lambda: mwu.bmatch(3, [0, 1, 2], [1, 2, 3])) == -5    # out of range
    assert _code(lambda: mwu.vertex_cover(0, [], [])) == -1             # empty graph
    assert _code(lambda: mwu.bmatch(3, u, v, eps=0.0)) == -1            # eps outside (0,1)
    assert _code(lambda: mwu.bmatch(3, u, v, eps=1.5)) == -1
    assert _code(lambda: mwu.bmatch(3, u, v, step_rule=4)) == -1        # unknown step rule
    assert _code(lambda: mwu.bmatch(3, u, v, step_rule=-1)) == -1


def test_invalid_csr_rejected():
    ptr = np.array([0, 2, 3], np.int64)
    col = np.array([0, 1, 1], np.int32)
    neg = mwu.csr_matrix(ptr, col, [1.0, -1.0, 2.0], shape=(2, 2))
    nan = mwu.csr_matrix(ptr, col, [1.0, np.nan, 2.0], shape=(2, 2))
    ok = mwu.csr_matrix(ptr, col, [1.0, 1.0, 2.0], shape=(2, 2))
    assert _code(lambda: mwu.Solver(mwu.PACKING, P=neg)) == -2
    assert _code(lambda: mwu.Solver(mwu.PACKING, P=nan)) == -3
    assert _code(lambda: mwu.Solver(mwu.PACKING, P=ok, b_P=[1.0, 0.0])) == -4
    assert _code(lambda: mwu.Solver(mwu.PACKING, P=ok, c=[1.0, -2.0])) == -4
    bad_col = mwu.csr_matrix(ptr, np.array([0, 5, 1], np.int32), shape=(2, 2))
    assert _code(lambda: mwu.Solver(mwu.PACKING, P=bad_col)) == -1
    # a packing column with no nonzero makes the LP unbounded
    empty_col = mwu.csr_matrix(np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32), shape=(2, 3))
    assert _code(lambda: mwu.Solver(mwu.PACKING, P=empty_col)) == -9
    # a covering row with no nonzero can never be satisfied
    empty_row = mwu.csr_matrix(np.array([0, 2, 2], np.int64), np.array([0, 1], np.int32), shape=(2, 2))
    assert _code(lambda: mwu.Solver(mwu.COVERING, C=empty_row)) == -1


def test_null_arguments():
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.mwu_create(None, None, ctypes.byref(h)) == -1
    assert L.mwu_solve(None, None, None, None, None) == -1
    L.mwu_destroy(None)   # NULL-safe
    lay = _lib.BatchLayout(2048, 4096, 8, 2, 0, 0, 0.0)
    assert L.mwu_batch_get_layout(None, ctypes.byref(lay)) == -1
    assert L.mwu_batch_set_layout(None, ctypes.byref(lay)) == -1


def test_valid_problem_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _code(lambda: mwu.bmatch(4, [0, 1], [2, 3])) == -8
    # every step rule passes validation and reaches the device
    for rule in (mwu.STEP_STD, mwu.STEP_BIN, mwu.STEP_BIN_WARM):
        assert _code(lambda: mwu.bmatch(4, [0, 1], [2, 3], step_rule=rule)) == -8


def test_create_batch_rejects_unsupported_problems():
    """The batched program solves matching LPs only; anything else, an empty
    batch or a NULL output handle is rejected before device work."""
    L = _lib.load()
    u = np.array([0, 1], np.int32)
    v = np.array([2, 3], np.int32)
    inc = mwu.incidence(4, u, v)
    empty = mwu._Mat(_lib.MAT_CSR)
    ok = _lib.Problem(_lib.PACKING, inc.c(), empty.c(), None, None, None)
    cov = _lib.Problem(_lib.COVERING, empty.c(), mwu.incidence_t(4, u, v).c(), None, None, None)
    h = ctypes.c_void_p()
    arr = (_lib.Problem * 2)(ok, cov)
    assert L.mwu_create_batch(arr, 2, None, ctypes.byref(h)) == -1
    assert L.mwu_create_batch(arr, 0, None, ctypes.byref(h)) == -1
    assert L.mwu_create_batch(arr, 1, None, None) == -1
    # a valid batch on a machine without a GPU: device error, no handle
    if not _has_gpu():
        assert L.mwu_create_batch(arr, 1, None, ctypes.byref(h)) == -8
        assert not h.value


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_mixed_optimization_arguments_rejected():
    """The mixed optimization forms (objective embedded as one more row)
    check their inputs before any device work: a cost vector is required and
    positive, the sides share their columns, there are covering rows, and
    when maximizing every column has a packing entry (else the LP is
    unbounded); a valid problem reaches the device."""
    P = mwu.csr_matrix(np.array([0, 2, 3], np.int64), np.array([0, 1, 1], np.int32), [1.0, 2.0, 1.0],
                       shape=(2, 2))
    C = mwu.csr_matrix(np.array([0, 2], np.int64), np.array([0, 1], np.int32), [1.0, 1.0], shape=(1, 2))
    C3 = mwu.csr_matrix(np.array([0, 1], np.int64), np.array([2], np.int32), [1.0], shape=(1, 3))
    P_gap = mwu.csr_matrix(np.array([0, 1], np.int64), np.array([0], np.int32), [1.0], shape=(1, 2))
    c = np.ones(2)
    for form in (mwu.MIXED_MAX, mwu.MIXED_MIN):
        assert _code(lambda: mwu.Solver(form, P=P, C=C)) == -1                     # no c
        assert _code(lambda: mwu.Solver(form, P=P, C=C, c=[1.0, 0.0])) == -4      # c must be positive
        assert _code(lambda: mwu.Solver(form, P=P, C=C3, c=c)) == -1              # column counts differ
        assert _code(lambda: mwu.Solver(form, P=P, C=C, c=c, b_C=[-1.0])) == -4   # bad right-hand side
    assert _code(lambda: mwu.Solver(mwu.MIXED_MAX, P=P_gap, C=C, c=c)) == -9      # column 1 unbounded
    if not _has_gpu():
        assert _code(lambda: mwu.Solver(mwu.MIXED_MAX, P=P, C=C, c=c)) == -8
        assert _code(lambda: mwu.Solver(mwu.MIXED_MIN, P=P_gap, C=C, c=c)) == -8   # minimizing keeps it
