"""Host-side checks of the C-ABI library (no GPU needed): it loads, it exports every
function the headers in include/ declare, and argument / matrix validation rejects bad
input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1904_12754_amd import _abi
from paper_1904_12754_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libmlmc_expv.so is not built (run __graft_entry__.build())")
    return _abi.load()


def _declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(mlmc_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    declared = _declared_functions()
    assert set(declared) == set(_abi.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib()
    for code in range(9):
        assert lib.mlmc_status_string(code).decode() != "unknown status"
    assert lib.mlmc_status_string(99).decode() == "unknown status"


def _plan_status(A, beta=1.0, precision=_abi.MLMC_PRECISION_FP32, l0=-1, rows=None,
                 values_dtype=np.float64, memory=_abi.MLMC_MEMORY_HOST):
    lib = _lib()
    rp = np.ascontiguousarray(A.row_ptr, np.int64)
    ci = np.ascontiguousarray(A.col_idx, np.int32)
    va = np.ascontiguousarray(A.values, values_dtype)
    csr = _abi.CSR(A.n, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                   ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   ctypes.c_void_p(va.ctypes.data),
                   _abi.MLMC_DTYPE_F64 if values_dtype == np.float64 else _abi.MLMC_DTYPE_F32,
                   memory)
    rr = None if rows is None else np.ascontiguousarray(rows, np.int64)
    opts = _abi.PlanOpts(beta, precision, l0,
                         None if rr is None else rr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         0 if rr is None else rr.size)
    h = ctypes.c_void_p()
    code = lib.mlmc_expv_plan(ctypes.byref(h), ctypes.byref(csr), ctypes.byref(opts), None)
    return code, lib.mlmc_last_error().decode()


def test_invalid_arguments_are_rejected_on_the_host():
    A = inputs.laplacian_1d(10)
    assert _plan_status(A, beta=0.0)[0] == _abi.MLMC_ERR_INVALID_ARG
    assert _plan_status(A, beta=float("nan"))[0] == _abi.MLMC_ERR_INVALID_ARG
    assert _plan_status(A, precision=7)[0] == _abi.MLMC_ERR_INVALID_ARG
    assert _plan_status(A, rows=[0, 10])[0] == _abi.MLMC_ERR_INVALID_ARG
    assert _plan_status(A, l0=99)[0] == _abi.MLMC_ERR_INVALID_ARG
    # the l0 rule with 2 beta r_max beyond the double range: refused, not a wrapped level
    assert _plan_status(A, beta=1e308)[0] == _abi.MLMC_ERR_INVALID_ARG
    assert _plan_status(A, memory=2)[0] == _abi.MLMC_ERR_INVALID_ARG
    lib = _lib()
    assert lib.mlmc_expv_plan(None, None, None, None) == _abi.MLMC_ERR_INVALID_ARG
    assert lib.mlmc_expv_run_learned(None, None, _abi.MLMC_DTYPE_F32, None, None, None, None,
                                     None, None, None) == _abi.MLMC_ERR_INVALID_ARG
    # probe modes: unknown bits, and an LDS table past 64 KB, are refused before any launch
    g, ms = ctypes.c_uint64(), ctypes.c_double()
    fake = ctypes.c_void_p(256)
    assert lib.mlmc_probe_gather_mode(fake, 10, 16, 1, 4, ctypes.byref(g), ctypes.byref(ms),
                                      None) == _abi.MLMC_ERR_INVALID_ARG
    assert lib.mlmc_probe_gather_mode(fake, 13, 16, 1, _abi.MLMC_PROBE_LDS, ctypes.byref(g),
                                      ctypes.byref(ms), None) == _abi.MLMC_ERR_INVALID_ARG


def test_jump_counter_overflow_is_refused_on_the_host():
    """A walk's j-th jump reads Philox block j of its jump stream (a 32-bit counter word):
    a plan whose walks take beta * max r >= 2^31 jumps on average is refused before anything
    is uploaded; just below that it passes the host checks."""
    A = inputs.laplacian_1d(10)          # r = 2 / h^2 = 242 on interior rows
    code, msg = _plan_status(A, beta=2.0 ** 31 / 242, l0=28)      # r dt_28 = 8: otherwise valid
    assert code == _abi.MLMC_ERR_RNG_OVERFLOW, msg
    assert "2^31" in msg
    code, msg = _plan_status(A, beta=2.0 ** 31 / 242 * 0.999, l0=28)
    assert code != _abi.MLMC_ERR_RNG_OVERFLOW, msg


def test_invalid_matrices_are_rejected_on_the_host():
    A = inputs.laplacian_1d(6)
    bad = inputs.CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.values.copy())
    bad.col_idx[3] = 6                                     # out of range
    code, msg = _plan_status(bad)
    assert code == _abi.MLMC_ERR_INVALID_MATRIX and "out of range" in msg
    bad = inputs.CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.values.copy())
    bad.col_idx[1] = bad.col_idx[0]                        # repeated column
    code, msg = _plan_status(bad)
    assert code == _abi.MLMC_ERR_INVALID_MATRIX and "repeated" in msg
    bad = inputs.CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.values.copy())
    bad.values[2] = np.inf                                 # non-finite
    code, msg = _plan_status(bad)
    assert code == _abi.MLMC_ERR_INVALID_MATRIX and "non-finite" in msg
    bad = inputs.CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.values.copy())
    bad.row_ptr[2], bad.row_ptr[3] = bad.row_ptr[3], bad.row_ptr[2]   # not monotone
    assert _plan_status(bad)[0] == _abi.MLMC_ERR_INVALID_MATRIX
    bad = inputs.CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.values.copy())
    bad.row_ptr[0] = 1
    assert _plan_status(bad)[0] == _abi.MLMC_ERR_INVALID_MATRIX


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(ImportError):
        _abi.load()
