"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and rejects invalid problems before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import mipgen
import paper_2605_05086_amd as chap
from helpers import make_mip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chap.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(chap.LIB_PATH):
        from paper_2605_05086_amd import build
        build.build()
    return chap.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chap_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert "chap_problem_create" in names and "chap_best_shift" in names and "chap_tabu_run" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in chap.h but not exported"


def test_options_defaults(lib):
    o = chap.default_options()
    assert o.feas_tol == 1e-6 and o.graph_iters == 64 and o.short_max == 8
    assert o.chunk_min == 4096 and o.chunk_len == 4096 and o.row_stage == 1 and o.rescore_cap == 0


@pytest.mark.parametrize("cap", [-1, 4097])
def test_rescore_cap_out_of_range(lib, cap):
    mip = mipgen.random_mixed(3, n=10, m=6)
    with pytest.raises(chap.ChapError, match="CHAP_EINVAL"):
        chap.Problem(mip, rescore_cap=cap)


def _create_rc(mip, **over):
    k = dict(
        csr_row_ptr=np.ascontiguousarray(mip.csr_row_ptr, dtype=np.int64),
        csr_col=np.ascontiguousarray(mip.csr_col, dtype=np.int32),
        csr_val=np.ascontiguousarray(mip.csr_val, dtype=np.float64),
        csc_col_ptr=np.ascontiguousarray(mip.csc_col_ptr, dtype=np.int64),
        csc_row=np.ascontiguousarray(mip.csc_row, dtype=np.int32),
        csc_val=np.ascontiguousarray(mip.csc_val, dtype=np.float64),
        sense=np.ascontiguousarray(mip.sense, dtype=np.uint8),
        rhs=np.ascontiguousarray(mip.rhs, dtype=np.float64),
        lb=np.ascontiguousarray(mip.lb, dtype=np.float64),
        ub=np.ascontiguousarray(mip.ub, dtype=np.float64),
        is_int=np.ascontiguousarray(mip.is_int, dtype=np.uint8),
        obj=np.ascontiguousarray(mip.obj, dtype=np.float64),
    )
    k.update(over)
    lib = chap.load_library()
    h = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.chap_problem_create(ctypes.byref(h), int(mip.n), int(mip.m), p(k["csr_row_ptr"]), p(k["csr_col"]),
                                 p(k["csr_val"]), p(k["csc_col_ptr"]), p(k["csc_row"]), p(k["csc_val"]),
                                 p(k["sense"]), p(k["rhs"]), p(k["lb"]), p(k["ub"]), p(k["is_int"]), p(k["obj"]),
                                 None)
    if rc == 0:
        lib.chap_problem_destroy(h)
    return rc, lib.chap_last_error().decode()


def test_invalid_problems_rejected(lib):
    mip = mipgen.random_mixed(3, n=10, m=8)
    # a valid problem passes validation (and then needs a device)
    rc, msg = _create_rc(mip)
    assert rc in (0, -5), msg
    bad_val = mip.csc_val.copy()
    bad_val[0] += 1.0
    assert _create_rc(mip, csc_val=bad_val)[0] == -1
    bad_row = mip.csc_row.copy()
    bad_row[0] = mip.m
    assert _create_rc(mip, csc_row=bad_row)[0] == -1
    bad_sense = mip.sense.copy()
    bad_sense[0] = ord("X")
    rc, msg = _create_rc(mip, sense=bad_sense)
    assert rc == -1 and "sense" in msg
    bad_rhs = mip.rhs.copy()
    bad_rhs[1] = np.nan
    assert _create_rc(mip, rhs=bad_rhs)[0] == -1
    lb = mip.lb.copy()
    ub = mip.ub.copy()
    lb[2], ub[2] = 3.0, 2.0
    rc, msg = _create_rc(mip, lb=lb, ub=ub)
    assert rc == -1 and "empty domain" in msg
    isint = mip.is_int.copy()
    lb2 = mip.lb.copy()
    ub2 = mip.ub.copy()
    isint[0], lb2[0], ub2[0] = 1, 0.2, 0.8  # no integer inside
    assert _create_rc(mip, is_int=isint, lb=lb2, ub=ub2)[0] == -1
    nanv = mip.csr_val.copy()
    nanv[0] = np.inf
    assert _create_rc(mip, csr_val=nanv)[0] == -1


def test_duplicate_entry_rejected(lib):
    # the same (row, col) twice in both CSR and CSC
    mip = make_mip(2, [({0: 1.0, 1: 2.0}, "L", 3.0)], [0, 0], [5, 5], [1, 1])
    csr_col = np.array([0, 0], dtype=np.int32)
    csr_val = np.array([1.0, 2.0])
    csc_ptr = np.array([0, 2, 2], dtype=np.int64)
    csc_row = np.array([0, 0], dtype=np.int32)
    rc, msg = _create_rc(mip, csr_col=csr_col, csr_val=csr_val, csc_col_ptr=csc_ptr, csc_row=csc_row, csc_val=csr_val)
    assert rc == -1 and "repeated" in msg


def test_stored_zeros_are_dropped(lib):
    mip = make_mip(2, [({0: 1.0, 1: 2.0}, "L", 3.0)], [0, 0], [5, 5], [1, 1])
    csr_val = np.array([1.0, 0.0])
    csc_val = np.array([1.0, 0.0])
    rc, msg = _create_rc(mip, csr_val=csr_val, csc_val=csc_val)
    assert rc in (0, -5), msg


def test_no_cpu_fallback_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(chap, "_lib", None)
    monkeypatch.setattr(chap, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        chap.load_library()
