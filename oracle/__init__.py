"""CPU oracle for sort-based duplicate removal, grouping and aggregation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the
benchmark's CPU-baseline leg are the only users.  The product library never
imports, links or calls anything here, and nothing here touches the GPU path.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc):
sort the rows on the grouping key, then aggregate in one in-stream pass
(the traditional "sort, then aggregate" plan of Section 1 / Figure 2, and the
in-stream grouping of sorted input quoted in Section 2.1).  This module only
marshals numpy arrays in and out.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, host only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-pthread", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        U = ctypes.c_uint64
        lib.oracle_group_by.restype = U
        lib.oracle_group_by.argtypes = [U, P, P, P, P, P, P, P, P, P]
        lib.oracle_group_by_parallel.restype = U
        lib.oracle_group_by_parallel.argtypes = [U, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_nproc.restype = ctypes.c_int
        lib.oracle_nproc.argtypes = []
        lib.oracle_group_by_pairs.restype = U
        lib.oracle_group_by_pairs.argtypes = [U, P, P, P, P, P, P, P, P, P]
        lib.oracle_exact_sum.restype = ctypes.c_double
        lib.oracle_exact_sum.argtypes = [P, U]
        lib.oracle_count_distinct.restype = U
        lib.oracle_count_distinct.argtypes = [U, P, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def nproc():
    """Online host cores (the default thread count of ``group_by(threads=0)``)."""
    return int(_load().oracle_nproc())


def group_by(keys, v_i64=None, v_f64=None, threads=1):
    """Group rows on a uint64 key.

    Returns a dict with ``keys``, ``count``, and, when the matching value
    column is given, ``sum_i64``/``min_i64``/``max_i64`` (int64 column) and
    ``sum_f64`` (float64 column, exact sum rounded once).

    ``threads`` other than 1 runs the same sort-then-scan plan on that many
    host threads (0: every online core) over key ranges cut at sampled
    splitters; the result is identical bit for bit.
    """
    lib = _load()
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    n = keys.shape[0]
    v = None if v_i64 is None else np.ascontiguousarray(v_i64, dtype=np.int64)
    f = None if v_f64 is None else np.ascontiguousarray(v_f64, dtype=np.float64)
    m = max(n, 1)
    ok = np.empty(m, np.uint64)
    oc = np.empty(m, np.uint64)
    os_ = np.empty(m, np.int64) if v is not None else None
    omn = np.empty(m, np.int64) if v is not None else None
    omx = np.empty(m, np.int64) if v is not None else None
    of = np.empty(m, np.float64) if f is not None else None
    if threads == 1:
        g = lib.oracle_group_by(n, _ptr(keys), _ptr(v), _ptr(f), _ptr(ok), _ptr(oc),
                                _ptr(os_), _ptr(of), _ptr(omn), _ptr(omx))
    else:
        g = lib.oracle_group_by_parallel(n, _ptr(keys), _ptr(v), _ptr(f), _ptr(ok), _ptr(oc),
                                         _ptr(os_), _ptr(of), _ptr(omn), _ptr(omx), int(threads))
    out = {"keys": ok[:g].copy(), "count": oc[:g].copy()}
    if v is not None:
        out["sum_i64"] = os_[:g].copy()
        out["min_i64"] = omn[:g].copy()
        out["max_i64"] = omx[:g].copy()
    if f is not None:
        out["sum_f64"] = of[:g].copy()
    return out


def group_by_pairs(a, b, v):
    """Group rows on the pair (a, b) of int32 columns, ordered by (a, b) signed."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int64)
    n = a.shape[0]
    m = max(n, 1)
    oa = np.empty(m, np.int32)
    ob = np.empty(m, np.int32)
    oc = np.empty(m, np.uint64)
    os_ = np.empty(m, np.int64)
    omn = np.empty(m, np.int64)
    omx = np.empty(m, np.int64)
    g = lib.oracle_group_by_pairs(n, _ptr(a), _ptr(b), _ptr(v), _ptr(oa), _ptr(ob),
                                  _ptr(oc), _ptr(os_), _ptr(omn), _ptr(omx))
    return {"a": oa[:g].copy(), "b": ob[:g].copy(), "count": oc[:g].copy(),
            "sum_i64": os_[:g].copy(), "min_i64": omn[:g].copy(),
            "max_i64": omx[:g].copy()}


def exact_sum(x):
    """Exact sum of a float64 array, rounded once to nearest-even."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib.oracle_exact_sum(_ptr(x), x.shape[0]))


def count_distinct(g, x):
    """count(*) and count(distinct x) per group g, from one sort on (g, x)."""
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.uint64)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    n = g.shape[0]
    m = max(n, 1)
    og = np.empty(m, np.uint64)
    oc = np.empty(m, np.uint64)
    od = np.empty(m, np.uint64)
    k = lib.oracle_count_distinct(n, _ptr(g), _ptr(x), _ptr(og), _ptr(oc), _ptr(od))
    return {"keys": og[:k].copy(), "count": oc[:k].copy(), "distinct": od[:k].copy()}
