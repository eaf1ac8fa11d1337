"""CPU oracle for C = A * B on CSR operands -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports, links or calls it, and
it imports nothing from the GPU library: the two share only the seeded input
generators in ``synthetic``.

The arithmetic lives in ``smash_oracle.c`` (row-wise Gustavson with a dense
sparse accumulator, long double sums; the Background chapter's eq.
"inner_product" evaluated in the order of eq. "row_wise").  This module loads
it through ctypes (compiling it with gcc when the shared object is missing)
and adds the numpy pieces: the per-row product count of the Window
Distribution Phase, CSR transpose and dense conversion.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smash_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_smash_oracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


_GCC = ["gcc", "-O3", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O3 for any x86-64 host (the built object
    travels to the machine that runs the tests, whose CPU may differ)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(_GCC + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def use_native_build() -> str:
    """Compile the oracle for the host it runs on (-O3 -march=native, in a
    temporary directory) and load that build instead: the CPU baseline of
    the benchmark times the oracle at the host's best, while the tests keep
    the portable build.  Returns the path of the shared object."""
    global _lib
    import tempfile
    d = tempfile.mkdtemp(prefix="smash_oracle_")
    path = os.path.join(d, "_smash_oracle_native.so")
    subprocess.check_call(_GCC + ["-march=native", "-o", path, _SRC, "-lm"])
    _lib = None
    _load(path)
    return path


def _load(path=None):
    global _lib
    if _lib is None:
        if path is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB_PATH
        lib = ctypes.CDLL(path)
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_validate.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i32p]
        lib.oracle_row_nnz.restype = ctypes.c_int
        lib.oracle_row_nnz.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                       ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                       _i64p, ctypes.c_int64, _i64p, ctypes.c_int]
        lib.oracle_fill.restype = ctypes.c_int
        lib.oracle_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i32p, _f64p,
                                    ctypes.c_int64, ctypes.c_int64, _i32p, _i32p, _f64p,
                                    _i64p, ctypes.c_int64, _i64p,
                                    _i32p, _f64p, _f64p, _i64p, ctypes.c_int]
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------------ checks

VALIDATE_MESSAGES = {
    0: "ok",
    1: "row_ptr[0] != 0",
    2: "row_ptr decreases",
    3: "column index out of range",
    4: "columns not strictly ascending within a row",
    5: "negative size",
}


def validate(M) -> int:
    """0 if M is canonical CSR (see VALIDATE_MESSAGES for the other codes)."""
    rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
    if rp.shape[0] != M.rows + 1:
        return 2
    return int(_load().oracle_validate(M.rows, M.cols, _p(rp, _i32p), _p(ci, _i32p)))


# ------------------------------------------------------------ the product

def products_per_row(A, B) -> np.ndarray:
    """Products (multiply-adds) of each output row, sum over k in row i of A of
    nnz(B row k): the per-row FMA count the Window Distribution Phase derives
    from the row pointers (Gustavson's two-step algorithm).  int64[m]."""
    brow = np.diff(B.row_ptr.astype(np.int64))
    per_entry = brow[A.col_idx.astype(np.int64)] if A.nnz else np.zeros(0, np.int64)
    pref = np.zeros(A.nnz + 1, dtype=np.int64)
    np.cumsum(per_entry, out=pref[1:])
    rp = A.row_ptr.astype(np.int64)
    return pref[rp[1:]] - pref[rp[:-1]]


def _sel(rows, m):
    if rows is None:
        return None, m
    sel = np.ascontiguousarray(rows, dtype=np.int64)
    if sel.size and (sel.min() < 0 or sel.max() >= m):
        raise IndexError("selected row out of range")
    return sel, int(sel.shape[0])


def row_nnz(A, B, rows=None, threads=None) -> np.ndarray:
    """Exact nnz of each (selected) row of C = A*B, int64."""
    if A.cols != B.rows:
        raise ValueError("inner dimensions differ")
    lib = _load()
    sel, nsel = _sel(rows, A.rows)
    out = np.zeros(nsel, dtype=np.int64)
    a_rp = np.ascontiguousarray(A.row_ptr, np.int32); a_ci = np.ascontiguousarray(A.col_idx, np.int32)
    b_rp = np.ascontiguousarray(B.row_ptr, np.int32); b_ci = np.ascontiguousarray(B.col_idx, np.int32)
    rc = lib.oracle_row_nnz(A.rows, A.cols, _p(a_rp, _i32p), _p(a_ci, _i32p),
                            B.rows, B.cols, _p(b_rp, _i32p), _p(b_ci, _i32p),
                            _p(sel, _i64p) if sel is not None else None, nsel,
                            _p(out, _i64p), threads or default_threads())
    if rc != 0:
        raise MemoryError("oracle_row_nnz failed")
    return out


def spgemm(A, B, rows=None, threads=None, with_stats=True):
    """C = A*B for all rows (or the selected ``rows``), in double.

    Returns a dict with ``row_ptr`` (int64, len(rows)+1, relative to the
    selection), ``col`` (int32), ``val`` (float64), and when ``with_stats``
    ``absmass`` (sum of |a_ik b_kj| per entry) and ``terms`` (products merged
    per entry)."""
    if A.cols != B.rows:
        raise ValueError("inner dimensions differ")
    lib = _load()
    th = threads or default_threads()
    sel, nsel = _sel(rows, A.rows)
    cnt = row_nnz(A, B, rows, th)
    rp = np.zeros(nsel + 1, dtype=np.int64)
    np.cumsum(cnt, out=rp[1:])
    nnz = int(rp[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    absm = np.empty(nnz, dtype=np.float64) if with_stats else None
    terms = np.empty(nnz, dtype=np.int64) if with_stats else None
    a_rp = np.ascontiguousarray(A.row_ptr, np.int32); a_ci = np.ascontiguousarray(A.col_idx, np.int32)
    b_rp = np.ascontiguousarray(B.row_ptr, np.int32); b_ci = np.ascontiguousarray(B.col_idx, np.int32)
    a_v = np.ascontiguousarray(A.val, np.float64); b_v = np.ascontiguousarray(B.val, np.float64)
    rc = lib.oracle_fill(A.rows, A.cols, _p(a_rp, _i32p), _p(a_ci, _i32p), _p(a_v, _f64p),
                         B.rows, B.cols, _p(b_rp, _i32p), _p(b_ci, _i32p), _p(b_v, _f64p),
                         _p(sel, _i64p) if sel is not None else None, nsel, _p(rp, _i64p),
                         _p(col, _i32p), _p(val, _f64p),
                         _p(absm, _f64p) if with_stats else None,
                         _p(terms, _i64p) if with_stats else None, th)
    if rc != 0:
        raise MemoryError("oracle_fill failed")
    out = {"row_ptr": rp, "col": col, "val": val}
    if with_stats:
        out["absmass"] = absm
        out["terms"] = terms
    return out


# --------------------------------------------------------------- helpers

def transpose(M):
    """CSR of M^T (stable: entries of a column keep ascending row order)."""
    from synthetic import CSR
    rows_of = np.repeat(np.arange(M.rows, dtype=np.int64), np.diff(M.row_ptr.astype(np.int64)))
    order = np.lexsort((rows_of, M.col_idx.astype(np.int64)))
    counts = np.bincount(M.col_idx.astype(np.int64), minlength=M.cols)[:M.cols] if M.nnz else np.zeros(M.cols, np.int64)
    rp = np.zeros(M.cols + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return CSR(M.cols, M.rows, rp.astype(np.int32), rows_of[order].astype(np.int32), M.val[order])


def to_dense(M, dtype=np.float64) -> np.ndarray:
    D = np.zeros((M.rows, M.cols), dtype=dtype)
    rows_of = np.repeat(np.arange(M.rows), np.diff(M.row_ptr.astype(np.int64)))
    D[rows_of, M.col_idx] = M.val
    return D
