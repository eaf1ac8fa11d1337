"""Comparison of a GPU product with the oracle (test helper).

Structure (row_ptr and col_idx) must be bit-exact.  Values must satisfy
|c_gpu - c_ref| <= tol * absmass per entry, absmass = sum |a_ik b_kj|, with
tol = 1e-5 for FP32 and 1e-12 for FP64; an entry with absmass = 0 must be
exactly zero.  Entries with a single term (m = 1) are one rounded product
and must match bitwise (FP64) or equal the FP32 rounding of the oracle value.
"""
import numpy as np

TOL = {np.float32: 1e-5, np.float64: 1e-12}


def check_rows(row_ptr, col, val, ref, dtype, where=""):
    """row_ptr/col/val: host arrays of the GPU result for the same rows as
    ``ref`` (an oracle.spgemm dict); row_ptr may be absolute (it is rebased)."""
    rp = np.asarray(row_ptr, np.int64)
    rp = rp - rp[0]
    assert np.array_equal(rp, ref["row_ptr"]), f"{where}: row_ptr differs"
    assert np.array_equal(np.asarray(col), ref["col"]), f"{where}: col_idx differs"
    v = np.asarray(val).astype(np.float64)
    tol = TOL[np.dtype(dtype).type]
    err = np.abs(v - ref["val"])
    bound = tol * ref["absmass"]
    bad = err > bound
    if bad.any():
        i = int(np.argmax(bad))
        raise AssertionError(f"{where}: {int(bad.sum())} values out of tolerance; first at {i}: "
                             f"gpu={v[i]!r} ref={ref['val'][i]!r} absmass={ref['absmass'][i]!r}")
    single = ref["terms"] == 1
    if np.dtype(dtype) == np.float64:
        assert np.array_equal(v[single], ref["val"][single]), f"{where}: single-term FP64 entries not bitwise"
    else:
        assert np.array_equal(np.asarray(val)[single], ref["val"][single].astype(np.float32)), \
            f"{where}: single-term FP32 entries not bitwise"
    margin = float(np.max(err / np.where(ref["absmass"] > 0, ref["absmass"], 1.0))) if err.size else 0.0
    return margin


def check_streaming(C, A, B, oracle_mod, dtype, where, chunk=1 << 27, log=print):
    """Every entry of C (device tensors: row_ptr int64, col_idx, val) against
    the oracle, in chunks of whole rows of about `chunk` entries: the
    oracle computes the chunk's rows, the GPU's slice is copied back, and
    check_rows compares them (row counts, columns, values).  Returns (the
    largest |err| / absmass, entries compared)."""
    rp = C.row_ptr.cpu().numpy()
    assert rp[0] == 0, f"{where}: row_ptr[0] != 0"
    m = A.rows
    worst, done, r0 = 0.0, 0, 0
    while r0 < m:
        r1 = int(np.searchsorted(rp, rp[r0] + chunk, side="right")) - 1
        r1 = min(max(r1, r0 + 1), m)
        s, e = int(rp[r0]), int(rp[r1])
        ref = oracle_mod.spgemm(A, B, rows=np.arange(r0, r1, dtype=np.int64))
        col = C.col_idx[s:e].cpu().numpy()
        val = C.val[s:e].cpu().numpy()
        worst = max(worst, check_rows(rp[r0:r1 + 1], col, val, ref, dtype, f"{where} rows {r0}..{r1 - 1}"))
        done += e - s
        del ref, col, val
        log(f"{where}: rows {r0}..{r1 - 1} ok ({done} entries so far, max err/absmass {worst:.2e})", flush=True)
        r0 = r1
    assert done == int(rp[m])
    return worst, done
