"""Work and byte accounting for C = A * B (measurement only, no kernels).

The byte model is the denominator of the paper's arithmetic-intensity bound
(Results chapter, eq. "ai_spgemm"): every CSR array of A, B and C moved once,
sized as in the tables "data_sizes_input" and "data_sizes_output" (int32 row
pointers and column indices, ``value_bytes`` per stored value).  The one
deliberate difference is C's row pointer, which this library writes as int64
because nnz(C) can exceed 2^31 - 1.

"flop" in the compression factor (eq. "ai_cf") counts products, i.e. merged
multiply-adds: with the paper's cf = 1.23 and Table "data_metrics" that reading
reproduces the printed AI = 0.09, while 2 x products would imply fewer
products than output entries.  Throughput is reported as GFLOP/s of
2 x products (one multiply and one add per product).
"""
from __future__ import annotations


def csr_bytes(rows: int, nnz: int, value_bytes: int, index_bytes: int = 4, row_ptr_bytes: int = 4) -> int:
    """Bytes of one CSR matrix: (rows + 1) row pointers, nnz indices, nnz values."""
    return (rows + 1) * row_ptr_bytes + nnz * index_bytes + nnz * value_bytes


def algorithmic_bytes(m: int, rows_b: int, nnz_a: int, nnz_b: int, nnz_c: int, value_bytes: int) -> int:
    """Compulsory HBM bytes of one product: read A and B once, write C once
    (C's row pointer as int64)."""
    return (csr_bytes(m, nnz_a, value_bytes)
            + csr_bytes(rows_b, nnz_b, value_bytes)
            + csr_bytes(m, nnz_c, value_bytes, row_ptr_bytes=8))


def compression_factor(products: int, nnz_c: int) -> float:
    """cf = flop / nnz(C), flop counted as products (eq. "ai_cf")."""
    return products / nnz_c if nnz_c else 0.0


def arithmetic_intensity(products: int, nnz_a: int, nnz_b: int, nnz_c: int, element_bytes: int) -> float:
    """The bound nnz(C) * cf / ((nnz(A) + nnz(B) + nnz(C)) * b) of eq. "ai_spgemm"."""
    tot = (nnz_a + nnz_b + nnz_c) * element_bytes
    return nnz_c * compression_factor(products, nnz_c) / tot if tot else 0.0


def gflops(products: int, seconds: float) -> float:
    """2 x products per second, in GFLOP/s."""
    return 2.0 * products / seconds / 1e9 if seconds > 0 else 0.0
