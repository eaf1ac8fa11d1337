"""Seeded synthetic CSR workloads.

This module only draws inputs: it holds none of the multiply's arithmetic,
and both the HIP path's tests/benchmarks and the CPU oracle's tests take
their inputs from here.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: output ``i`` of stream ``s`` is ``mix(s + (i + 1) * GOLDEN)``, so
any slice of a stream can be drawn independently and vectorised.

RMAT follows Chakrabarti, Zhan and Faloutsos (SDM 2004), the generator the
paper's evaluation uses (Results chapter, experimental methodology): each
sample descends ``scale`` levels, picking one of the four quadrants with
probabilities (a, b, c, d) at each level, most significant bit first.
Duplicates are merged in the structure, self-loops are kept, there is no
noise and no vertex permutation.  Values are drawn after deduplication, one
per stored entry in CSR order, as ``2u - 1`` with ``u`` a 53-bit uniform in
[0, 1); FP32 inputs round that double to nearest.
"""
from __future__ import annotations

import dataclasses
import os
import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream salts keep the structure and value draws of one seed independent.
SALT_STRUCT = 0x0
SALT_VALUES = 0x5A17F00D5A17F00D
SALT_SHAPE = 0x0BADC0DE0BADC0DE

# RMAT quadrant probabilities used by every RMAT workload here.
RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream ``seed``."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    """53-bit uniforms in [0, 1) from the SplitMix64 stream ``seed``."""
    return (splitmix64(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: int32 row_ptr/col_idx, float32 or float64 values."""

    rows: int
    cols: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def astype(self, dtype) -> "CSR":
        return CSR(self.rows, self.cols, self.row_ptr, self.col_idx, self.val.astype(dtype))


def _values(seed: int, nnz: int, dtype) -> np.ndarray:
    v = 2.0 * uniform01(seed ^ SALT_VALUES, 0, nnz) - 1.0
    return v.astype(dtype)


def csr_from_coo(rows: int, cols: int, r: np.ndarray, c: np.ndarray, seed: int, dtype) -> CSR:
    """Merge duplicate (r, c) pairs, order row-major with ascending columns,
    and draw one value per stored entry."""
    if cols <= 0:
        key = np.zeros(0, dtype=np.int64)
    else:
        key = np.unique(r.astype(np.int64) * cols + c.astype(np.int64))
    rr = (key // max(cols, 1)).astype(np.int64)
    cc = (key % max(cols, 1)).astype(np.int32)
    counts = np.bincount(rr, minlength=rows)[:rows] if rows > 0 else np.zeros(0, np.int64)
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("input nnz exceeds int32 indexing")
    return CSR(rows, cols, row_ptr.astype(np.int32), cc, _values(seed, key.shape[0], dtype))


def rmat_coo(scale: int, samples: int, seed: int, abcd=RMAT_ABCD, start: int = 0):
    """Raw RMAT samples ``start .. start+samples-1`` (row, col) of stream ``seed``."""
    a, b, c, _ = abcd
    r = np.zeros(samples, dtype=np.int64)
    cc = np.zeros(samples, dtype=np.int64)
    base = np.arange(start, start + samples, dtype=np.int64) * scale
    for level in range(scale):
        # draw index (sample * scale + level) of the structure stream
        idx = base + level
        u = _uniform_at(seed ^ SALT_STRUCT, idx)
        bit = np.int64(1) << np.int64(scale - 1 - level)
        down = u >= (a + b)              # quadrants c, d: lower half (row bit set)
        right = ((u >= a) & (u < a + b)) | (u >= a + b + c)  # quadrants b, d: column bit set
        r |= np.where(down, bit, 0)
        cc |= np.where(right, bit, 0)
    return r, cc


def _uniform_at(seed: int, idx: np.ndarray) -> np.ndarray:
    """Uniforms at arbitrary stream positions ``idx`` (int64 array)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx.astype(np.uint64) + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def rmat(scale: int, edge_factor: int, seed: int, dtype=np.float32, abcd=RMAT_ABCD) -> CSR:
    """Square 2^scale RMAT matrix from ``edge_factor * 2^scale`` samples."""
    n = 1 << scale
    e = edge_factor * n
    chunk = 1 << 22
    rs, cs = [], []
    for s0 in range(0, e, chunk):
        r, c = rmat_coo(scale, min(chunk, e - s0), seed, abcd, start=s0)
        rs.append(r)
        cs.append(c)
    r = np.concatenate(rs) if rs else np.zeros(0, np.int64)
    c = np.concatenate(cs) if cs else np.zeros(0, np.int64)
    return csr_from_coo(n, n, r, c, seed, dtype)


def rmat_rect(n: int, edge_factor: int, seed: int, dtype=np.float32, abcd=RMAT_ABCD) -> CSR:
    """n x n RMAT matrix for a non power-of-two n: samples are drawn at scale
    ceil(log2 n) and those falling outside [0, n)^2 are rejected until
    ``edge_factor * n`` samples have been accepted."""
    scale = max(1, math.ceil(math.log2(n)))
    need = edge_factor * n
    rs, cs = [], []
    got = 0
    pos = 0
    while got < need:
        batch = max(1024, 2 * (need - got))
        r, c = rmat_coo(scale, batch, seed, abcd, start=pos)
        pos += batch
        keep = (r < n) & (c < n)
        r, c = r[keep], c[keep]
        take = min(need - got, r.shape[0])
        rs.append(r[:take])
        cs.append(c[:take])
        got += take
    return csr_from_coo(n, n, np.concatenate(rs), np.concatenate(cs), seed, dtype)


def uniform_k_per_row(rows: int, cols: int, k: int, seed: int, dtype=np.float32) -> CSR:
    """Exactly ``k`` distinct uniform columns per row (requires k <= cols).

    Each row draws k candidates; rows holding a duplicate redraw all k from
    the next block of the stream until every row is duplicate-free."""
    if k > cols:
        raise ValueError("k > cols")
    if k * k > 8 * cols:
        # redraws would almost never succeed: take, per row, the k columns
        # with the smallest of cols uniform keys
        out = np.empty((rows, k), dtype=np.int64)
        for r in range(rows):
            u = uniform01(seed ^ SALT_STRUCT, r * cols, cols)
            out[r] = np.sort(np.argpartition(u, k - 1)[:k])
        rr = np.repeat(np.arange(rows, dtype=np.int64), k)
        return csr_from_coo(rows, cols, rr, out.reshape(-1), seed, dtype)
    out = np.empty((rows, k), dtype=np.int64)
    todo = np.arange(rows, dtype=np.int64)
    rnd = 0
    while todo.shape[0]:
        idx = (np.int64(rnd) * rows + todo)[:, None] * k + np.arange(k, dtype=np.int64)[None, :]
        u = _uniform_at(seed ^ SALT_STRUCT, idx.reshape(-1)).reshape(-1, k)
        cand = np.minimum((u * cols).astype(np.int64), cols - 1)
        cand.sort(axis=1)
        dup = (np.diff(cand, axis=1) == 0).any(axis=1) if k > 1 else np.zeros(cand.shape[0], bool)
        ok = ~dup
        out[todo[ok]] = cand[ok]
        todo = todo[dup]
        rnd += 1
    row_ptr = (np.arange(rows + 1, dtype=np.int64) * k)
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("input nnz exceeds int32 indexing")
    col = out.reshape(-1).astype(np.int32)
    return CSR(rows, cols, row_ptr.astype(np.int32), col, _values(seed, col.shape[0], dtype))


def random_sparse(rows: int, cols: int, density: float, seed: int, dtype=np.float64) -> CSR:
    """Bernoulli(density) structure, for small test shapes."""
    u = uniform01(seed ^ SALT_STRUCT, 0, rows * cols).reshape(rows, cols) if rows * cols else np.zeros((rows, cols))
    r, c = np.nonzero(u < density)
    return csr_from_coo(rows, cols, r, c, seed, dtype)


def identity(n: int, dtype=np.float64) -> CSR:
    return CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, dtype=dtype))


def permutation(n: int, seed: int, dtype=np.float64) -> CSR:
    """Permutation matrix P with P[i, perm[i]] = 1, perm a seeded shuffle."""
    perm = np.argsort(uniform01(seed ^ SALT_STRUCT, 0, n), kind="stable").astype(np.int32)
    return CSR(n, n, np.arange(n + 1, dtype=np.int32), perm, np.ones(n, dtype=dtype))


def diagonal(n: int, seed: int, dtype=np.float64) -> CSR:
    return CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), _values(seed, n, dtype))


def empty(rows: int, cols: int, dtype=np.float64) -> CSR:
    return CSR(rows, cols, np.zeros(rows + 1, dtype=np.int32), np.zeros(0, np.int32), np.zeros(0, dtype))


def strided_columns(rows: int, cols: int, k: int, stride: int, seed: int, dtype=np.float32) -> CSR:
    """Every row holds k columns that are multiples of ``stride`` (all share
    their low bits), with a seeded offset per row: an adversarial pattern for
    a hash on low-order bits."""
    slots = max(1, cols // stride)
    k = min(k, slots)
    start = (uniform01(seed ^ SALT_STRUCT, 0, rows) * slots).astype(np.int64)
    j = ((start[:, None] + np.arange(k)[None, :]) % slots) * stride
    j.sort(axis=1)
    r = np.repeat(np.arange(rows, dtype=np.int64), k)
    return csr_from_coo(rows, cols, r, j.reshape(-1), seed, dtype)


def dense_rows(rows: int, cols: int, which, seed: int, dtype=np.float32) -> CSR:
    """Rows listed in ``which`` are fully dense; the others are empty."""
    which = np.asarray(sorted(set(int(w) for w in which)), dtype=np.int64)
    r = np.repeat(which, cols)
    c = np.tile(np.arange(cols, dtype=np.int64), which.shape[0])
    return csr_from_coo(rows, cols, r, c, seed, dtype)


# ---------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    B: CSR


def workload_small(dtype=np.float32) -> Workload:
    """RMAT scale 10, edge factor 8, C = A.A (seed 0x5EED0101)."""
    A = rmat(10, 8, 0x5EED0101, dtype)
    return Workload("rmat_s10_ef8_AxA", A, A)


def workload_s16(dtype=np.float32) -> Workload:
    """RMAT scale 16, edge factor 16, C = A.A (seed 0x5EED0201)."""
    A = rmat(16, 16, 0x5EED0201, dtype)
    return Workload("rmat_s16_ef16_AxA", A, A)


def workload_s19(dtype=np.float32) -> Workload:
    """RMAT scale 19, edge factor 16, C = A.A (seed 0x5EED0301)."""
    A = rmat(19, 16, 0x5EED0301, dtype)
    return Workload("rmat_s19_ef16_AxA", A, A)


def workload_rect(dtype=np.float32) -> Workload:
    """RMAT scale 21, edge factor 8, times a 2^21 x 4096 matrix with 16
    distinct uniform columns per row (seed 0x5EED0501)."""
    A = rmat(21, 8, 0x5EED0501, dtype)
    B = uniform_k_per_row(1 << 21, 4096, 16, 0x5EED0501 ^ 0xB, dtype)
    return Workload("rmat_s21_ef8_x_uniform4096k16", A, B)


def batch_shapes(count: int = 512, seed: int = 0x5EED0400):
    """(n_i, edge_factor_i) of the batched workload: n_i log-uniform in
    [256, 32768] (rounded), edge factor uniform on {4, ..., 32}."""
    u = uniform01(seed ^ SALT_SHAPE, 0, 2 * count).reshape(count, 2)
    n = np.rint(np.exp(np.log(256.0) + u[:, 0] * (np.log(32768.0) - np.log(256.0)))).astype(np.int64)
    ef = 4 + np.minimum((u[:, 1] * 29).astype(np.int64), 28)
    return [(int(a), int(b)) for a, b in zip(n, ef)]


def workload_batch(count: int = 512, dtype=np.float32, seed0: int = 0x5EED0400):
    """The batched workload: C_i = A_i . B_i, A_i an n_i x n_i RMAT matrix
    (rejection at scale ceil(log2 n_i)), B_i n_i x n_i with 8 distinct
    uniform columns per row; problem i uses seed ``seed0 + i``."""
    from concurrent.futures import ThreadPoolExecutor
    shapes = batch_shapes(count, seed0)

    def one(i):
        n, ef = shapes[i]
        s = seed0 + i
        A = rmat_rect(n, ef, s, dtype)
        B = uniform_k_per_row(n, n, 8, s ^ 0xB, dtype)
        return Workload(f"batch{i}_n{n}_ef{ef}", A, B)

    # problems are independent; numpy releases the GIL in the bulk of the work
    with ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        return list(ex.map(one, range(count)))


# ---------------------------------------------------------------- predictor

MLP_FEATURES = 6
MLP_HIDDEN = 64
# packed parameter layout shared by every implementation of the row-size MLP:
# W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3
MLP_LAYOUT = (("W1", (MLP_HIDDEN, MLP_FEATURES)), ("b1", (MLP_HIDDEN,)), ("W2", (MLP_HIDDEN, MLP_HIDDEN)),
              ("b2", (MLP_HIDDEN,)), ("w3", (MLP_HIDDEN,)), ("b3", (1,)))
MLP_PARAMS = sum(int(np.prod(s)) for _, s in MLP_LAYOUT)


def normal01(seed: int, start: int, count: int) -> np.ndarray:
    """Standard normal draws by Box-Muller from two SplitMix64 uniforms."""
    u = uniform01(seed, 2 * start, 2 * count).reshape(count, 2)
    u1 = np.maximum(u[:, 0], 2.0 ** -53)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u[:, 1])


def mlp_init(seed: int = 0x11A7) -> np.ndarray:
    """He initialisation of the packed MLP parameters (float64): weights
    N(0, 2 / fan_in), biases zero."""
    out = []
    pos = 0
    for name, shape in MLP_LAYOUT:
        n = int(np.prod(shape))
        if name.startswith("b"):
            out.append(np.zeros(n))
        else:
            fan_in = shape[-1] if len(shape) == 2 else MLP_HIDDEN
            out.append(normal01(seed, pos, n) * np.sqrt(2.0 / fan_in))
        pos += n
    return np.concatenate(out)


def batch_orders(n: int, epochs: int, seed: int = 0x0DE5) -> np.ndarray:
    """One seeded permutation of range(n) per epoch (int32, epochs x n)."""
    return np.stack([np.argsort(uniform01(seed + e, 0, n), kind="stable") for e in range(epochs)]).astype(np.int32)
