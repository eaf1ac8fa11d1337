"""The seeded input generators: published SplitMix64 values, determinism and
the structural properties each workload promises."""
import hashlib

import numpy as np

import synthetic as syn


def _digest(M):
    h = hashlib.sha256()
    h.update(M.row_ptr.tobytes()); h.update(M.col_idx.tobytes()); h.update(M.val.tobytes())
    return h.hexdigest()[:16]


def test_splitmix64_reference_values():
    # The first outputs of SplitMix64 seeded with 0 (Steele et al. 2014).
    assert syn.splitmix64(0, 0, 3).tolist() == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # counter-based: any slice equals the same slice of the full stream
    assert np.array_equal(syn.splitmix64(7, 5, 10), syn.splitmix64(7, 0, 15)[5:])


def test_rmat_deterministic_and_canonical(oracle_mod):
    A = syn.rmat(10, 8, 0x5EED0101)
    assert _digest(A) == "e86c8c0ed838926e" and A.nnz == 6640
    assert oracle_mod.validate(A) == 0
    assert A.val.dtype == np.float32 and np.all(np.abs(A.val) <= 1.0)


def test_rmat_quadrant_frequencies():
    r, c = syn.rmat_coo(12, 200000, 3)
    top_r = (r >> 11) & 1
    top_c = (c >> 11) & 1
    # P(row bit) = c + d = 0.24, P(col bit) = b + d = 0.24, P(both) = d = 0.05
    assert abs(top_r.mean() - 0.24) < 0.005
    assert abs(top_c.mean() - 0.24) < 0.005
    assert abs((top_r & top_c).mean() - 0.05) < 0.003


def test_uniform_k_per_row(oracle_mod):
    B = syn.uniform_k_per_row(1000, 64, 16, 3)
    assert oracle_mod.validate(B) == 0
    assert np.all(np.diff(B.row_ptr) == 16)
    assert _digest(syn.uniform_k_per_row(100, 50, 8, 3)) == "58739cb8bd51308d"


def test_rmat_rect_bounds(oracle_mod):
    A = syn.rmat_rect(1990, 4, 17)
    assert A.rows == A.cols == 1990 and oracle_mod.validate(A) == 0
    assert A.nnz <= 4 * 1990


def test_batch_shapes():
    sh = syn.batch_shapes(512)
    assert len(sh) == 512
    assert all(256 <= n <= 32768 and 4 <= ef <= 32 for n, ef in sh)
    assert sh[:3] == [(1990, 30), (465, 7), (772, 30)]


def test_structured_generators(oracle_mod):
    for M in (syn.identity(7), syn.permutation(9, 1), syn.diagonal(5, 2), syn.empty(3, 4),
              syn.strided_columns(20, 4096, 12, 256, 5), syn.dense_rows(8, 300, [1, 5], 6)):
        assert oracle_mod.validate(M) == 0
    S = syn.strided_columns(20, 4096, 12, 256, 5)
    assert np.all(S.col_idx % 256 == 0)
