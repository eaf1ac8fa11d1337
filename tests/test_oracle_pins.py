"""Pins for the CPU oracle against things other than itself.

- dense brute force (numpy long-double and float64 matmul of the dense
  operands) on every small shape: the definition c_ij = sum_k a_ik b_kj
  (Background chapter, eq. "inner_product");
- scipy.sparse's independent SpGEMM on RMAT inputs;
- exact identities (A I = A, I A = A, permutations, diagonal scaling) and the
  transpose identity (A B)^T = B^T A^T, bitwise;
- structural bounds and the product count of the Window Distribution Phase;
- Freivalds' randomized check on a larger RMAT product.
Rectangular shapes catch a transposed operand, signed values catch a dropped
sign, and absmass/term checks catch a dropped or doubled term.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synthetic as syn


def _dense_ref(A, B, oracle):
    DA = oracle.to_dense(A, np.longdouble)
    DB = oracle.to_dense(B, np.longdouble)
    PA = (oracle.to_dense(A) != 0).astype(np.int64) if A.nnz else np.zeros((A.rows, A.cols), np.int64)
    PB = np.zeros((B.rows, B.cols), np.int64)
    rows_of = np.repeat(np.arange(B.rows), np.diff(B.row_ptr.astype(np.int64)))
    PB[rows_of, B.col_idx] = 1
    PA = np.zeros((A.rows, A.cols), np.int64)
    rows_a = np.repeat(np.arange(A.rows), np.diff(A.row_ptr.astype(np.int64)))
    PA[rows_a, A.col_idx] = 1
    terms = PA @ PB                                   # number of k with a_ik, b_kj stored
    val = DA @ DB
    absm = np.abs(DA) @ np.abs(DB)
    return terms, val, absm


def _expand(C, rows, cols):
    rows_of = np.repeat(np.arange(rows), np.diff(C["row_ptr"]))
    return rows_of, C["col"]


CASES = []
for s in range(40):
    u = syn.uniform01(0xC0FFEE + s, 0, 4)
    m = 1 + int(u[0] * 64)
    k = 1 + int(u[1] * 64)
    n = 1 + int(u[2] * 64)
    dens = [0.0, 0.02, 0.1, 0.3, 0.9][s % 5] if s >= 5 else 0.15
    CASES.append((m, k, n, dens, 1000 + s))
CASES += [(1, 1, 1, 1.0, 1), (64, 64, 64, 0.05, 2), (3, 64, 1, 0.5, 3), (64, 1, 64, 0.5, 4)]


@pytest.mark.parametrize("m,k,n,dens,seed", CASES)
def test_dense_brute_force(oracle_mod, m, k, n, dens, seed):
    A = syn.random_sparse(m, k, dens, seed, np.float64)
    B = syn.random_sparse(k, n, min(1.0, dens * 1.5), seed + 7, np.float64)
    C = oracle_mod.spgemm(A, B)
    terms, val, absm = _dense_ref(A, B, oracle_mod)
    ri, cj = _expand(C, m, n)
    # structure: exactly the (i, j) with at least one contributing k, sorted
    want_r, want_c = np.nonzero(terms > 0)
    assert np.array_equal(ri, want_r) and np.array_equal(cj, want_c)
    assert np.array_equal(C["terms"], terms[want_r, want_c])
    np.testing.assert_allclose(C["absmass"], absm[want_r, want_c].astype(np.float64), rtol=1e-15, atol=0)
    err = np.abs(C["val"].astype(np.longdouble) - val[want_r, want_c])
    assert np.all(err <= 2.3e-16 * absm[want_r, want_c] + 1e-300)
    # the float64 library matmul agrees to its own rounding bound
    d64 = oracle_mod.to_dense(A) @ oracle_mod.to_dense(B)
    assert np.all(np.abs(C["val"] - d64[want_r, want_c]) <= 64 * 2.3e-16 * absm[want_r, want_c].astype(np.float64))


def test_structural_zero_is_kept(oracle_mod):
    # A = [1 1], B = [1; -1]: the single entry cancels to 0.0 but stays stored.
    A = syn.CSR(1, 2, np.array([0, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    B = syn.CSR(2, 1, np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32), np.array([1.0, -1.0]))
    C = oracle_mod.spgemm(A, B)
    assert list(C["row_ptr"]) == [0, 1] and list(C["col"]) == [0]
    assert C["val"][0] == 0.0 and C["absmass"][0] == 2.0 and C["terms"][0] == 2


def test_empty_and_degenerate(oracle_mod):
    A = syn.empty(5, 7)
    B = syn.random_sparse(7, 3, 0.5, 9)
    C = oracle_mod.spgemm(A, B)
    assert C["row_ptr"].tolist() == [0] * 6 and C["col"].size == 0
    C = oracle_mod.spgemm(syn.empty(0, 4), syn.random_sparse(4, 4, 0.5, 1))
    assert C["row_ptr"].tolist() == [0]
    C = oracle_mod.spgemm(syn.random_sparse(3, 0, 0.5, 1), syn.empty(0, 5))
    assert C["row_ptr"].tolist() == [0, 0, 0, 0]


@pytest.fixture(scope="module")
def rmat12():
    return syn.rmat(12, 8, 0x1234, np.float64)


def test_scipy_independent_spgemm(oracle_mod, rmat12):
    A = rmat12
    B = syn.uniform_k_per_row(A.cols, 3000, 5, 77, np.float64)   # rectangular
    C = oracle_mod.spgemm(A, B)
    SA = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    SB = sp.csr_matrix((B.val, B.col_idx, B.row_ptr), shape=(B.rows, B.cols))
    SC = (SA @ SB).tocsr()
    SC.sort_indices()
    # random values: no exact cancellation, so scipy's pruning of zeros is moot
    assert np.array_equal(SC.indptr.astype(np.int64), C["row_ptr"])
    assert np.array_equal(SC.indices, C["col"])
    assert np.all(np.abs(SC.data - C["val"]) <= 1e-13 * C["absmass"])


def test_identities_bitwise(oracle_mod, rmat12):
    A = rmat12
    n = A.rows
    I = syn.identity(n)
    for C in (oracle_mod.spgemm(A, I), oracle_mod.spgemm(I, A)):
        assert np.array_equal(C["row_ptr"], A.row_ptr.astype(np.int64))
        assert np.array_equal(C["col"], A.col_idx)
        assert np.array_equal(C["val"], A.val)
    # P A permutes rows: row i of PA is row perm[i] of A
    P = syn.permutation(n, 5)
    perm = P.col_idx.astype(np.int64)
    C = oracle_mod.spgemm(P, A)
    rp = A.row_ptr.astype(np.int64)
    want_c = np.concatenate([A.col_idx[rp[p]:rp[p + 1]] for p in perm])
    want_v = np.concatenate([A.val[rp[p]:rp[p + 1]] for p in perm])
    assert np.array_equal(C["col"], want_c) and np.array_equal(C["val"], want_v)
    # A P relabels columns: column j of A moves to inv... A P [i, perm[j']] ... A[i,k] P[k, perm[k]]
    C = oracle_mod.spgemm(A, P)
    dense = oracle_mod.to_dense(A)
    want = np.zeros_like(dense)
    want[:, perm] = dense
    got = np.zeros_like(dense)
    got[np.repeat(np.arange(n), np.diff(C["row_ptr"])), C["col"]] = C["val"]
    assert np.array_equal(got, want)
    # D A scales row i by d_i: one product per entry, rounded once
    D = syn.diagonal(n, 11)
    C = oracle_mod.spgemm(D, A)
    rows_of = np.repeat(np.arange(n), np.diff(rp))
    assert np.array_equal(C["col"], A.col_idx)
    assert np.array_equal(C["val"], D.val[rows_of] * A.val)


def test_transpose_identity_bitwise(oracle_mod, rmat12):
    A = rmat12
    B = syn.rmat(12, 4, 0x99, np.float64)
    C = oracle_mod.spgemm(A, B)
    Ct = oracle_mod.spgemm(oracle_mod.transpose(B), oracle_mod.transpose(A))
    CC = syn.CSR(A.rows, B.cols, C["row_ptr"].astype(np.int32), C["col"], C["val"])
    T = oracle_mod.transpose(CC)
    assert np.array_equal(T.row_ptr.astype(np.int64), Ct["row_ptr"])
    assert np.array_equal(T.col_idx, Ct["col"])
    assert np.array_equal(T.val, Ct["val"])          # same products, same order


def test_bounds_and_product_count(oracle_mod, rmat12):
    A = rmat12
    C = oracle_mod.spgemm(A, A)
    ub = oracle_mod.products_per_row(A, A)
    nnz = np.diff(C["row_ptr"])
    assert int(C["terms"].sum()) == int(ub.sum())           # every product merged once
    bdeg = np.diff(A.row_ptr.astype(np.int64))
    rp = A.row_ptr.astype(np.int64)
    for i in range(A.rows):
        if rp[i + 1] == rp[i]:
            assert nnz[i] == 0
            continue
        lo = bdeg[A.col_idx[rp[i]:rp[i + 1]]].max()
        assert lo <= nnz[i] <= min(ub[i], A.cols)
    # |c| <= absmass up to absmass's own double rounding (m terms)
    assert np.all(np.abs(C["val"]) <= C["absmass"] * (1 + C["terms"] * 2.3e-16))
    # explicit brute-force loop for the product count on a few rows
    for i in (0, 1, 7, 100):
        assert ub[i] == sum(bdeg[k] for k in A.col_idx[rp[i]:rp[i + 1]])


def test_row_selection_matches_full(oracle_mod, rmat12):
    A = rmat12
    full = oracle_mod.spgemm(A, A)
    sel = np.array([4000, 3, 3, 0, 2047], np.int64)
    part = oracle_mod.spgemm(A, A, rows=sel)
    for t, i in enumerate(sel):
        a, b = full["row_ptr"][i], full["row_ptr"][i + 1]
        c, d = part["row_ptr"][t], part["row_ptr"][t + 1]
        assert np.array_equal(full["col"][a:b], part["col"][c:d])
        assert np.array_equal(full["val"][a:b], part["val"][c:d])


def test_freivalds(oracle_mod):
    A = syn.rmat(13, 8, 0x4242, np.float64)
    C = oracle_mod.spgemm(A, A)
    SA = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.rows, A.cols))
    SC = sp.csr_matrix((C["val"], C["col"], C["row_ptr"]), shape=(A.rows, A.cols))
    absA = abs(SA)
    for s in range(3):
        x = 2 * syn.uniform01(0xF00 + s, 0, A.cols) - 1
        lhs = SC @ x
        rhs = SA @ (SA @ x)
        bound = absA @ (absA @ np.abs(x))
        assert np.all(np.abs(lhs - rhs) <= 1e-12 * bound + 1e-300)


def test_validate_codes(oracle_mod):
    good = syn.random_sparse(4, 5, 0.5, 3)
    assert oracle_mod.validate(good) == 0
    bad = syn.CSR(2, 3, np.array([1, 1, 2], np.int32), np.array([0, 1], np.int32), np.ones(2))
    assert oracle_mod.validate(bad) == 1
    bad = syn.CSR(2, 3, np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32), np.ones(2))
    assert oracle_mod.validate(bad) == 2
    bad = syn.CSR(1, 3, np.array([0, 2], np.int32), np.array([0, 3], np.int32), np.ones(2))
    assert oracle_mod.validate(bad) == 3
    bad = syn.CSR(1, 3, np.array([0, 2], np.int32), np.array([1, 1], np.int32), np.ones(2))
    assert oracle_mod.validate(bad) == 4
    bad = syn.CSR(1, 3, np.array([0, 2], np.int32), np.array([2, 1], np.int32), np.ones(2))
    assert oracle_mod.validate(bad) == 4
