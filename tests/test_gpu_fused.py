"""GPU parity of the fused single pass (smash_spgemm_fused) against the oracle.

The fused pass must give the same canonical C as the two-phase path whatever
the predictor says: rows it sizes correctly are finished in one kernel, rows
it under-sizes overflow and are recomputed exactly, rows it sizes above the
LDS limit never enter it.  Checked with the shipped predictor, with
capacities forced far too small (every row overflows or nearly so) and far
too large (clamped to the exact upper bound), and on edge cases.  The last
test measures the shipped predictor on a matrix outside its training set.
"""
import numpy as np
import pytest

import synthetic as syn
from tests._parity import check_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_14156_amd import predictor, smash
    assert torch.cuda.is_available()
    ctx = smash.Context(0)
    ctx.predictor_load()
    params, ms, delta = predictor.load(predictor.DEFAULT_PATH)
    yield torch, smash, ctx, (params, ms, delta)
    ctx.close()


def fused_check(env, A, B, dtype, oracle_mod, where):
    torch, smash, ctx, _ = env
    A = A.astype(dtype)
    B = A if B is None else B.astype(dtype)
    dA = smash.to_device(A)
    dB = dA if B is A else smash.to_device(B)
    C = ctx.spgemm_fused(dA, dB)
    st = ctx.stats()
    ref = oracle_mod.spgemm(A, B)
    check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), ref, dtype, where)
    return st


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fused_rmat_s10(env, oracle_mod, dtype):
    st = fused_check(env, syn.workload_small().A, None, dtype, oracle_mod, "fused s10")
    assert st["fused_rows"] > 0.8 * (st["rows"] - st["rows_empty"] - st["rows_heavy"])


def test_fused_rmat_s14_ef16(env, oracle_mod):
    A = syn.rmat(14, 16, 0x5EED0601, np.float32)
    st = fused_check(env, A, None, np.float32, oracle_mod, "fused s14")
    assert st["fused_rows"] > 0 and st["rows_heavy"] > 0


def test_fused_rectangular(env, oracle_mod):
    A = syn.rmat(12, 8, 0x5EED0602, np.float32)
    B = syn.uniform_k_per_row(A.cols, 1000, 9, 0x5EED0603, np.float32)
    fused_check(env, A, B, np.float32, oracle_mod, "fused rect")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fused_with_global_heavy_rows(env, oracle_mod, dtype):
    """The fused pass beside the global-hash heavy-row path, its tables
    processed in waves under a small pool."""
    torch, smash, ctx, _ = env
    ctx.set_option(smash.OPT_HEAVY_MODE, 1)
    ctx.set_option(smash.OPT_GLOBAL_POOL, 1 << 14)
    try:
        st = fused_check(env, syn.rmat(13, 16, 0x5EED0608, np.float32), None, dtype, oracle_mod, "fused + global")
        assert st["fused_rows"] > 0 and st["rows_heavy"] > 0 and st["global_waves"] > 2
    finally:
        ctx.set_option(smash.OPT_HEAVY_MODE, 0)
        ctx.set_option(smash.OPT_GLOBAL_POOL, 0)


def test_fused_capacity_too_small(env, oracle_mod):
    """delta = -6 shrinks every predicted capacity 64-fold: nearly every
    fused row overflows and goes through the exact path."""
    torch, smash, ctx, (params, ms, delta) = env
    ctx.predictor_set(params, ms, -6.0)
    try:
        A = syn.rmat(12, 16, 0x5EED0604, np.float32)
        st = fused_check(env, A, None, np.float32, oracle_mod, "fused delta -6")
        assert st["fused_overflow"] > st["fused_rows"]
    finally:
        ctx.predictor_set(params, ms, delta)


def test_fused_capacity_too_large(env, oracle_mod):
    """delta = +20: capacities clamp to min(products, columns); every row
    with at most LDS-limit products is fused, none overflows."""
    torch, smash, ctx, (params, ms, delta) = env
    ctx.predictor_set(params, ms, 20.0)
    try:
        A = syn.rmat(12, 16, 0x5EED0605, np.float32)
        st = fused_check(env, A, None, np.float32, oracle_mod, "fused delta +20")
        assert st["fused_overflow"] == 0
        ub = np.asarray(oracle_mod.products_per_row(A, A))
        fused = (ub > 0) & (np.minimum(ub, A.cols) <= 1024)
        assert st["fused_rows"] == int(fused.sum())
        # entries of the fused rows (exact, from the oracle's row counts) and
        # the capacity reserved for them: min(products, columns) per row
        assert st["fused_entries"] == int(oracle_mod.row_nnz(A, A)[fused].sum())
        assert st["fused_capacity"] == int(np.minimum(ub, A.cols)[fused].sum())
    finally:
        ctx.predictor_set(params, ms, delta)


@pytest.mark.parametrize("case", ["empty", "no_rows", "identity", "dense_rows", "strided"])
def test_fused_edge_cases(env, oracle_mod, case):
    if case == "empty":
        A, B = syn.empty(300, 200, np.float32), syn.random_sparse(200, 50, 0.1, 3, np.float32)
    elif case == "no_rows":
        A, B = syn.empty(0, 40, np.float32), syn.random_sparse(40, 30, 0.2, 4, np.float32)
    elif case == "identity":
        A, B = syn.identity(777, np.float32), syn.random_sparse(777, 333, 0.02, 5, np.float32)
    elif case == "dense_rows":
        A, B = syn.dense_rows(64, 2000, [0, 7, 63], 6, np.float32), syn.random_sparse(2000, 1500, 0.003, 7,
                                                                                        np.float32)
    else:
        A = syn.strided_columns(500, 1 << 16, 40, 1024, 8, np.float32)
        B = syn.strided_columns(1 << 16, 1 << 16, 8, 512, 9, np.float32)
    fused_check(env, A, B, np.float32, oracle_mod, f"fused {case}")


def test_fused_requires_predictor(env):
    torch, smash, ctx, _ = env
    other = smash.Context(0)
    try:
        dA = smash.to_device(syn.identity(16, np.float32))
        with pytest.raises(smash.SmashError):
            other.spgemm_fused(dA, dA)
    finally:
        other.close()


def test_shipped_predictor_quality(env, oracle_mod):
    """On RMAT scale 16, edge factor 16 (a seed outside the training set) the
    shipped predictor fuses at least 90% of the rows it may fuse, and at
    most 5% of the fused attempts overflow."""
    torch, smash, ctx, _ = env
    A = syn.rmat(16, 16, 0x5EED0607, np.float32)
    dA = smash.to_device(A)
    C = ctx.spgemm_fused(dA, dA)
    st = ctx.stats()
    nz = oracle_mod.row_nnz(A, A)
    assert np.array_equal(np.diff(C.row_ptr.cpu().numpy()), nz)
    ub = np.asarray(oracle_mod.products_per_row(A, A))
    eligible = int(((ub > 0) & (nz <= 1024)).sum())
    attempts = st["fused_rows"] + st["fused_overflow"]
    print(f"eligible {eligible} fused {st['fused_rows']} overflow {st['fused_overflow']}", flush=True)
    assert st["fused_rows"] >= 0.9 * eligible
    assert st["fused_overflow"] <= 0.05 * attempts


def test_learned_sizing_gain(env, oracle_mod):
    """What the trained network gains over the method without it (exact
    upper-bound capacities min(products, columns)): on RMAT scale 16, edge
    factor 16 some rows have more than 1024 products but at most 1024
    entries; the upper bound sends them to the heavy-row path, the network
    sizes them into LDS, so the learned pass completes more rows in one
    pass.  Both passes give the exact C."""
    torch, smash, ctx, _ = env
    A = syn.rmat(16, 16, 0x5EED0607, np.float32)
    dA = smash.to_device(A)
    ub = np.asarray(oracle_mod.products_per_row(A, A))
    nz = oracle_mod.row_nnz(A, A)
    by_bound = int(((ub > 0) & (np.minimum(ub, A.cols) <= 1024)).sum())
    recoverable = int(((np.minimum(ub, A.cols) > 1024) & (nz <= 1024)).sum())
    got = {}
    try:
        for sizing in (1, 0):
            ctx.set_option(smash.OPT_FUSED_SIZING, sizing)
            C = ctx.spgemm_fused(dA, dA)
            assert np.array_equal(np.diff(C.row_ptr.cpu().numpy()), nz)
            got[sizing] = ctx.stats()
    finally:
        ctx.set_option(smash.OPT_FUSED_SIZING, 0)
    ln, bd = got[0], got[1]
    print(f"upper bound: fused {bd['fused_rows']} (of {by_bound} it may fuse); learned: fused {ln['fused_rows']}, "
          f"overflow {ln['fused_overflow']}; rows only the network can fuse: {recoverable}", flush=True)
    assert bd["fused_rows"] == by_bound and bd["fused_overflow"] == 0
    assert ln["fused_rows"] > bd["fused_rows"]
