"""GPU parity of the fused single pass (smash_spgemm_fused) against the oracle.

The fused pass must give the same canonical C as the two-phase path whatever
the predictor says: rows whose exact bound min(products, columns) fits the
LDS tables are finished in one kernel with that bound as their capacity;
rows above it are sized by the network: those it sizes correctly are
finished in one kernel too, those it under-sizes overflow and are recomputed
exactly, those it sizes above the LDS limit never enter it.  Checked with the
shipped predictor, with capacities forced far too small (every row the
network sizes overflows or nearly so) and far too large (clamped to the
exact upper bound), and on edge cases.  The last tests measure the shipped
predictor on products outside its training set and what it gains.
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
    """delta = -6 shrinks every predicted capacity 64-fold: nearly every row
    the network sizes overflows and goes through the exact path; the rows
    within the LDS limit keep their exact bound and are all fused."""
    torch, smash, ctx, (params, ms, delta) = env
    ctx.predictor_set(params, ms, -6.0)
    try:
        A = syn.rmat(12, 16, 0x5EED0604, np.float32)
        st = fused_check(env, A, None, np.float32, oracle_mod, "fused delta -6")
        ub = np.asarray(oracle_mod.products_per_row(A, A))
        by_bound = int(((ub > 0) & (np.minimum(ub, A.cols) <= 1024)).sum())
        assert st["fused_rows"] >= by_bound
        assert st["fused_overflow"] > 10 * (st["fused_rows"] - by_bound)
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


def _loose_bound_product():
    """RMAT scale 14 (edge factor 16) times a 14,000 x 1,500 uniform matrix
    with 24 entries per row: rows of 43 or more A entries have more than
    1024 products, but the 1,500 columns saturate, so many of them have at
    most 1024 entries."""
    A = syn.rmat(14, 16, 0x5EED0609, np.float32)
    B = syn.uniform_k_per_row(A.cols, 1500, 24, 0x5EED060A, np.float32)
    return A, B


def test_learned_sizing_gain(env, oracle_mod):
    """What the trained network gains over the method without it (exact
    upper-bound capacities min(products, columns)) where that bound is loose:
    the rows with more than 1024 products but at most 1024 entries can only
    be finished in the fused pass from a prediction; with the bound they take
    the heavy-row path (a symbolic count over column chunks, then dense or
    hashed chunk accumulation).  The network must fuse most of them, leaving
    fewer rows and products to the heavy-row path; both passes give the
    exact C.  The times of both passes are printed."""
    torch, smash, ctx, _ = env
    A, B = _loose_bound_product()
    dA, dB = smash.to_device(A), smash.to_device(B)
    ub = np.asarray(oracle_mod.products_per_row(A, B))
    nz = oracle_mod.row_nnz(A, B)
    bound = np.minimum(ub, B.cols)
    by_bound = int(((ub > 0) & (bound <= 1024)).sum())
    recoverable = (bound > 1024) & (nz <= 1024)
    ref = oracle_mod.spgemm(A, B)
    got, ms = {}, {}
    try:
        for sizing in (1, 0):
            ctx.set_option(smash.OPT_FUSED_SIZING, sizing)
            C = ctx.spgemm_fused(dA, dB)
            check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), ref, np.float32,
                       f"fused sizing {sizing}")
            got[sizing] = ctx.stats()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                C = ctx.spgemm_fused(dA, dB)
            e1.record()
            torch.cuda.synchronize()
            ms[sizing] = e0.elapsed_time(e1) / 5
    finally:
        ctx.set_option(smash.OPT_FUSED_SIZING, 0)
    ln, bd = got[0], got[1]
    heavy_ub = int(ub[bound > 1024].sum())
    print(f"upper bound: fused {bd['fused_rows']} (of {by_bound}), heavy rows {bd['rows_heavy']}, {ms[1]:.3f} ms; "
          f"learned: fused {ln['fused_rows']}, overflow {ln['fused_overflow']}, heavy rows {ln['rows_heavy']}, "
          f"{ms[0]:.3f} ms; rows only the network can fuse: {int(recoverable.sum())} "
          f"({int(ub[recoverable].sum())} of the {heavy_ub} heavy-row products)", flush=True)
    assert bd["fused_rows"] == by_bound and bd["fused_overflow"] == 0
    assert bd["rows_heavy"] == int((bound > 1024).sum())
    moved = bd["rows_heavy"] - ln["rows_heavy"]
    assert ln["fused_rows"] - bd["fused_rows"] == moved
    assert moved >= 0.5 * int(recoverable.sum()), "the network fused fewer than half of the recoverable rows"
