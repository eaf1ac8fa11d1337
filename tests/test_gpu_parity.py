"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Structure bit-exact, values within 1e-5 (FP32) / 1e-12 (FP64) of the sum of
|a_ik b_kj| per entry, single-term entries bitwise (see tests/_parity.py).
Workloads: RMAT scale 10 (edge factor 8) and scale 16 (edge factor 16) C = A.A,
both heavy-row strategies, both row-table hashes, forced heavy rows,
rectangular and structured edge cases, subnormal and cancelling sums on
every accumulation path.
"""
import numpy as np
import pytest

import synthetic as syn
from tests._parity import check_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch


@pytest.fixture(scope="module")
def sm(torch_mod):
    from paper_2105_14156_amd import smash
    return smash


@pytest.fixture()
def ctx(sm):
    c = sm.Context(0)
    yield c
    c.close()


def run(sm, ctx, A, B, dtype, split=False):
    dA = sm.to_device(A, dtype=dtype)
    dB = dA if B is A else sm.to_device(B, dtype=dtype)
    if split:
        import torch
        rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
        nnz = ctx.symbolic(dA, dB, rp)
        col = torch.empty(nnz, dtype=torch.int32, device="cuda")
        val = torch.empty(nnz, dtype=dA.val.dtype, device="cuda")
        ctx.numeric(dA, dB, rp, col, val)
        return rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    C = ctx.spgemm(dA, dB)
    return C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy()


def full_check(sm, ctx, A, B, dtype, oracle_mod, split=False, where=""):
    A = A.astype(dtype)
    B = A if B is None else B.astype(dtype)
    rp, col, val = run(sm, ctx, A, B, dtype, split)
    ref = oracle_mod.spgemm(A, B)
    return check_rows(rp, col, val, ref, dtype, where)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("split", [False, True])
def test_rmat_s10(sm, ctx, oracle_mod, dtype, split):
    w = syn.workload_small()
    full_check(sm, ctx, w.A, None, dtype, oracle_mod, split, "s10")
    st = ctx.stats()
    ub = oracle_mod.products_per_row(w.A, w.A)
    assert st["products"] == int(ub.sum())


@pytest.fixture(scope="module")
def s16():
    return syn.workload_s16().A


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rmat_s16(sm, ctx, oracle_mod, s16, dtype):
    full_check(sm, ctx, s16, None, dtype, oracle_mod, False, "s16")
    st = ctx.stats()
    assert st["rows_heavy"] > 0 and st["rows_lds"] > 0
    assert st["heavy_segments"] > 0 and st["heavy_dense_chunks"] > 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rmat_s16_global_hash(sm, ctx, oracle_mod, s16, dtype):
    ctx.set_option(sm.OPT_HEAVY_MODE, 1)
    full_check(sm, ctx, s16, None, dtype, oracle_mod, False, "s16 global")
    assert ctx.stats()["global_slots"] > 0


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("row_max", [32, 300])
def test_forced_heavy_rows(sm, ctx, oracle_mod, mode, row_max):
    # every row with more than row_max outputs takes the heavy-row path
    A = syn.rmat(13, 8, 0x77, np.float32)
    ctx.set_option(sm.OPT_LDS_ROW_MAX, row_max)
    ctx.set_option(sm.OPT_HEAVY_MODE, mode)
    for dtype in (np.float32, np.float64):
        full_check(sm, ctx, A, None, dtype, oracle_mod, False, f"forced heavy mode={mode} row_max={row_max}")
        assert ctx.stats()["rows_heavy"] > 100


@pytest.mark.parametrize("limit", [1, 1 << 15])
def test_global_hash_waves(sm, ctx, oracle_mod, limit):
    """Global mode with a bounded table pool: heavy rows run in waves of
    consecutive rows whose tables fit (limit 1: every row alone, the pool
    grows to the largest single table), in both phases."""
    A = syn.rmat(13, 8, 0x77, np.float32)
    ctx.set_option(sm.OPT_LDS_ROW_MAX, 64)
    ctx.set_option(sm.OPT_HEAVY_MODE, 1)
    full_check(sm, ctx, A, None, np.float32, oracle_mod, False, "global, one wave")
    st0 = ctx.stats()
    assert st0["global_waves"] == 2 and st0["rows_heavy"] > 100
    ctx.set_option(sm.OPT_GLOBAL_POOL, limit)
    for dtype in (np.float32, np.float64):
        for split in (False, True):
            full_check(sm, ctx, A, None, dtype, oracle_mod, split, f"global waves limit={limit} split={split}")
            st = ctx.stats()
            assert st["global_waves"] > 2 and st["global_pool"] < st0["global_pool"]
            assert st["global_slots"] == st0["global_slots"]
            if limit == 1:
                assert st["global_waves"] == 2 * st["rows_heavy"]
            else:
                assert st["global_pool"] <= limit


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rectangular(sm, ctx, oracle_mod, dtype):
    A = syn.rmat(14, 8, 0x5EED0501, dtype)
    B = syn.uniform_k_per_row(A.cols, 4096, 16, 0xB, dtype)
    full_check(sm, ctx, A, B, dtype, oracle_mod, False, "rect")
    # and with more columns than one heavy-row window
    B = syn.uniform_k_per_row(A.cols, 100_000, 16, 0xC, dtype)
    ctx.set_option(sm.OPT_LDS_ROW_MAX, 64)
    full_check(sm, ctx, A, B, dtype, oracle_mod, False, "rect wide")


def test_structured_cases(sm, ctx, oracle_mod):
    n = 3000
    cases = {
        "identity_left": (syn.identity(n), syn.rmat(11, 4, 3, np.float64)),
        "permutation": (syn.permutation(2048, 4), syn.rmat(11, 4, 5, np.float64)),
        "diagonal_right": (syn.rmat(11, 4, 6, np.float64), syn.diagonal(2048, 7)),
        "adversarial_stride": (syn.rmat(11, 4, 8, np.float64), syn.strided_columns(2048, 1 << 20, 64, 1024, 9)),
        "dense_rows": (syn.dense_rows(64, 64, [0, 5, 63], 10, np.float64), syn.dense_rows(64, 20000, range(64), 11, np.float64)),
        "n_equals_1": (syn.random_sparse(500, 40, 0.3, 12), syn.random_sparse(40, 1, 0.5, 13)),
        "empty_A": (syn.empty(100, 50), syn.random_sparse(50, 60, 0.2, 14)),
        "empty_B": (syn.random_sparse(100, 50, 0.2, 15), syn.empty(50, 60)),
        "no_rows": (syn.empty(0, 50), syn.random_sparse(50, 60, 0.2, 16)),
    }
    for name, (A, B) in cases.items():
        if name == "identity_left":
            A = syn.identity(B.rows)
        for dtype in (np.float32, np.float64):
            full_check(sm, ctx, A.astype(dtype), B.astype(dtype), dtype, oracle_mod, False, name)


def test_cancellation_keeps_structural_zero(sm, ctx, oracle_mod):
    A = syn.CSR(2, 2, np.array([0, 2, 3], np.int32), np.array([0, 1, 1], np.int32), np.array([1.0, 1.0, 2.0]))
    B = syn.CSR(2, 3, np.array([0, 2, 4], np.int32), np.array([0, 2, 0, 2], np.int32), np.array([1.0, 3.0, -1.0, 5.0]))
    rp, col, val = run(sm, ctx, A, B, np.float64)
    assert rp.tolist() == [0, 2, 4] and col.tolist() == [0, 2, 0, 2]
    assert val.tolist() == [0.0, 8.0, -2.0, 10.0]


def _zero_product_case():
    """Rows whose products are all exactly +-0.0 (explicit zero and negative
    zero values in A), landing in dense chunks: 3 rows of A, each reaching
    two B rows of 3000 columns within one 8192-column chunk."""
    B = syn.uniform_k_per_row(8, 8192, 3000, 0x2E0, np.float64)
    rp = np.array([0, 2, 4, 6], np.int32)
    ci = np.array([0, 1, 2, 3, 4, 5], np.int32)
    va = np.array([0.0, -0.0, -0.0, -0.0, 0.5, -0.0])      # row 2 mixes a nonzero in
    A = syn.CSR(3, 8, rp, ci, va)
    return A, B


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_zero_products_keep_structure(sm, ctx, oracle_mod, dtype):
    A, B = _zero_product_case()
    ctx.set_option(sm.OPT_LDS_ROW_MAX, 64)
    rp, col, val = run(sm, ctx, A.astype(dtype), B.astype(dtype), dtype)
    assert ctx.stats()["heavy_dense_chunks"] > 0
    ref = oracle_mod.spgemm(A.astype(dtype), B.astype(dtype))
    check_rows(rp, col, val, ref, dtype, "zero products")
    assert np.all(val[: rp[2]] == 0.0)


def test_dense_chunk_denormal_and_cancelling_sums(sm, ctx, oracle_mod):
    """FP64 dense chunks mark occupancy by leaving -0.0: an entry whose sum
    is a negative subnormal, or cancels to zero, must keep its place and
    value (a flush of subnormals in the LDS add would drop it)."""
    n, width = 8192, 1500
    cols = np.arange(width, dtype=np.int32)
    b0 = np.ones(width)
    b1 = np.ones(width)
    b0[7], b1[7] = -1e-320, 0.0            # product -1e-320 (subnormal); b1 adds an exact zero
    b0[9], b1[9] = 1.0, -1.0               # cancels to +0.0
    b0[11], b1[11] = -5e-324, -5e-324      # smallest subnormal, twice
    B = syn.CSR(2, n, np.array([0, width, 2 * width], np.int32), np.concatenate([cols, cols]),
                np.concatenate([b0, b1]))
    A = syn.CSR(1, 2, np.array([0, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    rp, col, val = run(sm, ctx, A, B, np.float64)
    st = ctx.stats()
    assert st["heavy_dense_chunks"] == 1, st
    ref = oracle_mod.spgemm(A, B)
    assert np.array_equal(col, ref["col"]) and rp[-1] == width
    assert val[7] == -1e-320 and val[9] == 0.0 and val[11] == -1e-323
    check_rows(rp, col, val, ref, np.float64, "subnormal dense chunk")


def test_repeat_numeric_and_determinism(sm, ctx, oracle_mod, torch_mod):
    torch = torch_mod
    A = syn.rmat(14, 8, 0x99, np.float32)
    dA = sm.to_device(A)
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    nnz = ctx.symbolic(dA, dA, rp)
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=torch.float32, device="cuda")
    ctx.numeric(dA, dA, rp, col, val)
    col0 = col.clone()
    for _ in range(3):
        col.fill_(-7)
        ctx.numeric(dA, dA, rp, col, val)
        assert torch.equal(col, col0)
    # new values, same structure: the plan is reused
    A2 = syn.CSR(A.rows, A.cols, A.row_ptr, A.col_idx, (A.val * -0.5).astype(np.float32))
    dA.val.copy_(torch.from_numpy(A2.val))
    ctx.numeric(dA, dA, rp, col, val)
    check_rows(rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), oracle_mod.spgemm(A2, A2), np.float32, "revalued")


def _mutated(base, how):
    rp, ci = base.row_ptr.copy(), base.col_idx.copy()
    how(rp, ci)
    return syn.CSR(base.rows, base.cols, rp, ci, np.ones(ci.size, np.float32))


def test_validation_walk(sm, ctx, torch_mod):
    """Validation reads each wave's 64 rows as one range of entries, 64 at a
    time: violations inside long rows, at a window boundary, at a row start
    and in the row pointers of a later wave are caught; valid matrices with
    empty rows and row starts below the previous row's last column pass."""
    torch = torch_mod
    n = 300
    lens = np.where(np.arange(n) % 7 == 3, 0, 100)                      # some empty rows
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(syn.uniform_k_per_row(1, 4096, 100, 7000 + i, np.float32).col_idx)
                         for i in range(n) if lens[i]]).astype(np.int32)
    base = syn.CSR(n, 4096, rp, ci, np.ones(ci.size, np.float32))
    B = syn.uniform_k_per_row(4096, 64, 2, 5, np.float32)
    dB = sm.to_device(B)
    out = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ctx.symbolic(sm.to_device(base), dB, out)                              # valid
    p0 = int(rp[64])                                                       # first entry of the second wave

    def dup_inside(rp, ci):
        ci[rp[200] + 50] = ci[rp[200] + 49]

    def desc_at_window(rp, ci):
        ci[p0 + 64], ci[p0 + 63] = ci[p0 + 63], ci[p0 + 64]

    def out_of_range(rp, ci):
        ci[rp[n] - 1] = 4096

    def negative(rp, ci):
        ci[rp[130]] = -1

    def rp_descends(rp, ci):
        rp[131] = rp[130] - 1

    def rp_last(rp, ci):
        rp[n] -= 1

    for how in (dup_inside, desc_at_window, out_of_range, negative, rp_descends, rp_last):
        M = _mutated(base, how)
        with pytest.raises(sm.SmashError) as e:
            ctx.symbolic(sm.to_device(M), dB, out)
        assert e.value.status == 2, how.__name__


def test_errors(sm, ctx, torch_mod):
    torch = torch_mod
    A = syn.rmat(10, 4, 1, np.float32)
    dA = sm.to_device(A)
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(10, dtype=torch.int32, device="cuda")
    val = torch.empty(10, dtype=torch.float32, device="cuda")
    with pytest.raises(sm.SmashError) as e:
        ctx.numeric(dA, dA, rp, col, val)           # no symbolic plan
    assert e.value.status == 7
    B = syn.rmat(9, 4, 1, np.float32)
    with pytest.raises(sm.SmashError) as e:
        ctx.symbolic(dA, sm.to_device(B), rp)       # A.cols != B.rows
    assert e.value.status == 1
    # invalid CSR: unsorted columns, column out of range, bad row_ptr
    bad = [
        syn.CSR(2, 4, np.array([0, 2, 3], np.int32), np.array([2, 1, 0], np.int32), np.ones(3, np.float32)),
        syn.CSR(2, 4, np.array([0, 2, 3], np.int32), np.array([0, 4, 0], np.int32), np.ones(3, np.float32)),
        syn.CSR(2, 4, np.array([0, 3, 2], np.int32), np.array([0, 1, 2], np.int32), np.ones(3, np.float32)),
    ]
    good = syn.random_sparse(4, 4, 0.5, 3, np.float32)
    for M in bad:
        dM = sm.to_device(M)
        rp2 = torch.empty(3, dtype=torch.int64, device="cuda")
        with pytest.raises(sm.SmashError) as e:
            ctx.symbolic(dM, sm.to_device(good), rp2)
        assert e.value.status == 2
    with pytest.raises(sm.SmashError):
        ctx.set_option(sm.OPT_LDS_ROW_MAX, 5)
    with pytest.raises(sm.SmashError):
        ctx.set_option(sm.OPT_GLOBAL_POOL, -1)
    with pytest.raises(sm.SmashError):
        ctx.set_option(sm.OPT_ROW_HASH, 2)
    with pytest.raises(sm.SmashError):
        ctx.set_option(7, 0)


def _subnormal_case(width, n, dtype=np.float64):
    """One output row from two B rows over the same `width` columns: entry 7
    sums to a negative subnormal (-1e-320 plus an exact zero), entry 9
    cancels to +0.0, entry 11 adds the smallest subnormal twice."""
    cols = np.arange(width, dtype=np.int32) * (n // width)
    b0 = np.ones(width)
    b1 = np.ones(width)
    b0[7], b1[7] = -1e-320, 0.0
    b0[9], b1[9] = 1.0, -1.0
    b0[11], b1[11] = -5e-324, -5e-324
    B = syn.CSR(2, n, np.array([0, width, 2 * width], np.int32), np.concatenate([cols, cols]),
                np.concatenate([b0, b1]).astype(dtype))
    A = syn.CSR(1, 2, np.array([0, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0], dtype))
    return A, B


@pytest.mark.parametrize("path", ["light", "light_ordered", "global", "segment"])
def test_subnormal_and_cancelling_sums(sm, ctx, oracle_mod, path):
    """FP64 sums that end subnormal or cancel keep their entries and values
    on the light-row tables (both hashes), the global-memory tables (FP64
    device atomics) and hashed heavy-row segments."""
    if path.startswith("light"):
        A, B = _subnormal_case(100, 1 << 16)
        if path == "light_ordered":
            ctx.set_option(sm.OPT_ROW_HASH, 1)
    elif path == "global":
        A, B = _subnormal_case(1500, 1 << 20)
        ctx.set_option(sm.OPT_HEAVY_MODE, 1)
    else:
        A, B = _subnormal_case(1500, 1 << 20)          # 1500 columns over 128 chunks: hashed segments
    rp, col, val = run(sm, ctx, A, B, np.float64)
    st = ctx.stats()
    if path.startswith("light"):
        assert st["rows_lds"] == 1, st
    elif path == "global":
        assert st["global_slots"] > 0, st
    else:
        assert st["heavy_segments"] > 0 and st["heavy_dense_chunks"] == 0, st
    ref = oracle_mod.spgemm(A, B)
    assert val[7] == -1e-320 and val[9] == 0.0 and val[11] == -1e-323
    check_rows(rp, col, val, ref, np.float64, f"subnormal {path}")


@pytest.mark.parametrize("mode", [0, 1])
def test_many_terms_one_column(sm, ctx, oracle_mod, mode):
    """One output column collects 1.0 and 3000 terms of 2^-24 (FP32 inputs):
    summed in FP32 in an order that adds 1.0 first, every small term would
    round away (an error of 1.8e-4 of the column's absolute mass, above the
    1e-5 tolerance); the FP64 accumulation of the LDS and global tables
    keeps them.  The row also has 2000 other columns, so it is heavy."""
    n_small = 3000
    k = n_small + 1
    rows_b = []
    vals_b = []
    for r in range(k):
        c = [0] + ([1 + (r % 2000)] if r else list(range(1, 2001)))
        rows_b.append(np.array(c, np.int32))
        vals_b.append(np.array([1.0 if r == 0 else 2.0 ** -24] + [0.5] * (len(c) - 1)))
    rp_b = np.zeros(k + 1, np.int32)
    rp_b[1:] = np.cumsum([len(r) for r in rows_b])
    B = syn.CSR(k, 1 << 20, rp_b, np.concatenate(rows_b), np.concatenate(vals_b).astype(np.float32))
    A = syn.CSR(1, k, np.array([0, k], np.int32), np.arange(k, dtype=np.int32), np.ones(k, np.float32))
    ctx.set_option(sm.OPT_HEAVY_MODE, mode)
    rp, col, val = run(sm, ctx, A, B, np.float32)
    assert ctx.stats()["rows_heavy"] == 1
    ref = oracle_mod.spgemm(A, B)
    assert ref["terms"][0] == k and col[0] == 0
    check_rows(rp, col, val, ref, np.float32, f"many terms mode={mode}")
    assert val[0] == np.float32(1.0 + n_small * 2.0 ** -24)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_order_preserving_row_hash(sm, ctx, oracle_mod, s16, dtype):
    """The order-preserving row hash with the bounded insertion write-back
    (SMASH_OPT_ROW_HASH = 1) gives the same C: RMAT scale 10 and 16, a
    rectangular product, rows of every table size (LDS row limit lowered and
    raised), identity and dense-row cases."""
    ctx.set_option(sm.OPT_ROW_HASH, 1)
    full_check(sm, ctx, syn.workload_small().A, None, dtype, oracle_mod, False, "s10 ordered")
    full_check(sm, ctx, syn.workload_small().A, None, dtype, oracle_mod, True, "s10 ordered split")
    full_check(sm, ctx, s16, None, dtype, oracle_mod, False, "s16 ordered")
    A = syn.rmat(14, 8, 0x5EED0501, dtype)
    full_check(sm, ctx, A, syn.uniform_k_per_row(A.cols, 4096, 16, 0xB, dtype), dtype, oracle_mod, False,
               "rect ordered")
    full_check(sm, ctx, syn.identity(2048), syn.rmat(11, 4, 3, np.float64), dtype, oracle_mod, False, "identity")
    full_check(sm, ctx, syn.dense_rows(64, 64, [0, 5, 63], 10, np.float64),
               syn.dense_rows(64, 900, range(64), 11, np.float64), dtype, oracle_mod, False, "dense rows ordered")
    ctx.set_option(sm.OPT_LDS_ROW_MAX, 64)
    full_check(sm, ctx, syn.rmat(12, 8, 5, dtype), None, dtype, oracle_mod, False, "small tables ordered")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_global_touched_lists_across_windows(sm, ctx, oracle_mod, dtype):
    """Global-mode heavy rows whose columns span three rank windows of 2^19
    columns: the write-out walks each row's touched-slot list once per
    window (every heavy row of RMAT scale 12 times 400 columns per row out
    of 1.5M)."""
    A = syn.rmat(12, 8, 0x44, dtype)
    B = syn.uniform_k_per_row(A.cols, 1_500_000, 400, 0x45, dtype)
    ctx.set_option(sm.OPT_HEAVY_MODE, 1)
    full_check(sm, ctx, A, B, dtype, oracle_mod, False, "global, 3 windows")
    st = ctx.stats()
    assert st["rows_heavy"] > 100 and st["global_slots"] > 0
