"""smash_spgemm_noalloc (the entry point for callers that cannot allocate
device memory) against smash_spgemm and the oracle, through the C ABI: two
calls in a row on one context (the second with a smaller product, so it
runs in what the first left in the library's scratch array), both dtypes,
and its two CAPACITY cases (output buffers too small: nnz(C) reported;
workspace beyond the array: the bytes needed reported)."""
import numpy as np
import pytest

import synthetic as syn
from tests._parity import check_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_14156_amd import smash
    assert torch.cuda.is_available()
    return torch, smash


def _noalloc(torch, smash, ctx, dA, dB, capacity):
    rp = torch.empty(dA.rows + 1, dtype=torch.int64, device="cuda")
    col = torch.full((capacity,), -7, dtype=torch.int32, device="cuda")
    val = torch.zeros(capacity, dtype=dA.val.dtype, device="cuda")
    nnz = ctx.spgemm_noalloc(dA, dB, rp, col, val)
    torch.cuda.synchronize()
    return rp, col[:nnz], val[:nnz], nnz


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_matches_spgemm(env, oracle_mod, dtype):
    torch, smash = env
    ctx = smash.Context(0)
    # the larger product first (heavy rows in segments and dense chunks), then a smaller one
    for A in (syn.rmat(15, 16, 0x6A, dtype), syn.workload_small(dtype).A):
        dA = smash.to_device(A)
        ref_c = ctx.spgemm(dA, dA)
        torch.cuda.synchronize()
        st = ctx.stats()
        rp, col, val, nnz = _noalloc(torch, smash, ctx, dA, dA, int(ref_c.col_idx.numel()) + 1000)
        ctx.sync()
        assert nnz == st["nnz_c"]
        assert torch.equal(rp, ref_c.row_ptr) and torch.equal(col, ref_c.col_idx)
        ref = oracle_mod.spgemm(A, A)
        check_rows(rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), ref, dtype, f"noalloc {A.rows}")
        if A.rows > 10000:
            assert ctx.stats()["rows_heavy"] > 0 and ctx.stats()["heavy_dense_chunks"] > 0
    ctx.close()


def test_noalloc_capacity(env):
    torch, smash = env
    ctx = smash.Context(0)
    A = syn.workload_small().A
    dA = smash.to_device(A)
    with pytest.raises(smash.SmashError) as e:
        _noalloc(torch, smash, ctx, dA, dA, 100)
    assert e.value.status == smash.CAPACITY and e.value.nnz > 100
    exact = e.value.nnz
    rp, col, val, nnz = _noalloc(torch, smash, ctx, dA, dA, exact)
    assert nnz == exact
    # 4M rows need more plan arrays than the 64 MiB array holds
    big = syn.empty(4_000_000, 16)
    dbig = smash.to_device(big)
    dB = smash.to_device(syn.random_sparse(16, 16, 0.5, 3))
    with pytest.raises(smash.SmashError) as e:
        _noalloc(torch, smash, ctx, dbig, dB, 16)
    assert e.value.status == smash.CAPACITY
    assert ctx.stats()["workspace_bytes"] > smash.NOALLOC_SCRATCH_BYTES
    ctx.set_option(smash.OPT_HEAVY_MODE, 1)
    with pytest.raises(smash.SmashError) as e:
        _noalloc(torch, smash, ctx, dA, dA, exact)
    assert e.value.status == 1
    ctx.close()
