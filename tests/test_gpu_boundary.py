"""The C ABI's device-memory contract, through ctypes: every buffer of a
multiply is the caller's (torch tensors here), the workspace size comes from
smash_workspace_size, a workspace that is too small gives CAPACITY with the
bytes needed and is never written beyond its end, and the numeric phase
reports device-detected errors at smash_sync instead of synchronising."""
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


def test_s16_in_caller_workspace(env, oracle_mod):
    """RMAT scale 16 (heavy rows in LDS segments and dense chunks) in a
    workspace sized by smash_workspace_size and allocated by torch; then
    one byte short (one heavy row too few: CAPACITY, the exact size
    reported, nothing written past the end), far too small (CAPACITY before
    any kernel), and the global-memory mode in its own workspace."""
    torch, smash = env
    A = syn.workload_s16().A
    dA = smash.to_device(A)
    ctx = smash.Context(0)
    need = ctx.workspace_size(dA, dA)
    guard = 1 << 20
    buf = torch.full((need + guard,), 0xA5, dtype=torch.uint8, device="cuda")
    ws = buf[:need]
    C = ctx.spgemm(dA, dA, ws=ws)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["rows_heavy"] > 0 and st["heavy_dense_chunks"] > 0
    assert st["workspace_bytes"] == need
    ref = oracle_mod.spgemm(A, A)
    check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), ref, np.float32, "s16 ws")
    assert bool((buf[need:] == 0xA5).all()), "the call wrote past its workspace"

    short = buf[:need - 1]
    buf[need - 1:].fill_(0x5A)
    with pytest.raises(smash.SmashError) as e:
        ctx.spgemm(dA, dA, ws=short)
    assert e.value.status == smash.CAPACITY
    assert ctx.stats()["workspace_bytes"] == need
    torch.cuda.synchronize()
    assert bool((buf[need - 1:] == 0x5A).all()), "a short workspace was written past its end"

    tiny = buf[:4096]
    with pytest.raises(smash.SmashError) as e:
        ctx.spgemm(dA, dA, ws=tiny)
    assert e.value.status == smash.CAPACITY
    assert ctx.stats()["workspace_bytes"] == need

    ctx.set_option(smash.OPT_HEAVY_MODE, 1)
    gneed = ctx.workspace_size(dA, dA)
    gws = torch.empty(gneed, dtype=torch.uint8, device="cuda")
    C = ctx.spgemm(dA, dA, ws=gws)
    torch.cuda.synchronize()
    assert ctx.stats()["global_slots"] > 0
    check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), ref, np.float32,
               "s16 global ws")
    # a global pool of half the tables: the heavy rows run in waves
    half = gws[:gneed // 2 + (1 << 16)]
    C = ctx.spgemm(dA, dA, ws=half)
    torch.cuda.synchronize()
    assert ctx.stats()["global_waves"] > 2
    check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), ref, np.float32,
               "s16 global half ws")
    ctx.close()


def test_context_grows_its_workspace(env, oracle_mod):
    """Without an explicit workspace the binding grows the context's own
    from the size each CAPACITY reports; a smaller product then reuses it."""
    torch, smash = env
    ctx = smash.Context(0)
    for A in (syn.workload_small().A, syn.rmat(14, 16, 3, np.float32), syn.workload_small().A):
        dA = smash.to_device(A)
        C = ctx.spgemm(dA, dA)
        torch.cuda.synchronize()
        check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(),
                   oracle_mod.spgemm(A, A), np.float32, f"grown ws {A.rows}")
    ctx.close()


def test_numeric_errors_reported_at_sync(env):
    """A C_row_ptr changed between the phases makes two light rows' counts
    wrong: numeric returns at once (no synchronisation) and smash_sync
    reports CAPACITY; a later sync is clean again."""
    torch, smash = env
    A = syn.workload_small().A
    dA = smash.to_device(A)
    ctx = smash.Context(0)
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    nnz = ctx.symbolic(dA, dA, rp)
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=torch.float32, device="cuda")
    cnt = np.diff(rp.cpu().numpy())
    mid = int(np.nonzero((cnt[:-1] > 2) & (cnt[1:] > 2))[0][0]) + 1      # rows mid-1 and mid both have entries
    rp[mid] += 1
    ctx.numeric(dA, dA, rp, col, val, check=False)
    with pytest.raises(smash.SmashError) as e:
        ctx.sync()
    assert e.value.status == smash.CAPACITY
    ctx.sync()
    ctx.close()
