"""GPU parity of the batched launch (smash_batch_plan_*) against the oracle.

Each problem's C_p, read from the shared output pool, must match the oracle
like any single product (structure bit-exact, values within tolerance), in
eager runs and in replays of the captured graph (several replays, with other
GPU work and synchronisations in between, each checked), under every
autotuner candidate shape class, and for degenerate batches.  The full
512-problem workload is checked exactly on every problem's row counts and
entry by entry on sampled problems.
"""
import os
import tempfile

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
    ctx = smash.Context(0)
    yield torch, smash, ctx
    ctx.close()


def _problems(count, dtype=np.float32):
    return [(w.A.astype(dtype), w.B.astype(dtype)) for w in syn.workload_batch(count, dtype)]


def _check_plan(plan, probs, refs, oracle_mod, where, stream=None):
    tot, per = plan.result(stream)
    assert tot == int(sum(r["row_ptr"][-1] for r in refs)), f"{where}: total entries"
    for p, ((A, B), ref) in enumerate(zip(probs, refs)):
        C = plan.problem(p)
        assert per[p] == ref["row_ptr"][-1], f"{where}: problem {p} entries"
        check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), ref, A.val.dtype,
                   f"{where} problem {p}")


def _make_plan(smash, ctx, probs, config=None):
    dA = [smash.to_device(A) for A, _ in probs]
    dB = [smash.to_device(B) for _, B in probs]
    return smash.BatchPlan(ctx, dA, dB, config)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batch_eager_and_graph(env, oracle_mod, dtype):
    torch, smash, ctx = env
    probs = _problems(40, dtype)
    refs = [oracle_mod.spgemm(A, B) for A, B in probs]
    plan = _make_plan(smash, ctx, probs)
    plan.run()
    _check_plan(plan, probs, refs, oracle_mod, "eager")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(stream)
    for rep in range(3):
        plan.C_col.fill_(-7)                       # other work between replays
        torch.cuda.synchronize()
        plan.launch(stream)
        _check_plan(plan, probs, refs, oracle_mod, f"replay {rep}", stream)
    plan.close()


@pytest.mark.parametrize("config", [
    dict(lds_row_max=256, table_shift=2, wide_groups=1, blocks_per_cu=1, row_hash=0),
    dict(lds_row_max=512, table_shift=2, wide_groups=0, blocks_per_cu=32, row_hash=1),
    dict(lds_row_max=32, table_shift=1, wide_groups=1, blocks_per_cu=4, row_hash=0),
    dict(lds_row_max=1024, table_shift=1, wide_groups=1, blocks_per_cu=16, row_hash=1),
    dict(lds_row_max=1024, table_shift=1, wide_groups=0, blocks_per_cu=8, row_hash=1),
])
def test_batch_configs(env, oracle_mod, config):
    torch, smash, ctx = env
    probs = _problems(24)
    refs = [oracle_mod.spgemm(A, B) for A, B in probs]
    plan = _make_plan(smash, ctx, probs, config)
    assert plan.config() == config
    plan.run()
    _check_plan(plan, probs, refs, oracle_mod, str(config))
    plan.close()


def test_batch_degenerate(env, oracle_mod):
    """Problems without rows, without entries, rectangular shapes and
    rows heavy enough for the global tables, in one batch."""
    torch, smash, ctx = env
    f32 = np.float32
    probs = [
        (syn.empty(0, 10, f32), syn.random_sparse(10, 7, 0.3, 1, f32)),
        (syn.empty(50, 40, f32), syn.random_sparse(40, 30, 0.2, 2, f32)),
        (syn.random_sparse(60, 80, 0.05, 3, f32), syn.random_sparse(80, 3000, 0.01, 4, f32)),
        (syn.dense_rows(8, 3000, [1, 5], 5, f32), syn.random_sparse(3000, 5000, 0.004, 6, f32)),
        (syn.identity(100, f32), syn.random_sparse(100, 9, 0.5, 7, f32)),
        (syn.random_sparse(1, 1, 1.0, 8, f32), syn.random_sparse(1, 1, 1.0, 9, f32)),
        # wider than the LDS bitmap limit: heavy rows use global tables
        (syn.random_sparse(30, 200, 0.3, 10, f32), syn.uniform_k_per_row(200, (1 << 20) + 3000, 40, 11, f32)),
        # products that are all +-0.0, in the LDS windows of heavy rows
        _zero_case(),
    ]
    refs = [oracle_mod.spgemm(A, B) for A, B in probs]
    plan = _make_plan(smash, ctx, probs, dict(lds_row_max=64, table_shift=1, wide_groups=0, blocks_per_cu=2))
    plan.run()
    _check_plan(plan, probs, refs, oracle_mod, "degenerate")
    plan.close()


def _zero_case():
    B = syn.uniform_k_per_row(8, 8192, 3000, 0x2E0, np.float32)
    A = syn.CSR(3, 8, np.array([0, 2, 4, 6], np.int32), np.arange(6, dtype=np.int32),
                np.array([0.0, -0.0, -0.0, -0.0, 0.5, -0.0], np.float32))
    return A, B


def test_batch_subnormal_wide_window(env, oracle_mod):
    """FP64 heavy rows in the LDS windows (occupancy by leaving -0.0): a
    negative subnormal sum and a cancelling sum keep their entries."""
    torch, smash, ctx = env
    n, width = 8192, 1500
    cols = np.arange(width, dtype=np.int32)
    b0, b1 = np.ones(width), np.ones(width)
    b0[7], b1[7] = -1e-320, 0.0
    b0[9], b1[9] = 1.0, -1.0
    B = syn.CSR(2, n, np.array([0, width, 2 * width], np.int32), np.concatenate([cols, cols]),
                np.concatenate([b0, b1]))
    A = syn.CSR(1, 2, np.array([0, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    probs = [(A, B), _problems(2, np.float64)[1]]
    refs = [oracle_mod.spgemm(a, b) for a, b in probs]
    plan = _make_plan(smash, ctx, probs, dict(lds_row_max=256, table_shift=1, wide_groups=0, blocks_per_cu=4))
    plan.run()
    _check_plan(plan, probs, refs, oracle_mod, "subnormal window")
    C = plan.problem(0)
    v = C.val.cpu().numpy()
    assert v[7] == -1e-320 and v[9] == 0.0
    plan.close()


def test_batch_without_rows(env):
    torch, smash, ctx = env
    probs = [(syn.empty(0, 5, np.float32), syn.random_sparse(5, 5, 0.5, 1, np.float32))] * 3
    plan = _make_plan(smash, ctx, probs)
    plan.run()
    stream = torch.cuda.Stream()
    plan.capture(stream)
    plan.launch(stream)
    tot, per = plan.result(stream)
    assert tot == 0 and list(per) == [0, 0, 0]
    assert plan.C_row_ptr.cpu().tolist() == [0]
    plan.close()


def test_batch_invalid_operand(env):
    """Creation validates every operand: one problem whose B has a repeated
    column in a row fails the whole batch with INVALID_CSR."""
    torch, smash, ctx = env
    probs = _problems(6)
    A, B = probs[4]
    ci = B.col_idx.copy()
    r = int(np.argmax(np.diff(B.row_ptr)))                 # a row with at least two entries
    ci[B.row_ptr[r] + 1] = ci[B.row_ptr[r]]
    probs[4] = (A, syn.CSR(B.rows, B.cols, B.row_ptr, ci, B.val))
    with pytest.raises(smash.SmashError) as e:
        _make_plan(smash, ctx, probs)
    assert e.value.status == 2


def test_batch_capacity_error(env):
    """A structure change after creation that needs more entries than the
    pool holds is reported as CAPACITY."""
    torch, smash, ctx = env
    n = 4096
    A = syn.strided_columns(n, n, 6, 2, 11, np.float32)          # even columns only
    B = syn.uniform_k_per_row(n, n, 8, 12, np.float32)
    dA, dB = smash.to_device(A), smash.to_device(B)
    plan = smash.BatchPlan(ctx, [dA], [dB])
    plan.run()
    plan.result()
    # same shape and nnz, but even rows hold 16 entries and odd rows none:
    # every row of A now reaches 96 products, twice the pool's 48 per row
    half = syn.uniform_k_per_row(n // 2, n, 16, 13, np.float32)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(np.where(np.arange(n) % 2 == 0, 16, 0))
    assert rp[-1] == B.nnz == half.nnz
    dB.row_ptr.copy_(torch.from_numpy(rp.astype(np.int32)))
    dB.col_idx.copy_(torch.from_numpy(half.col_idx.astype(np.int32)))
    plan.run()
    with pytest.raises(smash.SmashError) as ei:
        plan.result()
    assert ei.value.status == 4
    plan.close()


def test_batch_autotune_and_cache(env, oracle_mod):
    torch, smash, ctx = env
    probs = _problems(32)
    refs = [oracle_mod.spgemm(A, B) for A, B in probs]
    plan = _make_plan(smash, ctx, probs)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        cfg, ms = plan.autotune(reps=1, cache_path=path)
        assert ms > 0 and plan.config() == cfg
        plan.run()
        _check_plan(plan, probs, refs, oracle_mod, "autotuned")
        plan.configure(dict(lds_row_max=32, table_shift=1, wide_groups=0, blocks_per_cu=1))
        cfg2, ms2 = plan.autotune(reps=1, cache_path=path)      # cache hit
        assert ms2 == 0.0 and cfg2 == cfg and plan.config() == cfg
    plan.close()


@pytest.mark.timeout(600)
def test_batch_full_512(env, oracle_mod):
    """The 512-problem workload in its graph: exact row counts of every
    problem, entries of sampled problems (the largest ones and seeded picks)."""
    torch, smash, ctx = env
    probs = _problems(512)
    plan = _make_plan(smash, ctx, probs)
    stream = torch.cuda.Stream()
    plan.capture(stream)
    plan.launch(stream)
    plan.launch(stream)
    tot, per = plan.result(stream)
    crp = plan.C_row_ptr.cpu().numpy()
    for p, (A, B) in enumerate(probs):
        nz = oracle_mod.row_nnz(A, B)
        r0, r1 = plan.row0[p], plan.row0[p + 1]
        assert np.array_equal(np.diff(crp[r0:r1 + 1]), nz), f"problem {p} row counts"
    prods = np.array([int(np.diff(B.row_ptr)[A.col_idx].sum()) for A, B in probs])
    pick = set(np.argsort(-prods)[:4].tolist()) | set((syn.uniform01(0xBA7, 0, 8) * 512).astype(int).tolist())
    for p in sorted(pick):
        A, B = probs[p]
        C = plan.problem(p)
        check_rows(C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy(), C.val.cpu().numpy(), oracle_mod.spgemm(A, B),
                   np.float32, f"512 batch problem {p}")
    plan.close()
