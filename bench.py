"""Benchmark of the row-wise hash SpGEMM C = A * B on one MI355X.

A step is one whole product through the C ABI (symbolic phase, nnz(C)
readback, output allocation from torch's caching allocator, numeric phase)
on inputs already resident in HBM, in one workspace sized once by
smash_workspace_size and allocated by torch.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload s19|s16|s10|rect] [--dtype f32|f64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from paper_2105_14156_amd import metrics  # noqa: E402

_NATIVE_ORACLE = None
METRIC = "SpGEMM GFLOP/s (2·products/s) + HBM GB/s; learned/batched vs plain at exact C"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "s19": ("rmat_s19_ef16_AxA", synthetic.workload_s19, "RMAT scale 19, edge factor 16, a/b/c/d=.57/.19/.19/.05, C=A*A"),
    "s16": ("rmat_s16_ef16_AxA", synthetic.workload_s16, "RMAT scale 16, edge factor 16, C=A*A"),
    "s10": ("rmat_s10_ef8_AxA", synthetic.workload_small, "RMAT scale 10, edge factor 8, C=A*A"),
    "rect": ("rmat_s21_ef8_x_uniform4096k16", synthetic.workload_rect, "RMAT scale 21 ef 8 times 2^21x4096 (16/row)"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="s19", choices=sorted(WORKLOADS) + ["batch"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--heavy-mode", type=int, default=0)
    ap.add_argument("--path", default="plain", choices=["plain", "fused"],
                    help="plain: symbolic + numeric; fused: learned-capacity single pass for LDS rows")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the fused-pass and batched-launch comparison beside the main line")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-config", default="", metavar="L,S,W,B,H",
                    help="batch: use this configuration (lds_row_max,table_shift,wide_groups,blocks_per_cu,row_hash) "
                         "instead of autotuning")
    ap.add_argument("--no-plain-loop", action="store_true", help="batch: skip the loop of plain calls")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


def copy_calibration(mib: int, reps: int = 3):
    """A plain copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters: each launch reads and writes mib MiB."""
    import torch
    n = mib << 20
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_per_launch": n, "launches": reps, "gbs": round(2 * n / dt / 1e9, 1)}), flush=True)


def committed_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload (profiles/traffic_<workload>.json), or None when there is
    none or the HIP sources changed since the counters were taken."""
    from paper_2105_14156_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != profiling.source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return int(k["hbm_bytes_scaled"]) if k else None


def copy_gbs(mib: int = 1024, reps: int = 5) -> float:
    """Bandwidth of a plain device copy (read + write bytes per second), the
    measured counterpart of the 8 TB/s peak."""
    import torch
    x = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del x, y
    return 2.0 * (mib << 20) / dt / 1e9


def predictor_report(ctx, smash, dA, dB, counts, fused):
    """Quality of the shipped predictor on this product: log2 MAE of its
    prediction against the exact row counts (rows with products), the
    overflow rate and the LDS slots it reserves beyond the entries of the
    rows it completed, and the end-to-end gain over exact upper-bound
    sizing (T-gain)."""
    import torch
    from paper_2105_14156_amd import predictor
    params, ms, _ = predictor.load(predictor.DEFAULT_PATH)
    feats = ctx.features(dA, dB)
    yhat = ctx.mlp_predict(feats, torch.from_numpy(params).cuda(), torch.from_numpy(ms).cuda())
    keep = feats[:, 1] > 0
    mae = (yhat[keep] - torch.log2(1.0 + counts[keep].double()).float()).abs().mean().item()
    ln, ub = fused["learned"], fused["upper_bound"]
    tried = ln["fused_rows"] + ln["overflow_rows"]
    return {"log2_mae": round(mae, 4), "rows_with_products": int(keep.sum().item()),
            "overflow_rate": round(ln["overflow_rows"] / max(1, tried), 5),
            "reserved_slots": ln["reserved_slots"], "entries_of_fused_rows": ln["fused_entries"],
            "wasted_slots": ln["reserved_slots"] - ln["fused_entries"],
            "upper_bound_reserved_slots": ub["reserved_slots"],
            "t_gain": round(ub["ms_per_step"] / ln["ms_per_step"], 4)}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(A, B, target_s, threads=None):
    """The oracle timed on a seeded row sample of the same product (all host
    threads up to 16, or `threads`), scaled to GFLOP/s of 2 x products.  The
    oracle is compiled for this host (gcc -O3 -march=native) first."""
    import oracle
    global _NATIVE_ORACLE
    if _NATIVE_ORACLE is None:
        _NATIVE_ORACLE = oracle.use_native_build()
    ub = oracle.products_per_row(A, B)
    if threads is None:
        threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                             else os.cpu_count()))
    # calibrate on a small sample, then size the timed sample to about target_s
    total = int(ub.sum())
    rng_rows = np.argsort(synthetic.uniform01(0xBA5E, 0, A.rows), kind="stable")
    pref = np.cumsum(ub[rng_rows])
    probe_n = int(np.searchsorted(pref, min(total, 5e7))) + 1
    t0 = time.perf_counter()
    oracle.spgemm(A, B, rows=np.sort(rng_rows[:probe_n]), threads=threads, with_stats=False)
    t_probe = time.perf_counter() - t0
    rate = max(float(pref[probe_n - 1]) / max(t_probe, 1e-6), 1.0)
    want = min(total, int(rate * target_s))
    n_rows = int(np.searchsorted(pref, want)) + 1
    sel = np.sort(rng_rows[:n_rows])
    prods = int(ub[sel].sum())
    t0 = time.perf_counter()
    oracle.spgemm(A, B, rows=sel, threads=threads, with_stats=False)
    t = time.perf_counter() - t0
    return {"value": round(2.0 * prods / t / 1e9, 4), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_rows} seeded random rows of {A.rows} ({prods} of {total} products, "
                      f"{prods / total:.1%}), {t:.1f} s wall",
            "cpu": cpu_model(), "build": "gcc -O3 -march=native"}


def cpu_model() -> str:
    """The host CPU's model name and logical core count (/proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            names = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")]
        return f"{names[0]} ({len(names)} logical cores)" if names else "unknown"
    except OSError:
        return "unknown"


def products_of(A, B) -> int:
    """Sum over rows of A of the B-row lengths it selects (host arithmetic)."""
    return int(np.diff(B.row_ptr).astype(np.int64)[A.col_idx].sum()) if A.nnz else 0


def run_fused_compare(key: str, npdt, steps: int, warmup: int):
    """Plain two-phase against the fused pass (learned and exact upper-bound
    capacities) on another workload, each in its own workspace-sized loop."""
    import torch
    from paper_2105_14156_amd import smash
    name, make, _ = WORKLOADS[key]
    w = make(npdt)
    dA = smash.to_device(w.A)
    dB = dA if w.B is w.A else smash.to_device(w.B)
    ctx = smash.Context(0)
    ctx.predictor_load()
    ws = ctx.workspace(ctx.workspace_size(dA, dB))

    def timed(fn):
        C = None
        for _ in range(max(1, warmup)):
            C = None
            C = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            C = None
            C = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3, ctx.stats()

    plain_ms, _ = timed(lambda: ctx.spgemm(dA, dB, ws=ws))
    res = {"workload": name, "plain_ms_per_step": round(plain_ms, 4)}
    for sizing, label in ((0, "learned"), (1, "upper_bound")):
        ctx.set_option(smash.OPT_FUSED_SIZING, sizing)
        f_ms, st = timed(lambda: ctx.spgemm_fused(dA, dB, ws=ws))
        res[label] = {"ms_per_step": round(f_ms, 4), "fused_rows": st["fused_rows"],
                      "overflow_rows": st["fused_overflow"], "rows_heavy": st["rows_heavy"]}
    res["fused_speedup_vs_plain"] = round(plain_ms / res["learned"]["ms_per_step"], 4)
    res["network_speedup_vs_upper_bound"] = round(res["upper_bound"]["ms_per_step"] / res["learned"]["ms_per_step"], 4)
    ctx.close()
    log(f"{name}: plain {plain_ms:.3f} ms, fused learned {res['learned']['ms_per_step']:.3f}, "
        f"upper bound {res['upper_bound']['ms_per_step']:.3f}")
    return res


def run_batch(count: int, steps: int, warmup: int, plain_loops: int = 2, config: str = ""):
    """The batched workload: `count` products in one captured graph (after
    autotuning the plan), against a loop of plain smash_spgemm calls over the
    same problems on the same stream.  Returns a dict of the measurements."""
    import torch
    from paper_2105_14156_amd import smash
    t0 = time.perf_counter()
    probs = synthetic.workload_batch(count)
    log(f"batch of {count}: generated in {time.perf_counter() - t0:.1f} s")
    dA = [smash.to_device(w.A) for w in probs]
    dB = [smash.to_device(w.B) for w in probs]
    products = sum(products_of(w.A, w.B) for w in probs)
    ctx = smash.Context(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = smash.BatchPlan(ctx, dA, dB, stream=stream)
        if config:
            keys = ("lds_row_max", "table_shift", "wide_groups", "blocks_per_cu", "row_hash")
            plan.configure(dict(zip(keys, (int(v) for v in config.split(",")))))
            cfg, tune_ms = plan.config(), 0.0
            log(f"configured {cfg}")
        else:
            cfg, tune_ms = plan.autotune(reps=3, stream=stream)
            log(f"autotuned {cfg} ({tune_ms:.3f} ms per batch)")
        plan.capture(stream)
        for _ in range(warmup):
            plan.launch(stream)
        nnz_c, _ = plan.result(stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.launch(stream)
        e1.record(stream)
        plan.result(stream)
        graph_ms = e0.elapsed_time(e1) / steps
        # the same problems one plain call at a time
        loop_ms = float("nan")
        if plain_loops:
            for A, B in zip(dA[:8], dB[:8]):
                ctx.spgemm(A, B, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(plain_loops):
                for A, B in zip(dA, dB):
                    ctx.spgemm(A, B, stream)
            torch.cuda.synchronize()
            loop_ms = (time.perf_counter() - t0) / plain_loops * 1e3
    rows = sum(w.A.rows for w in probs)
    alg = sum(metrics.algorithmic_bytes(w.A.rows, w.B.rows, w.A.nnz, w.B.nnz, 0, 4) for w in probs) \
        + nnz_c * 8
    plan.close()
    ctx.close()
    log(f"batch graph {graph_ms:.3f} ms, plain loop {loop_ms:.3f} ms")
    return {"count": count, "rows": rows, "products": products, "nnz_c": nnz_c, "graph_ms": graph_ms,
            "plain_loop_ms": loop_ms, "config": cfg, "autotune_ms": tune_ms, "alg_bytes": alg}


def main_batch(args):
    r = run_batch(args.batch_count, args.steps, args.warmup, 0 if args.no_plain_loop else 2, args.batch_config)
    gflops = metrics.gflops(r["products"], r["graph_ms"] * 1e-3)
    gbs = r["alg_bytes"] / (r["graph_ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(gflops, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["graph_ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch{r['count']}_rmat_x_uniform8", "description":
                   "512 products A_i*B_i: A_i RMAT n_i log-uniform in [256, 32768], edge factor uniform 4..32; "
                   "B_i n_i x n_i with 8 uniform columns per row", "path": "batched graph replay (autotuned)",
                   "rows": r["rows"], "products": r["products"], "nnz_c": r["nnz_c"], "tuned": r["config"]},
        "hbm_gbs_algorithmic": round(gbs, 2), "path_roofline_frac": round(gbs / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "kernel": "whole batch graph", "achieved": round(gbs, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "plain_loop_ms": round(r["plain_loop_ms"], 3) if r["plain_loop_ms"] == r["plain_loop_ms"] else None,
        "speedup_vs_plain_loop": round(r["plain_loop_ms"] / r["graph_ms"], 2)
        if r["plain_loop_ms"] == r["plain_loop_ms"] else None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(row sharding across GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2105_14156_amd import smash

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batch":
        main_batch(args)
        return
    name, make, desc = WORKLOADS[args.workload]
    npdt = np.float32 if args.dtype == "f32" else np.float64
    vbytes = 4 if args.dtype == "f32" else 8
    t0 = time.perf_counter()
    w = make(npdt)
    A, B = w.A, w.B
    log(f"workload {name}: A {A.rows}x{A.cols} nnz {A.nnz}, B {B.rows}x{B.cols} nnz {B.nnz} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    dA = smash.to_device(A)
    dB = dA if B is A else smash.to_device(B)
    ctx = smash.Context(0)
    ctx.set_option(smash.OPT_HEAVY_MODE, args.heavy_mode)
    stream = torch.cuda.current_stream()
    # one caller-owned workspace for every call (sized with the predictor
    # installed, so that it also covers the fused pass)
    ctx.predictor_load()
    ws = ctx.workspace(ctx.workspace_size(dA, dB, stream))
    log(f"workspace {ws.numel() / 2**20:.1f} MiB")
    if args.path == "fused":
        run = lambda: ctx.spgemm_fused(dA, dB, stream, ws=ws)
    else:
        run = lambda: ctx.spgemm(dA, dB, stream, ws=ws)

    C = None
    for i in range(args.warmup):
        C = None
        C = run()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    st = ctx.stats()
    products, nnz_c = st["products"], st["nnz_c"]

    ctx.set_option(smash.OPT_TIMING, 1)
    ctx.reset_kernel_times()
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        C = None
        C = run()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    counts = C.row_ptr[1:] - C.row_ptr[:-1]
    kt = ctx.kernel_times()
    ctx.set_option(smash.OPT_TIMING, 0)
    st = ctx.stats()

    ms_step = elapsed / args.steps * 1e3
    gflops = metrics.gflops(products, elapsed / args.steps)
    alg = metrics.algorithmic_bytes(A.rows, B.rows, A.nnz, B.nnz, nnz_c, vbytes)
    path_gbs = alg / (elapsed / args.steps) / 1e9

    # dominant kernel; its algorithmic bytes per launch are its share of C's
    # entries times the path's compulsory bytes (read A and B, write C once)
    dom = max(kt.items(), key=lambda kv: kv[1][1])
    dname, (dlaunch, dms) = dom
    nnz_heavy, nnz_dense = st["nnz_heavy"], st["nnz_dense"]
    entries = {"num_rows": nnz_c - nnz_heavy, "sym_rows": nnz_c - nnz_heavy, "num_seg": nnz_heavy - nnz_dense,
               "num_dense": nnz_dense, "sym_heavy": nnz_heavy, "num_global": nnz_heavy, "sym_global": nnz_heavy}
    share = entries.get(dname, nnz_c) / max(1, nnz_c)
    launches_per_step = dlaunch / args.steps
    per_launch_bytes = alg * share / max(1e-9, launches_per_step)
    avg_ms = dms / max(1, dlaunch)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": name, "description": desc, "path": "plain two-phase (symbolic + numeric)" if args.path == "plain"
                   else "fused single pass with learned row capacities",
                   "heavy_mode": "lds_segments" if args.heavy_mode == 0 else "global_hash",
                   "rows": A.rows, "cols": B.cols, "nnz_a": A.nnz, "nnz_b": B.nnz, "nnz_c": nnz_c,
                   "products": products},
        "hbm_gbs_algorithmic": round(path_gbs, 2),
        "path_roofline_frac": round(path_gbs / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": committed_traffic(name, dname) if args.path == "plain" and args.dtype == "f32" else None,
                     "launches_per_step": launches_per_step, "avg_launch_ms": round(avg_ms, 4),
                     "alg_bytes_per_launch": int(per_launch_bytes), "c_entry_share": round(share, 4),
                     "alg_bytes_basis": "apportioned: the path's compulsory bytes (A, B, C once) times the "
                                        "kernel's share of C's entries, per launch"},
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in kt.items() if v[0]},
        "stats": st,
        "ms_median": round(float(np.median(step_ms)), 4),
        "ms_min": round(float(np.min(step_ms)), 4),
        # row-wise re-fetches of B (an entry per product) and the symbolic
        # pass's index reads on top of the compulsory bytes; mostly L2/MALL
        "streamed_gb_per_step": round((alg + products * (vbytes + 4) + products * 4) / 1e9, 3),
        "streamed_gbs": round((alg + products * (vbytes + 4) + products * 4) / (elapsed / args.steps) / 1e9, 1),
    }
    cg = copy_gbs()
    out["copy_gbs_measured"] = round(cg, 1)
    out["path_frac_of_copy"] = round(path_gbs / cg, 4)
    if not args.no_variants:
        # the fused pass on the same product, with the learned capacities and
        # with the exact upper bound min(products, cols) (no network), and the
        # batched launch
        ctx.predictor_load()

        def timed(fn):
            nonlocal_c = None
            for _ in range(max(1, args.warmup)):
                nonlocal_c = None
                nonlocal_c = fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                nonlocal_c = None
                nonlocal_c = fn()
            torch.cuda.synchronize()
            del nonlocal_c
            return (time.perf_counter() - t0) / args.steps * 1e3, ctx.stats()

        C = None
        fused = {}
        for sizing, name in ((0, "learned"), (1, "upper_bound")):
            ctx.set_option(smash.OPT_FUSED_SIZING, sizing)
            ms_f, st_f = timed(lambda: ctx.spgemm_fused(dA, dB, stream, ws=ws))
            fused[name] = {"ms_per_step": round(ms_f, 4), "fused_rows": st_f["fused_rows"],
                           "overflow_rows": st_f["fused_overflow"], "reserved_slots": st_f["fused_capacity"],
                           "fused_entries": st_f["fused_entries"]}
            log(f"fused ({name} capacities): {ms_f:.3f} ms per step")
        ctx.set_option(smash.OPT_FUSED_SIZING, 0)
        if args.path == "plain":
            ms_plain = ms_step
        else:
            ms_plain, _ = timed(lambda: ctx.spgemm(dA, dB, stream, ws=ws))
        rect = run_fused_compare("rect", npdt, args.steps, args.warmup) if args.workload != "rect" else None
        b = run_batch(args.batch_count, args.steps, args.warmup)
        out["variants"] = {
            "plain_ms_per_step": round(ms_plain, 4),
            "fused": fused,
            "fused_speedup_vs_plain": round(ms_plain / fused["learned"]["ms_per_step"], 4),
            "network_speedup_vs_upper_bound": round(fused["upper_bound"]["ms_per_step"]
                                                    / fused["learned"]["ms_per_step"], 4),
            "predictor": predictor_report(ctx, smash, dA, dB, counts, fused),
            "rect": rect,
            "batch": {"workload": f"batch{b['count']}_rmat_x_uniform8", "graph_ms": round(b["graph_ms"], 4),
                      "plain_loop_ms": round(b["plain_loop_ms"], 3),
                      "speedup_vs_plain_loop": round(b["plain_loop_ms"] / b["graph_ms"], 2),
                      "gflops": round(metrics.gflops(b["products"], b["graph_ms"] * 1e-3), 3),
                      "tuned": b["config"]},
        }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds)
        log("cpu baseline, one thread ...")
        out["cpu_baseline_1thread"] = cpu_baseline(A, B, args.cpu_seconds / 3, threads=1)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
