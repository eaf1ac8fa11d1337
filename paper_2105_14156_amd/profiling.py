"""Summaries of rocprofv3 output for this library's kernels (host tool).

    python -m paper_2105_14156_amd.profiling stats RUN_kernel_stats.csv --steps K --cmd "..." > summary.txt
    python -m paper_2105_14156_amd.profiling traffic --fetch F.csv --write W.csv \\
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N --steps K --cmd "..." --json out.json > summary.txt
    python -m paper_2105_14156_amd.profiling counters P1.csv P2.csv ... --kernels num_dense,num_seg \\
        --steps K --cmd "..." > summary.txt

``stats`` condenses a ``--kernel-trace --stats`` table to one line per kernel
(calls, total and average duration).  ``counters`` sums the counters of
several ``--pmc`` passes per kernel and step and derives the figures that
say what bounds a kernel (instruction mix, wait share, LDS bank conflicts,
L2 hit rate and read latency).  ``traffic`` turns two ``--pmc`` runs
(FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) into HBM bytes per launch,
each counter scaled by what it reads for a plain device copy of known size
(the copy reads and writes ``--copy-bytes`` bytes per launch).  The JSON
output carries a hash of the HIP sources, so a reader can tell whether the
counters still describe the kernels as built.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in sorted(os.listdir(os.path.join(HERE, "csrc")))
           if f.endswith((".hip", ".hpp"))] + [os.path.join(ROOT, "include", "smash.h")]


def source_hash() -> str:
    """sha256 over the HIP sources and the public header."""
    h = hashlib.sha256()
    for p in SOURCES:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(kernel: str) -> str:
    """'void smash::k_num_dense<float>(...)' -> 'num_dense'; other names as given."""
    m = re.search(r"smash::k_(\w+)", kernel)
    return m.group(1) if m else kernel.split("(")[0].strip()


def read_stats(path):
    out = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            n = short_name(r["Name"])
            calls, tot = int(r["Calls"]), float(r["TotalDurationNs"])
            c0, t0 = out.get(n, (0, 0.0))
            out[n] = (c0 + calls, t0 + tot)
    return out


def cmd_stats(args):
    st = read_stats(args.csv)
    total = sum(t for _, t in st.values())
    print(f"# rocprofv3 kernel statistics, {args.title}")
    print(f"# command: {args.cmd}")
    print(f"# {args.steps} timed steps plus warm-up; per-step = total / launches-per-step")
    print(f"{'kernel':24s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'share':>7s}")
    for n, (calls, tot) in sorted(st.items(), key=lambda kv: -kv[1][1]):
        print(f"{n:24s} {calls:7d} {tot / 1e6:10.3f} {tot / calls / 1e3:10.1f} {tot / total:7.1%}")


def read_pmc(path, counter):
    """{kernel: [values per dispatch]} of one counter (KiB)."""
    out = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            out[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return out


def cmd_traffic(args):
    fetch = read_pmc(args.fetch, "FETCH_SIZE")
    write = read_pmc(args.write, "WRITE_SIZE")
    cf = read_pmc(args.copy_fetch, "FETCH_SIZE")
    cw = read_pmc(args.copy_write, "WRITE_SIZE")
    # the copy kernel is the largest dispatch of the calibration run
    copy_f = max(max(v) for v in cf.values()) * 1024.0
    copy_w = max(max(v) for v in cw.values()) * 1024.0
    kf = args.copy_bytes / copy_f if copy_f else None
    kw = args.copy_bytes / copy_w if copy_w else None
    print(f"# HBM traffic from FETCH_SIZE / WRITE_SIZE, {args.title}")
    print(f"# command (one run per counter): {args.cmd}")
    print(f"# calibration: a device copy of {args.copy_bytes} bytes reads FETCH_SIZE {copy_f:.0f} B "
          f"(scale {kf:.3f}) and WRITE_SIZE {copy_w:.0f} B (scale {kw:.3f})")
    print(f"{'kernel':24s} {'launches':>8s} {'fetch MB/launch':>16s} {'write MB/launch':>16s} {'scaled GB/launch':>17s}")
    kernels = {}
    for n in sorted(set(fetch) | set(write), key=lambda k: -sum(fetch.get(k, [0]))):
        fl, wl = fetch.get(n, []), write.get(n, [])
        nf = max(len(fl), 1)
        f_avg = sum(fl) / nf * 1024.0
        w_avg = sum(wl) / max(len(wl), 1) * 1024.0
        scaled = f_avg * kf + w_avg * kw
        kernels[n] = {"launches": len(fl), "fetch_bytes": f_avg, "write_bytes": w_avg,
                      "hbm_bytes_scaled": scaled}
        print(f"{n:24s} {len(fl):8d} {f_avg / 1e6:16.2f} {w_avg / 1e6:16.2f} {scaled / 1e9:17.3f}")
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"title": args.title, "command": args.cmd, "source_sha256": source_hash(),
                       "copy_bytes": args.copy_bytes, "fetch_scale": kf, "write_scale": kw,
                       "kernels": kernels}, f, indent=1)


def read_counters(paths, kernels):
    """{kernel: {counter: sum over dispatches}} over several --pmc passes."""
    out = collections.defaultdict(lambda: collections.defaultdict(float))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                n = short_name(r["Kernel_Name"])
                if kernels and n not in kernels:
                    continue
                out[n][r["Counter_Name"]] += float(r["Counter_Value"])
    return out


# derived figures: (label, numerator, denominator, scale)
DERIVED = [
    ("VALU instructions per LDS instruction", "SQ_INSTS_VALU", "SQ_INSTS_LDS", 1.0),
    ("SALU instructions per VALU instruction", "SQ_INSTS_SALU", "SQ_INSTS_VALU", 1.0),
    ("share of wave cycles waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES)", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES", 1.0),
    ("LDS bank-conflict cycles per LDS-active cycle", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", 1.0),
    ("LDS atomics with return per LDS instruction", "SQ_LDS_ATOMIC_RETURN", "SQ_INSTS_LDS", 1.0),
    ("L2 hit rate (TCC_HIT / TCC_REQ)", "TCC_HIT_sum", "TCC_REQ_sum", 1.0),
    ("L2 read latency seen by L1, cycles per request", "TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum", 1.0),
    ("L2 misses that go to DRAM", "TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_RDREQ_sum", 1.0),
]


def cmd_counters(args):
    kernels = [k for k in args.kernels.split(",") if k] if args.kernels else []
    c = read_counters(args.csv, kernels)
    print(f"# rocprofv3 counters per step, {args.title}")
    print(f"# command (one run per counter group): {args.cmd}")
    print(f"# sums over the dispatches of {args.steps} step(s), divided by the step count; one --pmc pass per")
    print("# group, so counters of different groups come from different (identical) runs")
    for n in (kernels or sorted(c)):
        t = c.get(n)
        if not t:
            continue
        print(f"== {n}")
        for k in sorted(t):
            print(f"   {k:32s} {t[k] / args.steps:16.5g}")
        if "GRBM_GUI_ACTIVE" in t and "SQ_INSTS_VALU" in t:
            # GRBM_GUI_ACTIVE counts cycles once per XCD; a wave64 VALU
            # instruction holds one of the CU's four SIMDs for 4 cycles
            cycles = t["GRBM_GUI_ACTIVE"] / args.xcds
            busy = t["SQ_INSTS_VALU"] * 4.0 / (args.cus * 4.0 * cycles)
            print(f"   {'kernel cycles (GRBM_GUI_ACTIVE / XCDs)':58s} {cycles / args.steps:12.5g}")
            print(f"   {'VALU issue share (4 x VALU / (4 SIMDs x CUs x cycles))':58s} {busy:12.3f}")
        for label, num, den, sc in DERIVED:
            if num in t and den in t and t[den]:
                print(f"   {label:58s} {t[num] / t[den] * sc:12.3f}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--steps", type=int, default=1)
    a.add_argument("--cmd", default="")
    a.add_argument("--title", default="")
    b = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        b.add_argument("--" + k.replace("_", "-"), required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--steps", type=int, default=1)
    b.add_argument("--cmd", default="")
    b.add_argument("--title", default="")
    b.add_argument("--json")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--kernels", default="")
    c.add_argument("--steps", type=int, default=1)
    c.add_argument("--cus", type=int, default=256)
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--cmd", default="")
    c.add_argument("--title", default="")
    args = ap.parse_args(argv)
    if args.cmd_name == "stats":
        cmd_stats(args)
    elif args.cmd_name == "counters":
        cmd_counters(args)
    else:
        cmd_traffic(args)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main()
