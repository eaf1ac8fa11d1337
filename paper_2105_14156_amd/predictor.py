"""Training pipeline of the learned row-size predictor (runs on the GPU).

The training set is the plain method's own output: for RMAT matrices of
scales 12-17 (edge factors 8 and 16, two seeds each) the library computes the
per-row features (smash_features) and the exact row counts (the symbolic
phase); rows without products are left out.  Targets are log2(1 + nnz(C_i)).
The network is trained with the library's HIP forward/backward/Adam kernels
(smash_mlp_train).  The capacity margin delta is the 98th percentile of the
residual log2(1 + nnz) - yhat on a held-out scale-17 matrix, so about 2% of
its rows overflow their predicted capacity.

    python -m paper_2105_14156_amd.predictor train [--out PATH] [--epochs E]
"""
from __future__ import annotations

import argparse
import os
import struct
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "data", "predictor_v1.bin")

TRAIN_SET = [(s, ef, seed) for s in range(12, 18) for ef in (8, 16) for seed in (1, 2)]
HOLDOUT = (17, 16, 3)


def _rows(ctx, smash, A):
    """Features and exact counts of every row of A * A with products."""
    import torch
    dA = smash.to_device(A)
    feats = ctx.features(dA, dA)
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    ctx.symbolic(dA, dA, rp)
    cnt = (rp[1:] - rp[:-1]).to(torch.float32)
    keep = feats[:, 1] > 0           # ub_i > 0
    return feats[keep].contiguous(), torch.log2(1 + cnt[keep]).contiguous()


def build_dataset(ctx, smash, spec, log=print):
    import synthetic as syn
    import torch
    fs, ys = [], []
    for scale, ef, seed in spec:
        A = syn.rmat(scale, ef, 0xB0A7 + 97 * seed + scale, np.float32)
        f, y = _rows(ctx, smash, A)
        fs.append(f)
        ys.append(y)
        log(f"  rmat s{scale} ef{ef} seed{seed}: {y.numel()} rows")
    return torch.cat(fs), torch.cat(ys)


def train(epochs=40, batch=4096, lr=2e-3, seed=0x11A7, log=print):
    """Returns (params float32[4673], mean_std float32[12], delta, report)."""
    import torch
    import synthetic as syn
    from paper_2105_14156_amd import smash
    ctx = smash.Context(0)
    t0 = time.time()
    F, Y = build_dataset(ctx, smash, TRAIN_SET, log)
    mean = F.double().mean(0)
    std = F.double().std(0).clamp_min(1e-6)
    ms = torch.cat([mean, std]).float().contiguous()
    n = Y.numel()
    orders = torch.from_numpy(syn.batch_orders(n, epochs, seed ^ 0x0DE5)).cuda()
    params = torch.from_numpy(syn.mlp_init(seed).astype(np.float32)).cuda()
    losses = ctx.mlp_train(F, Y, ms, params, orders, batch, lr=lr)
    log(f"trained on {n} rows, {epochs} epochs: loss {losses[0]:.4f} -> {losses[-1]:.4f} ({time.time() - t0:.1f} s)")
    Fh, Yh = build_dataset(ctx, smash, [HOLDOUT], log)
    yhat = ctx.mlp_predict(Fh, params, ms)
    res = (Yh - yhat).cpu().numpy()
    delta = float(max(0.0, np.quantile(res, 0.98)))
    mae = float(np.mean(np.abs(res)))
    log(f"held-out rmat s{HOLDOUT[0]}: log2 MAE {mae:.4f}, delta {delta:.4f}")
    ctx.close()
    return (params.cpu().numpy(), ms.cpu().numpy(), delta,
            {"rows": n, "epochs": epochs, "loss": losses.tolist(), "holdout_log2_mae": mae, "delta": delta})


def save(path, params, mean_std, delta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "wb") as f:
        f.write(b"SMASHMLP")
        f.write(struct.pack("<iif", 1, params.size, float(delta)))
        f.write(np.ascontiguousarray(mean_std, "<f4").tobytes())
        f.write(np.ascontiguousarray(params, "<f4").tobytes())


def load(path):
    with open(path, "rb") as f:
        data = f.read()
    assert data[:8] == b"SMASHMLP"
    ver, npar, delta = struct.unpack("<iif", data[8:20])
    assert ver == 1
    ms = np.frombuffer(data[20:20 + 48], "<f4").copy()
    params = np.frombuffer(data[68:68 + 4 * npar], "<f4").copy()
    return params, ms, delta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--epochs", type=int, default=40)
    args = ap.parse_args(argv)
    params, ms, delta, rep = train(args.epochs, log=lambda m: print(m, flush=True))
    save(args.out, params, ms, delta)
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
