"""Training pipeline of the learned row-size predictor (runs on the GPU).

The training set is the plain method's own output: for products of RMAT
matrices of scales 12-17 (A * A, edge factors 8 and 16, two seeds each) and
of RMAT scales 12-16 with uniform matrices of 1024 or 4096 columns (16
entries per row: products whose rows saturate a narrow B, where the product
count overstates the output most) the library computes the per-row features
(smash_features) and the exact row counts (the symbolic phase); rows without
products are left out.  Targets are log2(1 + nnz(C_i)).  The network is
trained with the library's HIP forward/backward/Adam kernels
(smash_mlp_train).  The fused pass asks the network only about rows whose
bound min(products, columns) exceeds the LDS row limit, so the capacity
margin delta is the 98th percentile of the residual log2(1 + nnz) - yhat
over such rows of held-out products (RMAT scale 17 A * A, and RMAT scale 16
times a 4096-column matrix): about 2% of the rows it sizes overflow.

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
DEFAULT_PATH = os.path.join(HERE, "data", "predictor_v2.bin")

# (scale, edge factor, seed, columns of a uniform B with 16 per row, or 0 for A * A)
TRAIN_SET = [(s, ef, seed, 0) for s in range(12, 18) for ef in (8, 16) for seed in (1, 2)] + \
    [(s, ef, 1, n) for s in range(12, 17) for ef in (8, 16) for n in (1024, 4096)]
HOLDOUT = [(17, 16, 3, 0), (16, 8, 3, 4096)]
LDS_ROW_MAX = 1024


def _operands(spec):
    import synthetic as syn
    scale, ef, seed, ncols = spec
    A = syn.rmat(scale, ef, 0xB0A7 + 97 * seed + scale, np.float32)
    B = A if ncols == 0 else syn.uniform_k_per_row(A.cols, ncols, 16, 0xB1B + 31 * seed + scale, np.float32)
    return A, B


def _rows(ctx, smash, A, B):
    """Features and exact counts of every row of A * B with products."""
    import torch
    dA = smash.to_device(A)
    dB = dA if B is A else smash.to_device(B)
    feats = ctx.features(dA, dB)
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    ctx.symbolic(dA, dB, rp)
    cnt = (rp[1:] - rp[:-1]).to(torch.float32)
    keep = feats[:, 1] > 0           # ub_i > 0
    return feats[keep].contiguous(), torch.log2(1 + cnt[keep]).contiguous()


def build_dataset(ctx, smash, spec, log=print):
    import torch
    fs, ys = [], []
    for sp in spec:
        A, B = _operands(sp)
        f, y = _rows(ctx, smash, A, B)
        fs.append(f)
        ys.append(y)
        log(f"  rmat s{sp[0]} ef{sp[1]} seed{sp[2]} " + ("* itself" if sp[3] == 0 else f"* uniform {sp[3]} cols") +
            f": {y.numel()} rows")
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
    Fh, Yh = build_dataset(ctx, smash, HOLDOUT, log)
    yhat = ctx.mlp_predict(Fh, params, ms)
    res = (Yh - yhat).cpu().numpy()
    # feature 4 is log2(1 + min(ub, cols)): the rows the fused pass asks about
    asked = (Fh[:, 4] > float(np.log2(1 + LDS_ROW_MAX))).cpu().numpy()
    delta = float(max(0.0, np.quantile(res[asked], 0.98))) if asked.any() else 0.0
    mae = float(np.mean(np.abs(res)))
    mae_asked = float(np.mean(np.abs(res[asked]))) if asked.any() else 0.0
    log(f"held-out: log2 MAE {mae:.4f} (rows above the LDS limit: {mae_asked:.4f}, {int(asked.sum())} rows), "
        f"delta {delta:.4f}")
    ctx.close()
    return (params.cpu().numpy(), ms.cpu().numpy(), delta,
            {"rows": n, "epochs": epochs, "loss": losses.tolist(), "holdout_log2_mae": mae,
             "holdout_log2_mae_above_limit": mae_asked, "delta": delta})


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
