"""GPU predictor kernels (features, inference, gradients, Adam training)
against the numpy FP64 oracle, and GPU training against a closed form (the
least-squares fit of an affine target, reached in the network's linear
regime)."""
import numpy as np
import pytest

import synthetic as syn
from oracle import mlp
from tests._mlp_cases import AFFINE_SCHEDULE, affine_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_14156_amd import smash
    assert torch.cuda.is_available()
    ctx = smash.Context(0)
    yield torch, smash, ctx
    ctx.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_features_match_oracle(env, oracle_mod):
    torch, smash, ctx = env
    A = syn.rmat(12, 8, 21, np.float32)
    B = syn.uniform_k_per_row(A.cols, 3000, 7, 22, np.float32)
    for (X, Y) in ((A, A), (A, B)):
        F = ctx.features(smash.to_device(X), smash.to_device(Y)).cpu().numpy()
        ref = mlp.features(X, Y)
        np.testing.assert_allclose(F, ref, rtol=2e-6, atol=1e-6)


def _setup(torch, n=3000, seed=3):
    F = np.abs(syn.normal01(seed, 0, n * 6).reshape(n, 6)) * 4
    y = F[:, 1] * 0.7 + np.sin(F[:, 0]) + 0.1 * syn.normal01(seed + 1, 0, n)
    mean, std = F.mean(0), F.std(0)
    ms = np.concatenate([mean, std])
    th = syn.mlp_init(seed) + 0.01 * syn.normal01(seed + 2, 0, syn.MLP_PARAMS)
    t = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    return F, y, ms, th, t


def test_predict_and_gradient_parity(env):
    torch, smash, ctx = env
    F, y, ms, th, t = _setup(torch)
    X = (F - ms[:6]) / ms[6:]
    yhat = ctx.mlp_predict(t(F), t(th), t(ms)).cpu().numpy()
    ref, _ = mlp.forward(th, X)
    assert np.max(np.abs(yhat - ref)) < 1e-4 * max(1.0, np.abs(ref).max())
    idx = np.sort((syn.uniform01(9, 0, 1000) * len(y)).astype(np.int32))
    loss, grad = ctx.mlp_loss_grad(t(F), t(y), t(idx, torch.int32), t(ms), t(th))
    rloss, rgrad = mlp.loss_grad(th, X[idx], y[idx])
    assert abs(loss - rloss) <= 1e-5 * rloss
    g = grad.cpu().numpy().astype(np.float64)
    pos = 0
    for name, shape in syn.MLP_LAYOUT:
        k = int(np.prod(shape))
        assert _rel(g[pos:pos + k], rgrad[pos:pos + k]) < 1e-4, name
        pos += k


def test_training_parity(env):
    torch, smash, ctx = env
    F, y, ms, th, t = _setup(torch, n=2000, seed=5)
    orders = syn.batch_orders(len(y), 4, 77)
    p = t(th)
    losses = ctx.mlp_train(t(F), t(y), t(ms), p, t(orders, torch.int32), batch=256, lr=1e-3)
    rth, rlosses = mlp.train(th, F, y, ms[:6], ms[6:], orders, 256, lr=1e-3)
    np.testing.assert_allclose(losses, rlosses, rtol=1e-3)
    assert _rel(p.cpu().numpy().astype(np.float64), rth) < 1e-4
    assert losses[-1] < losses[0]


def test_training_affine_target_reaches_lstsq(env):
    """smash_mlp_train (full-batch Adam, FP32) on an exact affine target from
    the linear regime ends at numpy's least-squares fit."""
    torch, smash, ctx = env
    F, y, mean, std, th, fitted = affine_case()
    n = len(y)
    t = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    ms = t(np.concatenate([mean, std]))
    p = t(th)
    for lr, epochs in AFFINE_SCHEDULE:
        losses = ctx.mlp_train(t(F), t(y), ms, p, t(syn.batch_orders(n, epochs, 3), torch.int32), batch=n, lr=lr)
    yhat = ctx.mlp_predict(t(F), p, ms).cpu().numpy().astype(np.float64)
    dev = float(np.max(np.abs(yhat - fitted)))
    print(f"max |yhat - lstsq fit| = {dev:.2e} (fit spread {fitted.std():.2f}); final loss {losses[-1]:.2e}")
    assert dev < 1e-2
    assert losses[-1] < 1e-5 * y.var()
