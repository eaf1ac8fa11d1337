"""Pins for the predictor's CPU oracle: central finite differences, torch's
autograd (an independent implementation) and torch.optim.Adam."""
import numpy as np
import torch

import synthetic as syn
from oracle import mlp


def _data(n=37, seed=5):
    X = syn.normal01(seed, 0, n * 6).reshape(n, 6)
    y = syn.normal01(seed + 1, 0, n)
    return X, y


def test_layout():
    assert syn.MLP_PARAMS == 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1 == 4673
    th = syn.mlp_init()
    assert th.shape == (4673,)
    p = mlp.unpack(th)
    assert np.all(p["b1"] == 0) and np.all(p["b2"] == 0) and p["b3"][0] == 0
    assert abs(p["W2"].std() - np.sqrt(2 / 64)) < 0.01


def test_finite_differences():
    X, y = _data()
    th = syn.mlp_init(3) + 0.01 * syn.normal01(9, 0, syn.MLP_PARAMS)
    loss, g = mlp.loss_grad(th, X, y)
    idx = (syn.uniform01(17, 0, 60) * syn.MLP_PARAMS).astype(np.int64)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss_grad(th + e, X, y)[0] - mlp.loss_grad(th - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_against_torch_autograd():
    X, y = _data(64, 7)
    th = syn.mlp_init(4)
    loss, g = mlp.loss_grad(th, X, y)
    t = torch.tensor(th, requires_grad=True, dtype=torch.float64)
    sizes = [int(np.prod(s)) for _, s in syn.MLP_LAYOUT]
    W1, b1, W2, b2, w3, b3 = torch.split(t, sizes)
    W1 = W1.view(64, 6); W2 = W2.view(64, 64)
    Xt = torch.tensor(X); yt = torch.tensor(y)
    h1 = torch.relu(Xt @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    yh = h2 @ w3 + b3
    L = ((yh - yt) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    np.testing.assert_allclose(t.grad.numpy(), g, rtol=1e-10, atol=1e-13)


def test_adam_matches_torch():
    th = syn.mlp_init(2)
    X, y = _data(50, 8)
    p = torch.tensor(th, requires_grad=True, dtype=torch.float64)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(th); v = np.zeros_like(th); cur = th.copy()
    for t in range(1, 6):
        _, g = mlp.loss_grad(cur, X, y)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        cur, m, v = mlp.adam(cur, g, m, v, t)
        np.testing.assert_allclose(p.detach().numpy(), cur, rtol=1e-12, atol=1e-15)


def test_features_small(oracle_mod):
    A = syn.CSR(3, 4, np.array([0, 2, 2, 3], np.int32), np.array([0, 3, 1], np.int32), np.ones(3))
    B = syn.CSR(4, 5, np.array([0, 3, 3, 4, 6], np.int32), np.array([0, 1, 2, 4, 0, 3], np.int32), np.ones(6))
    F = mlp.features(A, B)
    # row 0 takes B rows 0 (3 entries) and 3 (2 entries): ub 5, max 3, min 2, sumsq/ub = 13/5
    np.testing.assert_allclose(F[0], np.log2(1 + np.array([2, 5, 3, 2, 5, 13 / 5])))
    assert np.all(F[1] == 0)
    # row 2 takes B row 1, which is empty
    np.testing.assert_allclose(F[2], np.log2(1 + np.array([1, 0, 0, 0, 0, 0])))
    assert np.allclose(oracle_mod.products_per_row(A, B), [5, 0, 0])


def test_training_reduces_loss():
    X, y = _data(512, 11)
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    th, losses = mlp.train(syn.mlp_init(1), X, y, np.zeros(6), np.ones(6), syn.batch_orders(512, 20), 64, lr=3e-3)
    assert losses[-1] < 0.2 * losses[0]
