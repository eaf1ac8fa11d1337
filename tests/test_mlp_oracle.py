"""Pins for the predictor's CPU oracle: central finite differences, torch's
autograd (an independent implementation), torch.optim.Adam, a torch training
loop that cuts its own batches, and the least-squares optimum of an affine
target that the network reaches in its linear regime."""
import numpy as np
import torch

import synthetic as syn
from oracle import mlp
from tests._mlp_cases import AFFINE_SCHEDULE, affine_case


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


def _torch_net(p, X):
    sizes = [int(np.prod(s)) for _, s in syn.MLP_LAYOUT]
    W1, b1, W2, b2, w3, b3 = torch.split(p, sizes)
    h1 = torch.relu(X @ W1.view(64, 6).T + b1)
    h2 = torch.relu(h1 @ W2.view(64, 64).T + b2)
    return h2 @ w3 + b3


def test_train_matches_torch_adam_loop():
    """mlp.train against torch autograd + torch.optim.Adam over the same
    epoch orders, with the batches cut by torch.split (300 samples in
    batches of 64: the last batch of every epoch holds 44) and one Adam
    state carried across epochs."""
    n, batch, epochs, lr = 300, 64, 3, 2e-3
    F = np.abs(syn.normal01(21, 0, n * 6).reshape(n, 6)) * 3
    y = np.sin(F[:, 0]) + 0.3 * F[:, 2]
    mean, std = F.mean(0), F.std(0)
    th0 = syn.mlp_init(6)
    orders = syn.batch_orders(n, epochs, 5)
    th, losses = mlp.train(th0, F, y, mean, std, orders, batch, lr=lr)

    p = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    X = torch.tensor((F - mean) / std)
    Y = torch.tensor(y)
    ref_losses = []
    for order in orders:
        batch_losses = []
        for idx in torch.split(torch.as_tensor(np.asarray(order), dtype=torch.long), batch):
            loss = ((_torch_net(p, X[idx]) - Y[idx]) ** 2).mean()
            opt.zero_grad()
            loss.backward()
            opt.step()
            batch_losses.append(loss.item())
        assert len(batch_losses) == 5 and len(idx) == 44
        ref_losses.append(sum(batch_losses) / len(batch_losses))
    np.testing.assert_allclose(losses, ref_losses, rtol=1e-11)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-9, atol=1e-12)


def test_train_affine_target_reaches_lstsq():
    """Closed form: from the linear regime, training on an exact affine target
    ends at numpy's least-squares fit (predictions within 1e-4 of the fitted
    values, whose spread is about 3)."""
    F, y, mean, std, th, fitted = affine_case()
    n = len(y)
    for lr, epochs in AFFINE_SCHEDULE:
        th, losses = mlp.train(th, F, y, mean, std, syn.batch_orders(n, epochs, 3), n, lr=lr)
    yhat, _ = mlp.forward(th, (F - mean) / std)
    assert np.max(np.abs(yhat - fitted)) < 1e-4
    assert losses[-1] < 1e-9 * y.var()
