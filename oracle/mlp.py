"""CPU oracle of the row-size predictor -- TEST INFRASTRUCTURE ONLY.

A plain numpy float64 implementation of the MLP 6 -> 64 -> 64 -> 1 with ReLU
hidden layers, mean-squared-error loss, hand-written backpropagation and the
Adam update (Kingma and Ba, 2015), on the packed parameter layout of
synthetic.MLP_LAYOUT.  Also the six per-row features the predictor reads.
The predictor is an addition to the paper's method (its nearest hook is the
flop-estimate work distribution of its Future Work section); its target is
log2(1 + nnz(C_i)).
"""
from __future__ import annotations

import numpy as np

from synthetic import MLP_FEATURES, MLP_HIDDEN, MLP_LAYOUT, MLP_PARAMS


def unpack(theta):
    out, pos = {}, 0
    for name, shape in MLP_LAYOUT:
        n = int(np.prod(shape))
        out[name] = theta[pos:pos + n].reshape(shape)
        pos += n
    return out


def features(A, B) -> np.ndarray:
    """Per row i of C = A*B: log2(1+x) of nnz(A_i), the products ub_i, the
    largest and smallest nnz(B_k) over the row's k, min(ub_i, cols(B)) and
    sum_k nnz(B_k)^2 / ub_i.  float64 (m x 6); empty rows give zeros."""
    brow = np.diff(B.row_ptr.astype(np.int64))
    rp = A.row_ptr.astype(np.int64)
    m = A.rows
    F = np.zeros((m, MLP_FEATURES))
    for i in range(m):
        ks = A.col_idx[rp[i]:rp[i + 1]]
        if ks.size == 0:
            continue
        L = brow[ks].astype(np.float64)
        ub = L.sum()
        F[i, 0] = np.log2(1 + ks.size)
        F[i, 1] = np.log2(1 + ub)
        F[i, 2] = np.log2(1 + L.max())
        F[i, 3] = np.log2(1 + L.min())
        F[i, 4] = np.log2(1 + min(ub, B.cols))
        F[i, 5] = np.log2(1 + ((L * L).sum() / ub if ub > 0 else 0.0))
    return F


def standardize(F, mean, std):
    return (F - mean) / std


def forward(theta, X):
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    yhat = h2 @ p["w3"] + p["b3"][0]
    return yhat, (X, z1, h1, z2, h2)


def loss_grad(theta, X, y):
    """MSE loss over the batch and its gradient (packed), by backpropagation."""
    p = unpack(theta)
    yhat, (X, z1, h1, z2, h2) = forward(theta, X)
    n = X.shape[0]
    r = yhat - y
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return loss, np.concatenate([g[name].reshape(-1) for name, _ in MLP_LAYOUT])


def adam(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta0, F, y, mean, std, orders, batch, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Mini-batch Adam over the epochs given by `orders` (one permutation per
    epoch); returns the parameters and the mean batch loss of every epoch."""
    X = standardize(F, mean, std)
    theta = theta0.astype(np.float64).copy()
    m = np.zeros(MLP_PARAMS)
    v = np.zeros(MLP_PARAMS)
    t = 0
    losses = []
    n = X.shape[0]
    for order in orders:
        tot = 0.0
        steps = 0
        for s in range(0, n, batch):
            idx = order[s:s + batch]
            loss, g = loss_grad(theta, X[idx], y[idx])
            t += 1
            theta, m, v = adam(theta, g, m, v, t, lr, b1, b2, eps)
            tot += loss
            steps += 1
        losses.append(tot / steps)
    return theta, np.array(losses)
