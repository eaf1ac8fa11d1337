"""Shared training cases of the predictor tests (inputs only; no arithmetic
of the network lives here)."""
import numpy as np

import synthetic as syn

# Affine-target case: y is an exact affine function of the six features, and
# the network starts in its linear regime (every hidden pre-activation
# positive: small first- and second-layer weights, biases of 6).  There the
# 6 -> 64 -> 64 -> 1 ReLU network computes u . x + c with u = w3^T W2 W1, so
# the least-squares optimum of its loss is numpy's lstsq solution of y on
# [x, 1]; training must reach it.  Schedule: Adam at 3e-4, then at 3e-5.
AFFINE_SCHEDULE = ((3e-4, 3000), (3e-5, 2000))


def affine_case(n=512):
    F = np.abs(syn.normal01(31, 0, n * 6).reshape(n, 6)) * 3
    beta = np.array([0.7, -0.4, 0.25, 1.1, -0.8, 0.3])
    y = F @ beta + 0.5
    mean, std = F.mean(0), F.std(0)
    X = (F - mean) / std
    Xa = np.hstack([X, np.ones((n, 1))])
    coef = np.linalg.lstsq(Xa, y, rcond=None)[0]
    th = syn.mlp_init(8)
    sizes = [int(np.prod(s)) for _, s in syn.MLP_LAYOUT]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    part = {name: th[offs[i]:offs[i + 1]] for i, (name, _) in enumerate(syn.MLP_LAYOUT)}
    part["W1"] *= 0.1
    part["b1"][:] = 6.0
    part["W2"] *= 0.02
    part["b2"][:] = 6.0
    part["w3"] *= 0.05
    return F, y, mean, std, th, Xa @ coef
