"""Learned temperature initial guess: a small MLP, forward / backward / Adam
(oracle).  Test infrastructure only (see the package docstring).

Reading (the build's learned-guess growth direction; the paper describes
none):
* features x = (log rho, e, Y_1 .. Y_7), standardised by the training
  mean / std; target (T - mu_T) / sigma_T;
* h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), h3 = tanh(W3 h2 + b3),
  out = W4 h3 + b4 with widths 9 -> 64 -> 64 -> 64 -> 1 (9,025 parameters);
* Glorot-uniform weights, zero biases; MSE loss; Adam (lr 1e-3, betas 0.9 /
  0.999, eps 1e-8) on FP32 master weights and moments.
Two arithmetic modes:
* "fp64": everything in double precision (the mathematical reference);
* "bf16": the rounding points of the matrix-core implementation — inputs,
  weights, post-tanh activations and the backward products' operands
  (deltas, weights, activations) rounded to BF16 (nearest, ties to even),
  products accumulated in FP32, bias, tanh and (1 - h^2) in FP32.
"""
from __future__ import annotations

import numpy as np

from .precision import round_bf16

WIDTHS = (9, 64, 64, 64, 1)


def n_params() -> int:
    return sum(WIDTHS[i] * WIDTHS[i + 1] + WIDTHS[i + 1] for i in range(4))


def init_params(seed: int = 4002):
    rng = np.random.default_rng(seed)
    params = []
    for i in range(4):
        fi, fo = WIDTHS[i], WIDTHS[i + 1]
        lim = np.sqrt(6.0 / (fi + fo))
        params.append((rng.uniform(-lim, lim, (fo, fi)), np.zeros(fo)))
    return params


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _mm(A, B, mode):
    """A @ B with the mode's operand rounding and accumulation."""
    if mode == "fp64":
        return A @ B
    return (_f32(round_bf16(A)) @ _f32(round_bf16(B))).astype(np.float64)


def forward(params, X, mode="fp64"):
    """X [B, 9] -> (out [B], cache)."""
    h = X
    cache = [h]
    for i, (W, b) in enumerate(params):
        z = _mm(h, W.T, mode)
        if mode == "bf16":
            z = (_f32(z) + _f32(b)).astype(np.float64)
        else:
            z = z + b
        if i < 3:
            if mode == "bf16":
                h = round_bf16(np.tanh(_f32(z)).astype(np.float64))
            else:
                h = np.tanh(z)
            cache.append(h)
        else:
            h = z
    return h[:, 0], cache


def loss_and_grads(params, X, y, mode="fp64"):
    """MSE loss mean((out - y)^2) and its gradients [(dW, db), ...]."""
    out, cache = forward(params, X, mode)
    B = X.shape[0]
    r = out - y
    loss = float(np.mean(r * r))
    delta = (2.0 / B) * r[:, None]  # dL/dout, [B, 1]
    grads = [None] * 4
    for i in range(3, -1, -1):
        W, _ = params[i]
        h_in = cache[i]
        dW = _mm(delta.T, h_in, mode)
        db = delta.sum(axis=0)
        grads[i] = (dW, db)
        if i > 0:
            g = _mm(delta, W, mode)
            h = cache[i]
            if mode == "bf16":
                delta = (_f32(g) * (np.float32(1.0) - _f32(h) * _f32(h))).astype(np.float64)
            else:
                delta = g * (1.0 - h * h)
    return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        new = []
        for i, ((W, b), (dW, db)) in enumerate(zip(params, grads)):
            out = []
            for j, (p, g) in enumerate(((W, dW), (b, db))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * g
                v = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                self.m[i] = (m, self.m[i][1]) if j == 0 else (self.m[i][0], m)
                self.v[i] = (v, self.v[i][1]) if j == 0 else (self.v[i][0], v)
                out.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            new.append(tuple(out))
        return new


def normalization(F, T):
    """Feature means / standard deviations and target mean / std of a
    training set; a (numerically) constant feature, std < 1e-6 max(|mean|, 1),
    is centred but not scaled (std := 1)."""
    mean = F.mean(axis=0)
    std = F.std(axis=0)
    std = np.where(std >= 1e-6 * np.maximum(np.abs(mean), 1.0), std, 1.0)
    return mean, std, float(np.mean(T)), float(np.std(T))


def features(q):
    """Raw features (log rho, e, Y_1 .. Y_7) [n, 9] of a reacting state q[12][...]."""
    rho = q[0].ravel()
    u, v, w = q[1].ravel() / rho, q[2].ravel() / rho, q[3].ravel() / rho
    e = q[4].ravel() / rho - 0.5 * (u * u + v * v + w * w)
    Y = q[5:].reshape(q.shape[0] - 5, -1) / rho
    return np.concatenate([np.log(rho)[:, None], e[:, None], Y.T], axis=1)
