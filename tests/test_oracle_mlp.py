"""Pins of the oracle MLP: parameter count, FP64 backward against central
finite differences, the BF16-emulating forward within BF16 rounding of FP64,
Adam's closed-form first step, and that training fits a known function."""
import numpy as np

from oracle import mlp


def _data(n=256, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 9))
    y = np.tanh(X[:, 0] - 0.5 * X[:, 1]) + 0.3 * X[:, 2] * X[:, 3]
    return X, y


def test_parameter_count():
    assert mlp.n_params() == 9025
    p = mlp.init_params(1)
    assert sum(W.size + b.size for W, b in p) == 9025
    for W, b in p:
        lim = np.sqrt(6.0 / (W.shape[0] + W.shape[1]))
        assert np.abs(W).max() <= lim and np.all(b == 0)


def test_fp64_backward_matches_finite_differences():
    X, y = _data(64)
    p = mlp.init_params(2)
    p = [(W, b + 0.05 * np.random.default_rng(5).standard_normal(b.shape)) for W, b in p]
    _, grads = mlp.loss_and_grads(p, X, y, "fp64")
    rng = np.random.default_rng(3)
    h = 1e-6
    for li in range(4):
        for which in (0, 1):
            P = p[li][which]
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in P.shape)
                orig = P[idx]
                P[idx] = orig + h
                lp, _ = mlp.loss_and_grads(p, X, y, "fp64")
                P[idx] = orig - h
                lm, _ = mlp.loss_and_grads(p, X, y, "fp64")
                P[idx] = orig
                fd = (lp - lm) / (2 * h)
                an = grads[li][which][idx]
                assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (li, which, idx, fd, an)


def test_bf16_forward_and_grads_close_to_fp64():
    X, y = _data(512)
    p = mlp.init_params(4)
    o64, _ = mlp.forward(p, X, "fp64")
    o16, _ = mlp.forward(p, X, "bf16")
    assert np.abs(o16 - o64).max() < 0.05 * np.abs(o64).max()  # a few BF16 roundings deep
    _, g64 = mlp.loss_and_grads(p, X, y, "fp64")
    _, g16 = mlp.loss_and_grads(p, X, y, "bf16")
    for (a, _), (b, _) in zip(g64, g16):
        assert np.linalg.norm(a - b) < 0.05 * np.linalg.norm(a)


def test_adam_first_step_closed_form():
    p = mlp.init_params(6)
    X, y = _data(32)
    _, g = mlp.loss_and_grads(p, X, y)
    opt = mlp.Adam(p, lr=1e-3)
    new = opt.step(p, g)
    for (W, b), (W1, b1), (dW, db) in zip(p, new, g):
        np.testing.assert_allclose(W1 - W, -1e-3 * dW / (np.abs(dW) + 1e-8), rtol=1e-9, atol=1e-15)


def test_training_reduces_loss():
    X, y = _data(2048, seed=7)
    p = mlp.init_params(8)
    opt = mlp.Adam(p, lr=3e-3)
    l0, _ = mlp.loss_and_grads(p, X, y, "bf16")
    for it in range(300):
        sl = slice((it * 256) % 2048, (it * 256) % 2048 + 256)
        _, g = mlp.loss_and_grads(p, X[sl], y[sl], "bf16")
        p = opt.step(p, g)
    l1, _ = mlp.loss_and_grads(p, X, y, "bf16")
    assert l1 < 0.1 * l0


def test_normalization_centres_constant_features():
    rng = np.random.default_rng(9)
    F = rng.standard_normal((500, 9))
    F[:, 8] = 0.72  # constant (inert species)
    mean, std, tm, ts = mlp.normalization(F, rng.uniform(300, 2000, 500))
    assert std[8] == 1.0 and abs(mean[8] - 0.72) < 1e-13
    np.testing.assert_allclose(std[:8], F[:, :8].std(0))
