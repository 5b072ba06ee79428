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


# ---- hand-computed pins of the BF16-emulating mode's rounding points ------
# Scalar nets (every layer one unit wide).  Layers after the one under test
# pass their input through exactly: for a BF16 value h with |W h| <= 2^-5 and
# W a power of two, tanh(W h) = W h (1 - (W h)^2 / 3 + ...) differs from W h by
# less than a quarter of BF16's spacing, so bf16(tanh(W h)) = W h.  Each pin
# states the output with the rounding (asserted for mode "bf16") and without
# it (what "fp64" mode, which rounds nowhere, gives): dropping the rounding
# point changes the answer.

def _net(*layers):
    """layers: (W [out, in] as nested lists, b list) per layer."""
    return [(np.array(W, dtype=np.float64), np.array(b, dtype=np.float64)) for W, b in layers]


def test_bf16_pin_input_rounding():
    # x = 1 + 2^-9 rounds to bf16 1 (spacing 2^-7 at 1); z1 = 1 * 1 - 1 = 0, so
    # h1 = h2 = h3 = 0 and out = 2^9 * 0 = 0.  Unrounded: z1 = 2^-9, passed
    # through, out = 2^9 * 2^-9 = 1.
    p = _net(([[1.0]], [-1.0]), ([[1.0]], [0.0]), ([[1.0]], [0.0]), ([[2.0 ** 9]], [0.0]))
    X = np.array([[1.0 + 2.0 ** -9]])
    assert mlp.forward(p, X, "bf16")[0][0] == 0.0
    assert abs(mlp.forward(p, X, "fp64")[0][0] - 1.0) < 1e-5


def test_bf16_pin_weight_rounding():
    # W1 = 1 + 2^-9 rounds to 1: z1 = 0 -> out 0; unrounded z1 = 2^-9 -> out 1
    p = _net(([[1.0 + 2.0 ** -9]], [-1.0]), ([[1.0]], [0.0]), ([[1.0]], [0.0]), ([[2.0 ** 9]], [0.0]))
    X = np.array([[1.0]])
    assert mlp.forward(p, X, "bf16")[0][0] == 0.0
    assert abs(mlp.forward(p, X, "fp64")[0][0] - 1.0) < 1e-5


def test_bf16_pin_fp32_accumulation():
    # x = (1, 2^-30), W1 = (1, 1), both exact in BF16: the FP32 sum 1 + 2^-30
    # is 1 (FP32 spacing at 1 is 2^-23), minus the bias 1 gives z1 = 0 and
    # out = 0; accumulated in FP64 it is 2^-30 and out = 2^30 * 2^-30 = 1.
    p = _net(([[1.0, 1.0]], [-1.0]), ([[1.0]], [0.0]), ([[1.0]], [0.0]), ([[2.0 ** 30]], [0.0]))
    X = np.array([[1.0, 2.0 ** -30]])
    assert mlp.forward(p, X, "bf16")[0][0] == 0.0
    assert abs(mlp.forward(p, X, "fp64")[0][0] - 1.0) < 1e-5


def test_bf16_pin_fp32_bias():
    # b1 = 1 + 2^-40 is 1 in FP32: z1 = -1 + 1 = 0, out 0; in FP64 z1 = 2^-40
    # and out = 2^40 * 2^-40 = 1
    p = _net(([[-1.0]], [1.0 + 2.0 ** -40]), ([[1.0]], [0.0]), ([[1.0]], [0.0]), ([[2.0 ** 40]], [0.0]))
    X = np.array([[1.0]])
    assert mlp.forward(p, X, "bf16")[0][0] == 0.0
    assert abs(mlp.forward(p, X, "fp64")[0][0] - 1.0) < 1e-5


def test_bf16_pin_activation_rounding():
    # h1 = bf16(tanh(0.5)) = bf16(0.4621171...) = 237 * 2^-9 (spacing 2^-9 in
    # [0.25, 0.5): 0.4621171 / 2^-9 = 236.60); W2 = 2^-5 gives 237 * 2^-14,
    # which layers 2 and 3 pass through (tanh(0.0144653) = 0.0144643 is
    # 236.98 * 2^-14 -> 237 * 2^-14), and out = 2^14 * 237 * 2^-14 = 237.
    # Unrounded activations: out = 2^14 tanh(tanh(2^-5 tanh(0.5))) = 236.57.
    p = _net(([[1.0]], [0.0]), ([[2.0 ** -5]], [0.0]), ([[1.0]], [0.0]), ([[2.0 ** 14]], [0.0]))
    X = np.array([[0.5]])
    assert mlp.forward(p, X, "bf16")[0][0] == 237.0
    o64 = mlp.forward(p, X, "fp64")[0][0]
    assert abs(o64 - 236.57) < 0.01


def test_bf16_pin_delta_rounding():
    # the activation pin's net (out = 237) with target y = 237 - (1 + 2^-9) / 2:
    # dL/dout = 2 (out - y) / 1 = 1 + 2^-9, which rounds to bf16 1, so
    # dW4 = 1 * h3 = 237 * 2^-14 exactly; without the rounding it would be
    # (1 + 2^-9) 237 * 2^-14.
    p = _net(([[1.0]], [0.0]), ([[2.0 ** -5]], [0.0]), ([[1.0]], [0.0]), ([[2.0 ** 14]], [0.0]))
    X = np.array([[0.5]])
    y = np.array([237.0 - (1.0 + 2.0 ** -9) / 2.0])
    _, g = mlp.loss_and_grads(p, X, y, "bf16")
    assert g[3][0][0, 0] == 237.0 * 2.0 ** -14
    assert g[3][0][0, 0] != (1.0 + 2.0 ** -9) * 237.0 * 2.0 ** -14


def test_bf16_pin_weight_gradient_fp32_accumulation():
    # W1 = 0 and zero biases make every activation 0 for both samples, so
    # out = b4 = 1 and, with y = 0 and a batch of 2, dL/dout = 2 * 1 / 2 = 1;
    # back through W4 = W3 = W2 = 1 and (1 - 0^2) every sample's layer-1
    # delta is 1.  dW1 = 1 * 1 + 1 * 2^-30 over the batch: 1 in FP32
    # (2^-30 is below half of FP32's spacing at 1), 1 + 2^-30 in FP64.
    p = _net(([[0.0]], [0.0]), ([[1.0]], [0.0]), ([[1.0]], [0.0]), ([[1.0]], [1.0]))
    X = np.array([[1.0], [2.0 ** -30]])
    y = np.zeros(2)
    _, g16 = mlp.loss_and_grads(p, X, y, "bf16")
    _, g64 = mlp.loss_and_grads(p, X, y, "fp64")
    assert g16[0][0][0, 0] == 1.0
    assert g64[0][0][0, 0] == 1.0 + 2.0 ** -30
