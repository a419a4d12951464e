"""Pins of the oracle's learned warm-start MLP (12 -> 64 -> 64 -> 64 -> 3,
SiLU): special parameter choices with closed-form outputs, the analytic
gradient against central finite differences, Adam's first step, and a loss
decrease on a fitted function.  CPU only."""
import numpy as np
import pytest

import oracle as O

NP = 9347
SIZES = [(64, 12), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]


def split(theta):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def test_param_count():
    assert O.mlp_nparam() == NP == sum(int(np.prod(s)) for s in SIZES)


def test_bias_only_output():
    th = np.zeros(NP)
    split(th)[7][:] = [0.3, -1.2, 2.5]
    x = np.random.default_rng(0).normal(size=(5, 12))
    np.testing.assert_allclose(O.mlp_forward(th, x), np.tile([0.3, -1.2, 2.5], (5, 1)), atol=0)


def test_activation_is_silu():
    """A chain that passes x_0 through the three hidden units 0 gives
    y_0 = silu(silu(silu(x_0))) with silu(z) = z / (1 + exp(-z))."""
    th = np.zeros(NP)
    W1, b1, W2, b2, W3, b3, W4, b4 = split(th)
    W1[0, 0] = W2[0, 0] = W3[0, 0] = W4[0, 0] = 1.0
    silu = lambda z: z / (1.0 + np.exp(-z))
    x = np.zeros((4, 12))
    x[:, 0] = [-3.0, -0.5, 0.7, 4.0]
    y = O.mlp_forward(th, x)
    np.testing.assert_allclose(y[:, 0], silu(silu(silu(x[:, 0]))), rtol=1e-14)
    np.testing.assert_allclose(y[:, 1:], 0.0, atol=0)


def test_weight_layout_out_by_in():
    """The flat layout is row-major out x in: one non-symmetric path
    W1[3][7], W2[5][3], W3[9][5], W4[2][9] = 1 routes input 7 through hidden
    units 3, 5 and 9 to output 2, so y_2 = silu(silu(silu(x_7))), the other
    outputs are 0 and no other input matters.  A transposed (in x out) read
    of any of the four matrices sends the path elsewhere."""
    th = np.zeros(NP)
    W1, b1, W2, b2, W3, b3, W4, b4 = split(th)
    W1[3, 7] = W2[5, 3] = W3[9, 5] = W4[2, 9] = 1.0
    silu = lambda z: z / (1.0 + np.exp(-z))
    rng = np.random.default_rng(5)
    x = rng.normal(size=(6, 12))
    x[:, 7] = [-2.5, -0.3, 0.0, 0.4, 1.1, 3.0]
    y = O.mlp_forward(th, x)
    np.testing.assert_allclose(y[:, 2], silu(silu(silu(x[:, 7]))), rtol=1e-14, atol=1e-300)
    np.testing.assert_array_equal(y[:, :2], 0.0)
    x2 = rng.normal(size=(6, 12))
    x2[:, 7] = x[:, 7]
    np.testing.assert_array_equal(O.mlp_forward(th, x2), y)


def test_loss_zero_at_fit():
    rng = np.random.default_rng(1)
    th = rng.normal(scale=0.2, size=NP)
    x = rng.normal(size=(7, 12))
    t = O.mlp_forward(th, x)
    loss, g = O.mlp_loss_grad(th, x, t)
    assert loss == 0.0
    np.testing.assert_array_equal(g, 0.0)


def test_gradient_finite_differences():
    rng = np.random.default_rng(2)
    th = rng.normal(scale=0.3, size=NP)
    x = rng.normal(size=(6, 12))
    t = rng.normal(size=(6, 3))
    loss, g = O.mlp_loss_grad(th, x, t)
    # the loss is the stated mean squared error
    assert abs(loss - np.mean((O.mlp_forward(th, x) - t) ** 2)) < 1e-14
    idx = rng.choice(NP, size=80, replace=False)
    idx = np.concatenate([idx, [0, 767, 768, 831, 832, 4927, 9151, 9152, 9346]])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (O.mlp_loss_grad(tp, x, t)[0] - O.mlp_loss_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_adam_first_step():
    """With m = v = 0 the bias-corrected first step moves every parameter
    by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    th = rng.normal(size=NP)
    g = rng.normal(size=NP)
    m, v = np.zeros(NP), np.zeros(NP)
    th0 = th.copy()
    O.adam_step(th, g, m, v, 1, 1e-3)
    np.testing.assert_allclose(th, th0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(256, 12))
    A = rng.normal(scale=0.3, size=(12, 3))
    t = np.tanh(x @ A)
    th = rng.normal(scale=0.1, size=NP)
    m, v = np.zeros(NP), np.zeros(NP)
    l0, _ = O.mlp_loss_grad(th, x, t)
    for s in range(1, 301):
        _, g = O.mlp_loss_grad(th, x, t)
        O.adam_step(th, g, m, v, s, 3e-3)
    l1, _ = O.mlp_loss_grad(th, x, t)
    assert l1 < 0.05 * l0
