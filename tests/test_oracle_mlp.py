"""Pins for the oracle's surrogate network: forward and loss gradient against
PyTorch float64 (an independent implementation of the same layers and
autograd), the gradient against central finite differences, and Adam's
first step in closed form (m_hat = g, v_hat = g^2, so the step is
-lr g / (|g| + eps))."""
import numpy as np
import pytest
import torch

import oracle


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    P = oracle.mlp_num_params()
    p = np.zeros(P)
    W1, b1, W2, b2, W3, b3, W4, b4 = oracle.mlp_unpack(p)
    for W, fan in ((W1, 11), (W2, 256), (W3, 256), (W4, 256)):
        W[...] = rng.uniform(-1, 1, W.shape) * scale / np.sqrt(fan)
    for b in (b1, b2, b3, b4):
        b[...] = rng.uniform(-0.1, 0.1, b.shape)
    return p


def _torch_net(p):
    W1, b1, W2, b2, W3, b3, W4, b4 = (torch.tensor(a, dtype=torch.float64, requires_grad=True)
                                      for a in oracle.mlp_unpack(p))
    def f(x):
        h = torch.nn.functional.silu(x @ W1.T + b1)
        h = torch.nn.functional.silu(h @ W2.T + b2)
        h = torch.nn.functional.silu(h @ W3.T + b3)
        return (h @ W4.T + b4)[:, 0]
    return f, (W1, b1, W2, b2, W3, b3, W4, b4)


def test_parameter_count():
    assert oracle.mlp_num_params() == 134913


def test_forward_and_gradient_match_torch():
    p = _params(1)
    rng = np.random.default_rng(2)
    x = rng.random((64, 11))
    x[:, 4:] = 0.0  # four sampled inputs, zero padded
    t = rng.standard_normal(64)
    y = oracle.mlp_forward(p, x)
    f, ws = _torch_net(p)
    yt = f(torch.tensor(x))
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss, g = oracle.mlp_loss_grad(p, x, t)
    lt = torch.mean((yt - torch.tensor(t)) ** 2)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12 * max(1, abs(loss))
    gt = np.concatenate([w.grad.numpy().reshape(-1) for w in ws])
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-12)


def test_gradient_against_finite_differences():
    p = _params(3)
    rng = np.random.default_rng(4)
    x = rng.random((8, 11))
    t = rng.standard_normal(8)
    _, g = oracle.mlp_loss_grad(p, x, t)
    idx = rng.choice(p.size, 40, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.mlp_loss_grad(pp, x, t)[0] - oracle.mlp_loss_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    n = 100
    p = rng.standard_normal(n)
    g = rng.standard_normal(n)
    m = np.zeros(n); v = np.zeros(n)
    p0 = p.copy()
    oracle.adam_step(p, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_constant_gradient_over_many_steps():
    """With a constant gradient the moments are m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected step is -lr g / (|g| + eps)
    at every t: after T steps p = p0 - T lr g / (|g| + eps).  A bias
    correction without the power t (1 - b instead of 1 - b^t) fails from
    t = 2 on."""
    rng = np.random.default_rng(6)
    n, T, lr = 50, 25, 3e-3
    p = rng.standard_normal(n)
    g = rng.standard_normal(n)
    m = np.zeros(n); v = np.zeros(n)
    p0 = p.copy()
    for t in range(1, T + 1):
        oracle.adam_step(p, g, m, v, t, lr=lr, beta1=0.8, beta2=0.95)
        np.testing.assert_allclose(m, (1 - 0.8**t) * g, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(v, (1 - 0.95**t) * g * g, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + 1e-8), rtol=1e-11, atol=1e-13)


def test_adam_sign_flip_closed_form():
    """Gradient +g at t = 1 and -g at t = 2: m_2 = (b1 (1 - b1) - (1 - b1)) g,
    v_2 = (1 - b2^2) g^2, so the second step is
    -lr [(b1 - 1)(1 - b1) / (1 - b1^2)] g / (|g| + eps) = +lr (1 - b1)/(1 + b1) g/(|g| + eps)."""
    rng = np.random.default_rng(7)
    n, lr, b1, b2 = 40, 1e-2, 0.9, 0.999
    p = rng.standard_normal(n)
    g = rng.standard_normal(n) + 0.5
    m = np.zeros(n); v = np.zeros(n)
    oracle.adam_step(p, g, m, v, 1, lr=lr, beta1=b1, beta2=b2)
    p1 = p.copy()
    oracle.adam_step(p, -g, m, v, 2, lr=lr, beta1=b1, beta2=b2)
    want = p1 + lr * (1 - b1) / (1 + b1) * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p, want, rtol=1e-11, atol=1e-14)
