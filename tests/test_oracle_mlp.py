"""Pins of the FP64 surrogate oracle (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp


def _loop_forward(params, x):
    """Pure-Python evaluation of the same definition (no numpy algebra)."""
    out = []
    for row in x:
        h = [float(v) for v in row]
        for li, (W, b) in enumerate(params):
            K, N = W.shape
            z = [sum(h[k] * float(W[k, n]) for k in range(K)) + float(b[n]) for n in range(N)]
            if li < len(params) - 1:
                h = [0.5 * v * (1 + math.tanh(math.sqrt(2 / math.pi) * (v + 0.044715 * v ** 3))) for v in z]
            else:
                m = max(z)
                e = [math.exp(v - m) for v in z]
                s = sum(e)
                h = [v / s for v in e]
        out.append(h)
    return np.array(out)


def test_forward_matches_loop_evaluation():
    params = mlp.init(3, sizes=(8, 5, 4, 6, 3))
    rng = np.random.default_rng(1)
    for W, b in params:
        b[:] = rng.normal(0, 0.3, b.shape)
    x = rng.normal(size=(7, 8))
    p, _ = mlp.forward(params, x)
    assert np.allclose(p, _loop_forward(params, x), rtol=0, atol=1e-14)
    assert np.allclose(p.sum(1), 1.0, atol=1e-15)


def test_gelu_values_and_derivative():
    z = np.linspace(-6, 6, 241)
    g = mlp.gelu(z)
    assert abs(mlp.gelu(np.array([0.0]))[0]) == 0.0
    assert np.allclose(g[z > 5], z[z > 5], rtol=1e-6)
    assert np.all(np.abs(g[z < -5]) < 1e-6)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_backward_matches_central_finite_differences():
    params = mlp.init(5, sizes=(8, 6, 5, 7, 3))
    rng = np.random.default_rng(2)
    for W, b in params:
        b[:] = rng.normal(0, 0.2, b.shape)
    x = rng.normal(size=(9, 8))
    y = rng.dirichlet(np.ones(3), size=9)
    p, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, p, y)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss(mlp.forward(params, x)[0], y)
                flat[idx] = old - h
                lm = mlp.loss(mlp.forward(params, x)[0], y)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (li, idx, fd, gflat[idx])


def test_logit_gradient_is_p_minus_y():
    params = mlp.init(0, sizes=(8, 4, 3))
    x = np.random.default_rng(0).normal(size=(5, 8))
    y = np.full((5, 3), 1 / 3)
    p, cache = mlp.forward(params, x)
    g = mlp.backward(params, cache, p, y)
    assert np.allclose(g[-1][1], (p - y).sum(0) / 5, atol=1e-15)


def test_adam_first_step_moves_by_lr_times_sign():
    params = mlp.init(1, sizes=(8, 4, 3))
    grads = [(np.full_like(W, 0.37) * np.sign(np.random.default_rng(3).normal(size=W.shape)), -0.5 * np.ones_like(b))
             for W, b in params]
    opt = mlp.Adam(params, lr=1e-3)
    new = opt.step(params, grads)
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, new, grads):
        assert np.allclose(W1 - W0, -1e-3 * np.sign(gW), rtol=1e-6)
        assert np.allclose(b1 - b0, -1e-3 * np.sign(gb), rtol=1e-6)


def test_adam_constant_gradient_moves_by_lr_every_step():
    # with a gradient that never changes, the bias-corrected moments are
    # exactly g and g^2 at every step t, so each step moves every weight by
    # lr g / (|g| + eps) -- steps 2..10 fail without the (1 - beta^t)
    # corrections or with a correction that does not follow t
    params = mlp.init(2, sizes=(8, 4, 3))
    rng = np.random.default_rng(5)
    grads = [(rng.choice([-1.0, 1.0], size=W.shape) * rng.uniform(0.01, 3.0, size=W.shape),
              rng.uniform(-2.0, 2.0, size=b.shape)) for W, b in params]
    eps = 1e-8
    opt = mlp.Adam(params, lr=2e-3, eps=eps)
    cur = params
    for t in range(1, 11):
        lr = 2e-3 * (1.0 - 0.05 * t)       # a schedule changes only the step size
        new = opt.step(cur, grads, lr=lr)
        for (W0, b0), (W1, b1), (gW, gb) in zip(cur, new, grads):
            assert np.allclose(W1 - W0, -lr * gW / (np.abs(gW) + eps), rtol=1e-9, atol=0)
            assert np.allclose(b1 - b0, -lr * gb / (np.abs(gb) + eps), rtol=1e-9, atol=0)
        cur = new


def test_adam_alternating_gradient_closed_form():
    # gradients g, -g, g, -g, ...: the first moment is the geometric sum
    # m_t = (1 - b1) g (-1)^(t-1) (1 - (-b1)^t) / (1 + b1) and the second
    # v_t = (1 - b2^t) g^2, so the step of iteration t is
    # lr m_t / (1 - b1^t) / (sqrt(v_t / (1 - b2^t)) + eps)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-3
    params = mlp.init(4, sizes=(8, 3))
    g = np.random.default_rng(6).normal(size=params[0][0].shape)
    opt = mlp.Adam(params, lr=lr, b1=b1, b2=b2, eps=eps)
    cur = params
    for t in range(1, 13):
        s = (-1.0) ** (t - 1)
        new = opt.step(cur, [(s * g, np.zeros_like(params[0][1]))])
        m = (1 - b1) * g * s * (1 - (-b1) ** t) / (1 + b1)
        step = lr * (m / (1 - b1**t)) / (np.abs(g) + eps)
        assert np.allclose(new[0][0] - cur[0][0], -step, rtol=1e-9, atol=1e-18)
        cur = new


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(256, 8))
    logits = np.stack([x[:, 0], x[:, 1] - x[:, 2], 0.5 * x[:, 3]], 1)
    y = mlp.softmax(logits)
    params = mlp.init(6, sizes=(8, 32, 32, 3))
    opt = mlp.Adam(params, lr=3e-3)
    l0 = mlp.loss(mlp.forward(params, x)[0], y)
    for _ in range(200):
        p, c = mlp.forward(params, x)
        params = opt.step(params, mlp.backward(params, c, p, y))
    l1 = mlp.loss(mlp.forward(params, x)[0], y)
    ent = mlp.loss(y, y)   # the floor: entropy of the targets
    assert l1 - ent < 0.1 * (l0 - ent)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7 + 2**-9, -3.14159, 1e-30])
    r = mlp.to_bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0          # tie rounds to even
    assert r[2] == 1.0 + 2**-7
    assert abs(r[3] + 3.140625) < 1e-12
