"""FP64 oracle of the MLP surrogate -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this module.  It shares nothing with the HIP kernels.

The network maps the transport problem of one single-layer item to its
R/A/T fractions, replacing the Monte Carlo walk as the paper's pre-trained
network does (Methodology, Photon transport; Table 1 lists that network's
validity domain).  Architecture: 8 inputs -> 4 hidden layers of width 256
with the tanh form of GELU -> 3 logits -> softmax.  Loss: cross-entropy of
the softmax against the Monte Carlo fractions (mean over the batch), whose
gradient with respect to the logits is (p - y) / B.  Optimiser: Adam.

Parity status: forward pinned by a pure-Python loop evaluation on a tiny
network; backward pinned by central finite differences; Adam pinned by its
first-step property (each weight moves by lr * sign(gradient)), by the
constant-gradient property at every later step (the bias-corrected moments
are exactly g and g^2, so each step is lr g / (|g| + eps)) and by the closed
form of the moments under an alternating gradient.
"""
from __future__ import annotations

import math

import numpy as np

GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def gelu(z):
    """0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))."""
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z**3)))


def gelu_grad(z):
    u = GELU_C * (z + GELU_A * z**3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def softmax(a):
    a = a - a.max(axis=1, keepdims=True)
    e = np.exp(a)
    return e / e.sum(axis=1, keepdims=True)


def init(seed: int, sizes=(8, 256, 256, 256, 256, 3)):
    """List of (W [K, N], b [N]) with W ~ N(0, 2/K) (He), b = 0."""
    rng = np.random.default_rng(seed)
    return [(rng.normal(0.0, math.sqrt(2.0 / k), (k, n)), np.zeros(n))
            for k, n in zip(sizes[:-1], sizes[1:])]


def forward(params, x):
    """x [B, 8] standardised features -> (p [B, 3], cache)."""
    h = np.asarray(x, dtype=np.float64)
    zs, hs = [], [h]
    for W, b in params[:-1]:
        z = h @ W + b
        h = gelu(z)
        zs.append(z)
        hs.append(h)
    W, b = params[-1]
    logits = h @ W + b
    return softmax(logits), (zs, hs, logits)


def loss(p, y):
    """Mean over the batch of -sum_c y_c log p_c."""
    return float(-(np.asarray(y) * np.log(np.maximum(p, 1e-300))).sum(axis=1).mean())


def backward(params, cache, p, y):
    """Gradients (dW, db) of loss() for every layer, same structure as params."""
    zs, hs, _ = cache
    B = p.shape[0]
    d = (p - np.asarray(y)) / B            # d loss / d logits
    grads = [None] * len(params)
    W, _ = params[-1]
    grads[-1] = (hs[-1].T @ d, d.sum(axis=0))
    dh = d @ W.T
    for i in range(len(params) - 2, -1, -1):
        dz = dh * gelu_grad(zs[i])
        grads[i] = (hs[i].T @ dz, dz.sum(axis=0))
        if i > 0:
            dh = dz @ params[i][0].T
    return grads


class Adam:
    """Adam (Kingma & Ba) with bias correction."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps, self.t = lr, b1, b2, eps, 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        out = []
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (w, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * g
                v = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                mh = m / (1 - self.b1**self.t)
                vh = v / (1 - self.b2**self.t)
                new.append(w - lr * mh / (np.sqrt(vh) + self.eps))
                if j == 0:
                    self.m[i] = (m, self.m[i][1]); self.v[i] = (v, self.v[i][1])
                else:
                    self.m[i] = (self.m[i][0], m); self.v[i] = (self.v[i][0], v)
            out.append(tuple(new))
        return out


def to_bf16(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
