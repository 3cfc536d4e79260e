"""The chooser network 16-64-64-3 -- oracle (fp64, plain loops over layers).

Test infrastructure only (see the package docstring).  No counterpart in the
paper (parity unpinned by the paper); the tests pin the gradient by central
finite differences and Adam by its closed-form first step.

Network: ``h1 = tanh(xn W1 + b1)``, ``h2 = tanh(h1 W2 + b2)``, ``y = h2 W3 + b3``
with ``xn = (x - shift) * scale`` feature-wise.  Loss: mean squared error over
batch and outputs, ``L = sum (y - t)^2 / (B * 3)``.  Adam (Kingma & Ba) with
bias correction: ``m = b1 m + (1-b1) g``, ``v = b2 v + (1-b2) g^2``,
``w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)``.

Flat parameter layout (row-major, [in][out]):
W1 16x64 | b1 64 | W2 64x64 | b2 64 | W3 64x3 | b3 3   -> 5443 values.
"""

from __future__ import annotations

import numpy as np

SIZES = (16, 64, 64, 3)
NPARAM = 16 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out = []
    o = 0
    for i in range(3):
        fi, fo = SIZES[i], SIZES[i + 1]
        W = p[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        bb = p[o:o + fo]
        o += fo
        out.append((W, bb))
    assert o == NPARAM
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def init_params(seed: int) -> np.ndarray:
    """Deterministic Glorot-uniform initialisation (input generator for tests)."""
    rng = np.random.default_rng(seed)
    layers = []
    for i in range(3):
        fi, fo = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / (fi + fo))
        layers.append((rng.uniform(-lim, lim, (fi, fo)), np.zeros(fo)))
    return pack(layers)


def forward(p, X, shift=None, scale=None):
    X = np.asarray(X, dtype=np.float64)
    if shift is not None:
        X = (X - shift) * scale
    (W1, b1), (W2, b2), (W3, b3) = unpack(p)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3


def loss_and_grad(p, X, T, shift=None, scale=None):
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    if shift is not None:
        X = (X - shift) * scale
    (W1, b1), (W2, b2), (W3, b3) = unpack(p)
    B = X.shape[0]
    a1 = X @ W1 + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2 + b2
    h2 = np.tanh(a2)
    y = h2 @ W3 + b3
    diff = y - T
    loss = float(np.sum(diff * diff) / (B * 3))
    dy = 2.0 * diff / (B * 3)
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    da2 = dh2 * (1.0 - h2 * h2)
    gW2 = h1.T @ da2
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2.T
    da1 = dh1 * (1.0 - h1 * h1)
    gW1 = X.T @ da1
    gb1 = da1.sum(axis=0)
    return loss, pack([(gW1, gb1), (gW2, gb2), (gW3, gb3)])


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (``step`` counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
