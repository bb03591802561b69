"""Plain FP64 reference of the surrogate network (numpy).

TEST INFRASTRUCTURE ONLY (imported by tests/): forward pass, mean-squared
error and its gradient by backpropagation, for the network the library
trains: 5 -> 128 -> 128 -> 128 -> 16, tanh on hidden layers, linear output,
parameters as one flat vector (per layer W [in][out] then b [out]).
The backpropagation is pinned by central finite differences in
tests/test_oracle_mlp.py.
"""
from __future__ import annotations

import numpy as np

SIZES = [(5, 128), (128, 128), (128, 128), (128, 16)]
N_PARAMS = sum(i * o + o for i, o in SIZES)


def unpack(p: np.ndarray):
    """Flat parameters -> [(W, b)] (views)."""
    out, k = [], 0
    for i, o in SIZES:
        W = p[k:k + i * o].reshape(i, o)
        k += i * o
        b = p[k:k + o]
        k += o
        out.append((W, b))
    return out


def forward(p: np.ndarray, X: np.ndarray):
    """Returns the output [n,16] and the hidden activations."""
    h = np.asarray(X, dtype=np.float64)
    hs = [h]
    layers = unpack(np.asarray(p, dtype=np.float64))
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        h = np.tanh(z) if li < len(layers) - 1 else z
        hs.append(h)
    return h, hs


def loss(p, X, T) -> float:
    Y, _ = forward(p, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_grad(p, X, T):
    """Mean squared error over all outputs and its gradient (flat)."""
    p = np.asarray(p, dtype=np.float64)
    Y, hs = forward(p, X)
    T = np.asarray(T, dtype=np.float64)
    n, m = Y.shape
    d = 2.0 * (Y - T) / (n * m)
    grads = []
    layers = unpack(p)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        x_in = hs[li]
        grads.append((x_in.T @ d, d.sum(axis=0)))
        if li > 0:
            d = (d @ W.T) * (1.0 - hs[li] ** 2)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return float(np.mean((Y - T) ** 2)), flat


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1), FP64: moment
    estimates m, v of the gradient g are updated in place, bias-corrected by
    1 - b1^t and 1 - b2^t (t >= 1 the step number), and the parameters are
    returned as p - lr * m_hat / (sqrt(v_hat) + eps)."""
    g = np.asarray(g, dtype=np.float64)
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return np.asarray(p, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
