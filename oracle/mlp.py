"""Oracle: forward and backward of the learned preconditioner's network.

The paper has no learned component; this is the plain FP64 reference of the
small network the Davidson preconditioner uses (three dense layers, ReLU
between them, mean-squared-error loss, Adam).  Parity unpinned against the
paper (it has no such network); pinned by central finite differences.

Layout: X [N, F_in] rows are samples; W1 [F_in, H], b1 [H], W2 [H, H], b2 [H],
W3 [H, K], b3 [K];  Y = relu(relu(X W1 + b1) W2 + b2) W3 + b3.
Loss = mean over rows and outputs of (Y - T)^2.
"""
from __future__ import annotations

import numpy as np


def init_params(f_in: int, hidden: int, k_out: int, seed: int):
    """He-style initialisation (seeded), last layer scaled down."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.standard_normal((f_in, hidden)) * np.sqrt(2.0 / f_in),
        "b1": np.zeros(hidden),
        "W2": rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden),
        "b2": np.zeros(hidden),
        "W3": rng.standard_normal((hidden, k_out)) * np.sqrt(2.0 / hidden) * 0.1,
        "b3": np.zeros(k_out),
    }
    return p


def forward(p, X):
    Z1 = X @ p["W1"] + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ p["W3"] + p["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(p, cache, Y, T):
    """Gradients of the mean-squared error with respect to every parameter."""
    X, Z1, H1, Z2, H2 = cache
    dY = 2.0 * (Y - T) / Y.size
    g = {"W3": H2.T @ dY, "b3": dY.sum(0)}
    dH2 = dY @ p["W3"].T
    dZ2 = dH2 * (Z2 > 0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dH1 = dZ2 @ p["W2"].T
    dZ1 = dH1 * (Z1 > 0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(0)
    return g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
