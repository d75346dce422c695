"""Float64 oracle of the kernel-variant selector network.

TEST INFRASTRUCTURE ONLY (see the package docstring). The paper has no
learned component; this is the plain definition of a 16 -> 64 -> 64 -> 7
multilayer perceptron with ReLU activations, squared-error loss over the
targets that are present (a NaN target marks a variant without a time and
adds nothing), and the Adam update (Kingma and Ba, 2015, Algorithm 1),
written with numpy matrix products as the only library step.

Flat parameter layout (float, 5703 entries), shared with the GPU kernels as a
*format* only: W1[64,16] b1[64] W2[64,64] b2[64] W3[7,64] b3[7], each weight
matrix row-major as [out, in].
"""
from __future__ import annotations

import numpy as np

N_IN, N_H1, N_H2, N_OUT = 16, 64, 64, 7
SHAPES = [(N_H1, N_IN), (N_H1,), (N_H2, N_H1), (N_H2,), (N_OUT, N_H2), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 5703


def unpack(theta: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta: np.ndarray, X: np.ndarray):
    """X (batch, 16) -> (Y (batch, 7), cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.where(z1 > 0.0, z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.where(z2 > 0.0, z2, 0.0)
    Y = h2 @ W3.T + b3
    return Y, (X, z1, h1, z2, h2)


def loss(Y: np.ndarray, T: np.ndarray) -> float:
    """Sum of (Y - T)^2 over the targets that are not NaN, divided by the
    number of all entries (batch x outputs)."""
    T = np.asarray(T, dtype=np.float64)
    d = np.where(np.isnan(T), 0.0, np.asarray(Y, dtype=np.float64) - T)
    return float(np.sum(d * d) / d.size)


def backward(theta: np.ndarray, cache, Y: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Gradient of :func:`loss` w.r.t. the flat parameters (ReLU'(0) = 0)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X, z1, h1, z2, h2 = cache
    nb = Y.shape[0]
    T = np.asarray(T, np.float64)
    dY = np.where(np.isnan(T), 0.0, 2.0 * (np.asarray(Y, np.float64) - T) / (nb * N_OUT))
    dW3 = dY.T @ h2
    db3 = dY.sum(axis=0)
    dz2 = (dY @ W3) * (z2 > 0.0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0.0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def loss_and_grad(theta, X, T):
    Y, cache = forward(theta, X)
    return loss(Y, T), backward(theta, cache, Y, T)


def adam_step(theta, g, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def grad_fd(theta, X, T, h=1e-6, idx=None) -> np.ndarray:
    """Central finite differences of the loss (slow; for pinning only)."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(theta.size) if idx is None else idx
    g = np.zeros(theta.size)
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        g[i] = (loss(forward(tp, X)[0], T) - loss(forward(tm, X)[0], T)) / (2.0 * h)
    return g


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)
