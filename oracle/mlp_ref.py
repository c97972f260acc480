"""FP64 reference of the recipe/tile picker's network -- TEST INFRASTRUCTURE ONLY.

The picker is not in the paper (which picks its slicing by the class rules of
Sec. 3.2); this module is the plain definition the GPU training kernels are
checked against:

  * network: x -> h1 = relu(x W0 + b0) -> h2 = relu(h1 W1 + b1) -> y = h2 W2 + b2,
    weights row-major W[i][o], parameters flattened as W0, b0, W1, b1, W2, b2;
  * loss: masked mean squared error  sum(M (y - t)^2) / sum(M);
  * gradient: the chain rule written out layer by layer;
  * Adam (Kingma and Ba, 2015) with bias-corrected first and second moments.

Everything is numpy float64.  Pinned in tests by central finite differences,
closed forms (a network that reduces to a known linear map, the sign-like
first Adam step and constant-gradient trajectories) and hand-checked values.
"""
import numpy as np


def num_params(n_in, hidden, n_out):
    return n_in * hidden + hidden + hidden * hidden + hidden + hidden * n_out + n_out


def unpack(params, n_in, hidden, n_out):
    """The six parameter arrays (views into `params`)."""
    p = np.asarray(params, dtype=np.float64)
    if p.size != num_params(n_in, hidden, n_out):
        raise ValueError("parameter count does not match the dimensions")
    shapes = [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, n_out), (n_out,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def forward(params, X, n_in, hidden, n_out):
    """(y, cache) for a batch X of shape (B, n_in)."""
    W0, b0, W1, b1, W2, b2 = unpack(params, n_in, hidden, n_out)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W0 + b0
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W1 + b1
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W2 + b2
    return y, (X, z1, h1, z2, h2)


def masked_mse(Y, T, M):
    M = np.asarray(M, dtype=np.float64)
    cnt = M.sum()
    if cnt <= 0:
        return 0.0
    d = np.asarray(Y, dtype=np.float64) - np.asarray(T, dtype=np.float64)
    return float((M * d * d).sum() / cnt)


def loss_and_grad(params, X, T, M, n_in, hidden, n_out):
    """(loss, flat gradient in the parameter layout)."""
    W0, b0, W1, b1, W2, b2 = unpack(params, n_in, hidden, n_out)
    y, (X, z1, h1, z2, h2) = forward(params, X, n_in, hidden, n_out)
    M = np.asarray(M, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    cnt = M.sum()
    loss = masked_mse(y, T, M)
    dy = 2.0 * M * (y - T) / (cnt if cnt > 0 else 1.0)
    gW2 = h2.T @ dy
    gb2 = dy.sum(axis=0)
    dz2 = (dy @ W2.T) * (z2 > 0)
    gW1 = h1.T @ dz2
    gb1 = dz2.sum(axis=0)
    dz1 = (dz2 @ W1.T) * (z1 > 0)
    gW0 = X.T @ dz1
    gb0 = dz1.sum(axis=0)
    g = np.concatenate([gW0.ravel(), gb0, gW1.ravel(), gb1, gW2.ravel(), gb2])
    return loss, g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns new (params, m, v).  `step` counts from 1."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = np.asarray(params, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v


def init_params(rng, n_in, hidden, n_out):
    """He-style random initialisation (biases zero), float64."""
    parts = []
    for fan_in, fan_out in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        parts.append(rng.standard_normal(fan_in * fan_out) * np.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
