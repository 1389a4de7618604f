"""FP64 reference of the learned cost model: a 3-layer MLP regressor (test infrastructure).

The cost model predicts the log of an operation's duration from its features.  Network:
  z1 = x W1^T + b1, h1 = relu(z1)      (W1: hidden x f)
  z2 = h1 W2^T + b2, h2 = relu(z2)     (W2: hidden x hidden)
  y  = h2 W3^T + b3                    (W3: 1 x hidden)
Loss: mean squared error over the batch, L = mean((y - t)^2).
Gradients by back-propagation (Rumelhart, Hinton and Williams, 1986); optimiser Adam (Kingma and
Ba, 2015) with bias-corrected first and second moments.  Parameters are a dict of float64 arrays
named W1, b1, W2, b2, W3, b3; b3 has shape (1,).
"""
import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def _f64(p):
    return {k: np.asarray(v, dtype=np.float64) for k, v in p.items()}


def forward(params, x):
    p = _f64(params)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss(y, t):
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients of the MSE loss with respect to every parameter."""
    p = _f64(params)
    bsz = y.shape[0]
    dy = (2.0 / bsz) * (np.asarray(y, np.float64) - np.asarray(t, np.float64))[:, None]
    g = {}
    g["W3"] = dy.T @ cache["h2"]
    g["b3"] = dy.sum(axis=0)
    dz2 = (dy @ p["W3"]) * (cache["z2"] > 0)
    g["W2"] = dz2.T @ cache["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (cache["z1"] > 0)
    g["W1"] = dz1.T @ cache["x"]
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at 1-based ``step``; returns new (params, m, v)."""
    newp, newm, newv = {}, {}, {}
    for k in NAMES:
        gk = np.asarray(grads[k], np.float64)
        mk = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * gk
        vk = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * gk * gk
        mhat = mk / (1.0 - beta1 ** step)
        vhat = vk / (1.0 - beta2 ** step)
        newp[k] = np.asarray(params[k], np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        newm[k], newv[k] = mk, vk
    return newp, newm, newv


def zeros_like(params):
    return {k: np.zeros_like(np.asarray(params[k], np.float64)) for k in NAMES}
