"""Multi-head attention inference written directly as formulas (test infrastructure).

Sec. V: each head h of a transformer layer computes Q = X*W^Q_h, K = X*W^K_h, V = X*W^V_h,
A = Q*K^T, B = softmax(A), C = B*V; the head outputs are concatenated and a layer's output is the
next layer's input.  Readings used here (stated in the design notes): the scores are scaled by
1/sqrt(dh) (exact for dh = 64: 1/8); head h uses columns [h*dh, (h+1)*dh) of d x d weight
matrices Wq, Wk, Wv; the join is the concatenation followed by one output projection Y = Ocat*Wo;
layers stack with no residual or normalisation.  Everything is float64.
"""
import math

import numpy as np

from . import kernels as K


def mha_layer(x, wq, wk, wv, wo, heads):
    x = np.asarray(x, dtype=np.float64)
    n, d = x.shape
    dh = d // heads
    ocat = np.empty((n, d), dtype=np.float64)
    for h in range(heads):
        cols = slice(h * dh, (h + 1) * dh)
        q = x @ np.asarray(wq, dtype=np.float64)[:, cols]
        k = x @ np.asarray(wk, dtype=np.float64)[:, cols]
        v = x @ np.asarray(wv, dtype=np.float64)[:, cols]
        a = (q @ k.T) / math.sqrt(dh)
        b = K.softmax(a)
        ocat[:, cols] = b @ v
    return ocat @ np.asarray(wo, dtype=np.float64)


def mha_stack(x, weights, heads):
    """``weights`` is a list of (Wq, Wk, Wv, Wo) per layer; returns the last layer's output."""
    y = np.asarray(x, dtype=np.float64)
    for (wq, wk, wv, wo) in weights:
        y = mha_layer(y, wq, wk, wv, wo, heads)
    return y
