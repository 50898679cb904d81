"""CNN surrogate of Eq. (1): X_{k+1} = CNN_theta(X_k, U_k), in FP64.

Conventions (the paper gives none; these are the readings taken here):
* the control enters as a second input channel B @ U, with B in R^{n x l};
* every layer is a 3x3 cross-correlation with zero padding of one cell and
  stride one, weights in [C_out][C_in][3][3] order, optional bias;
* the activation (tanh or the exact erf form of GELU) sits between layers,
  none after the last; the last layer has one output channel, the next state.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

ACT_TANH = 0
ACT_GELU = 1


def conv3x3(x: np.ndarray, w: np.ndarray, b=None) -> np.ndarray:
    """Zero-padded 3x3 cross-correlation.

    x: (..., C_in, n, m); w: (C_out, C_in, 3, 3); returns (..., C_out, n, m) with
    out[o, y, x] = sum_c sum_{a,b in 0..2} w[o, c, a, b] * in[c, y+a-1, x+b-1].
    Written as one matrix product of the (C_out, 9 C_in) weights with the
    (9 C_in, n m) matrix of shifted copies of the input (im2col), in batch chunks.
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    *lead, cin, n, m = x.shape
    cout = w.shape[0]
    assert w.shape == (cout, cin, 3, 3)
    xb = x.reshape(-1, cin, n, m)
    B = xb.shape[0]
    pad = np.zeros((B, cin, n + 2, m + 2))
    pad[:, :, 1:n + 1, 1:m + 1] = xb
    out = np.empty((B, cout, n * m))
    step = max(1, (1 << 23) // (cin * 9 * n * m))
    for s in range(0, B, step):
        e = min(B, s + step)
        cols = np.empty((e - s, cin, 9, n * m))
        for a in range(3):
            for b_ in range(3):
                # row (c, 3a+b) of the column matrix holds in[c, y+a-1, x+b-1]
                cols[:, :, 3 * a + b_, :] = pad[s:e, :, a:a + n, b_:b_ + m].reshape(e - s, cin, n * m)
        np.matmul(w.reshape(cout, cin * 9), cols.reshape(e - s, cin * 9, n * m), out=out[s:e])
    if b is not None:
        out += np.asarray(b, dtype=np.float64)[:, None]
    return out.reshape(tuple(lead) + (cout, n, m))


def activation(x: np.ndarray, kind: int) -> np.ndarray:
    if kind == ACT_TANH:
        return np.tanh(x)
    if kind == ACT_GELU:
        return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))
    raise ValueError(kind)


def cnn_forward(X: np.ndarray, U: np.ndarray, B: np.ndarray, weights, act: int, biases=None):
    """Eq. (1) for one field or a batch of fields.

    X: (..., n, m); U: (..., l, m); B: (n, l).  Returns X_next with the shape of X.
    """
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    BU = np.matmul(B, U)  # (..., n, m)
    h = np.stack([X, BU], axis=-3)  # (..., 2, n, m)
    L = len(weights)
    for ell, w in enumerate(weights):
        bias = None if biases is None else biases[ell]
        h = conv3x3(h, w, bias)
        if ell < L - 1:
            h = activation(h, act)
    assert h.shape[-3] == 1
    return h[..., 0, :, :]
