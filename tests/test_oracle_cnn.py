"""Pins for the oracle's CNN (Eq. (1)): a library routine and brute force."""
import itertools

import numpy as np
import pytest
import torch

from oracle import cnn


def _dense_conv_matrix(w, n, m):
    """Brute force: the (C_out n m) x (C_in n m) matrix of a zero-padded 3x3 cross-correlation."""
    cout, cin = w.shape[:2]
    T = np.zeros((cout * n * m, cin * n * m))
    for o, y, x in itertools.product(range(cout), range(n), range(m)):
        for c, a, b in itertools.product(range(cin), range(3), range(3)):
            yy, xx = y + a - 1, x + b - 1
            if 0 <= yy < n and 0 <= xx < m:
                T[(o * n + y) * m + x, (c * n + yy) * m + xx] += w[o, c, a, b]
    return T


@pytest.mark.parametrize("n,m,cin,cout", [(4, 4, 2, 3), (5, 7, 2, 1), (3, 6, 4, 2)])
def test_conv_matches_dense_matrix(n, m, cin, cout):
    rng = np.random.default_rng(n * 100 + m)
    x = rng.standard_normal((cin, n, m))
    w = rng.standard_normal((cout, cin, 3, 3))
    T = _dense_conv_matrix(w, n, m)
    ref = (T @ x.reshape(-1)).reshape(cout, n, m)
    assert np.max(np.abs(cnn.conv3x3(x, w) - ref)) <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,m", [(4, 4), (5, 7), (16, 16)])
def test_conv_matches_torch_conv2d(n, m):
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 2, n, m))
    w = rng.standard_normal((5, 2, 3, 3))
    b = rng.standard_normal(5)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w),
                                     torch.from_numpy(b), padding=1).numpy()
    assert np.max(np.abs(cnn.conv3x3(x, w, b) - ref)) <= 1e-13


@pytest.mark.parametrize("act", [cnn.ACT_TANH, cnn.ACT_GELU])
def test_cnn_forward_matches_torch_stack(act):
    rng = np.random.default_rng(11)
    n, m, l = 6, 5, 2
    B = rng.standard_normal((n, l))
    chans = [2, 4, 3, 1]
    ws = [rng.standard_normal((co, ci, 3, 3)) * 0.5 for ci, co in zip(chans[:-1], chans[1:])]
    X = rng.standard_normal((3, n, m))
    U = rng.standard_normal((3, l, m))
    h = torch.from_numpy(np.stack([X, B @ U], axis=1))
    for i, w in enumerate(ws):
        h = torch.nn.functional.conv2d(h, torch.from_numpy(w), padding=1)
        if i < len(ws) - 1:
            h = torch.tanh(h) if act == cnn.ACT_TANH else torch.nn.functional.gelu(h, approximate="none")
    ref = h[:, 0].numpy()
    got = cnn.cnn_forward(X, U, B, ws, act)
    assert got.shape == (3, n, m)
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_gelu_exact_form():
    x = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    assert np.max(np.abs(cnn.activation(x, cnn.ACT_GELU) - ref)) <= 1e-14
