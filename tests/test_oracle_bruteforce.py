"""Pins the oracle's matrix-variate statistics, gain and update against dense vectorised
brute force on 4x4 grids: every member is vectorised (column stacking), the full
cross-covariance of the vectors is formed, its m diagonal column blocks are pooled
(the matrix-normal estimate with Psi = I), and the update is applied as the dense
matrix I_m kron K.  The CNN is applied as dense per-layer Toeplitz matrices."""
import itertools

import numpy as np
import pytest

from oracle import cnn, enks


def vec(a):
    return a.reshape(a.shape[:-2] + (-1,), order="F") if a.ndim == 2 else \
        np.stack([x.reshape(-1, order="F") for x in a])


def unvec(v, rows, cols):
    return v.reshape(cols, rows).T


def brute_analysis(Xcal, Y, Ybar):
    N, a, m = Xcal.shape
    p = Y.shape[1]
    xv = np.stack([Xcal[i].reshape(-1, order="F") for i in range(N)])  # (N, a m)
    yv = np.stack([Y[i].reshape(-1, order="F") for i in range(N)])      # (N, p m)
    xa = xv - xv.mean(axis=0)
    ya = yv - yv.mean(axis=0)
    Cxy = sum(np.outer(xa[i], ya[i]) for i in range(N))  # (a m, p m)
    Cyy = sum(np.outer(ya[i], ya[i]) for i in range(N))
    Sxy = sum(Cxy[c * a:(c + 1) * a, c * p:(c + 1) * p] for c in range(m))
    Syy = sum(Cyy[c * p:(c + 1) * p, c * p:(c + 1) * p] for c in range(m))
    K = Sxy @ np.linalg.inv(Syy)
    big = np.kron(np.eye(m), K)  # (a m, p m)
    out = np.empty_like(Xcal)
    yb = Ybar.reshape(-1, order="F")
    for i in range(N):
        out[i] = unvec(xv[i] + big @ (yb - yv[i]), a, m)
    return out, K


def toeplitz(w, n, m):
    cout, cin = w.shape[:2]
    T = np.zeros((cout * n * m, cin * n * m))
    for o, y, x in itertools.product(range(cout), range(n), range(m)):
        for c, a, b in itertools.product(range(cin), range(3), range(3)):
            yy, xx = y + a - 1, x + b - 1
            if 0 <= yy < n and 0 <= xx < m:
                T[(o * n + y) * m + x, (c * n + yy) * m + xx] += w[o, c, a, b]
    return T


def brute_cnn(X, U, B, ws, act):
    n, m = X.shape
    h = np.concatenate([X.reshape(-1), (B @ U).reshape(-1)])
    for i, w in enumerate(ws):
        h = toeplitz(w, n, m) @ h
        if i < len(ws) - 1:
            h = cnn.activation(h, act)
    return h.reshape(n, m)


def test_analysis_matches_vectorised_bruteforce():
    rng = np.random.default_rng(3)
    N, a, p, m = 9, 14, 6, 4
    Xcal = rng.standard_normal((N, a, m))
    Y = rng.standard_normal((N, p, m)) + 0.3 * Xcal[:, :p]
    Ybar = rng.standard_normal((p, m))
    got, K, Syy = enks.analysis(Xcal, Y, Ybar)
    ref, Kref = brute_analysis(Xcal, Y, Ybar)
    assert np.max(np.abs(K - Kref)) <= 1e-12 * np.abs(Kref).max()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("act", [cnn.ACT_TANH, cnn.ACT_GELU])
def test_full_solve_matches_bruteforce_4x4(act):
    rng = np.random.default_rng(4)
    n = m = 4
    l, N, H = 2, 12, 3
    B = 0.5 * rng.standard_normal((n, l))
    ws = [rng.standard_normal((3, 2, 3, 3)) * 0.4, rng.standard_normal((1, 3, 3, 3)) * 0.4]
    X0 = rng.standard_normal((n, m))
    Xref = rng.standard_normal((H + 1, n, m))
    QdU = np.array([[0.1, 0.02], [0.02, 0.08]])
    QU = np.array([[0.2, 0.0], [0.0, 0.15]])
    R = 0.02 * np.eye(n) + 0.005
    Up = 0.1 * rng.standard_normal((l, m))
    z0 = rng.standard_normal((N, l, m))
    zw = rng.standard_normal((H, N, l, m))
    zx = rng.standard_normal((H, N, n, m))
    zu = rng.standard_normal((H, N, l, m))
    res = enks.solve(B, ws, act, X0, Xref, QU, QdU, R, N, H, z0, zw, zx, zu, U_prev=Up)

    # brute force: member-by-member dense algebra
    Ld, Lu, Lr = (np.linalg.cholesky(M) for M in (QdU, QU, R))
    r = n + 2 * l
    traj = [[np.concatenate([X0, Up + Ld @ z0[i], Ld @ z0[i]])] for i in range(N)]
    for t in range(1, H + 1):
        Ys = []
        for i in range(N):
            s = traj[i][-1]
            w = Ld @ zw[t - 1, i]
            xn = brute_cnn(s[:n], s[n:n + l], B, ws, act)
            new = np.concatenate([xn, s[n:n + l] + w, w])
            traj[i].append(new)
            Ys.append(np.concatenate([xn + Lr @ zx[t - 1, i], new[n:n + l] + Lu @ zu[t - 1, i]]))
        Xcal = np.stack([np.concatenate(traj[i]) for i in range(N)])
        upd, _ = brute_analysis(Xcal, np.stack(Ys), np.concatenate([Xref[t], np.zeros((l, m))]))
        for i in range(N):
            traj[i] = [upd[i][s * r:(s + 1) * r] for s in range(t + 1)]
    mean = np.mean([np.stack(traj[i]) for i in range(N)], axis=0)
    assert np.max(np.abs(res.U_mean - mean[:, n:n + l])) <= 1e-12
    assert np.max(np.abs(res.X_mean - mean[:, :n])) <= 1e-12
    assert np.max(np.abs(res.dU_mean - mean[:, n + l:])) <= 1e-12
