"""Closed-form references that pin the smoother in the linear-Gaussian case.

With a single linear conv layer whose 3x3 kernel is nonzero only in its centre
column, the surrogate acts column by column:
    x_{t+1}[:, c] = F x_t[:, c] + G u_t[:, c],  F = tridiag(f), G = tridiag(g) B,
and the virtual system of Eq. (4) is, per column, a linear-Gaussian state-space
model with state z = [x; u; du], process noise [0; w; w], w ~ N(0, Q_dU), and
observation [x; u] + v, v ~ N(0, diag(R, Q_U)).  All columns share the same
covariances, so the matrix-normal assumption (8) holds exactly and the pooled
gain equals the per-column Kalman gain.  Two textbook results then fix the
posterior mean of the trajectory given the observations at t = k+1..k+H:

* ``kalman_rts``: Kalman filter forward, Rauch-Tung-Striebel smoother backward
  (with a pseudo-inverse, since the predicted covariance is singular when
  l < n);
* ``dense_ls``: the minimiser of the MPC cost over U_k..U_{k+H} by dense least
  squares, which Theorem 1 equates with the MAP smoothing estimate.

The initial ensemble (X_k exact, U_k = U_prev + W_0) becomes the prior
z_k ~ N([x_k; u_prev; 0], [[0,0,0],[0,Q,Q],[0,Q,Q]]).
"""
from __future__ import annotations

import numpy as np


def tridiag(taps, n) -> np.ndarray:
    """n x n matrix of a zero-padded vertical 3-tap cross-correlation: (T x)[y] = sum_a taps[a] x[y+a-1]."""
    T = np.zeros((n, n))
    for y in range(n):
        for a in range(3):
            yy = y + a - 1
            if 0 <= yy < n:
                T[y, yy] = taps[a]
    return T


def linear_weights(f, g) -> np.ndarray:
    """Conv weights (1, 2, 3, 3) whose only nonzero column is the centre one."""
    w = np.zeros((1, 2, 3, 3))
    w[0, 0, :, 1] = f
    w[0, 1, :, 1] = g
    return w


def _system(F, G, QdU):
    n, l = G.shape
    r = n + 2 * l
    A = np.zeros((r, r))
    A[:n, :n] = F
    A[:n, n:n + l] = G
    A[n:n + l, n:n + l] = np.eye(l)
    Qz = np.zeros((r, r))
    Qz[n:, n:] = np.kron(np.ones((2, 2)), QdU)
    Hz = np.zeros((n + l, r))
    Hz[:, :n + l] = np.eye(n + l)
    return A, Qz, Hz


def kalman_rts(F, G, QU, QdU, R, x0, u_prev, xref, uref=None):
    """Per-column Kalman filter + RTS smoother.  x0 (n,m); u_prev (l,m); xref (H+1,n,m).
    Returns the smoothed means (H+1, n+2l, m) for t = k..k+H."""
    F = np.asarray(F, np.float64)
    G = np.asarray(G, np.float64)
    n, l = G.shape
    H = xref.shape[0] - 1
    m = x0.shape[1]
    r = n + 2 * l
    uref = np.zeros((l, m)) if uref is None else uref
    A, Qz, Hz = _system(F, G, np.asarray(QdU, np.float64))
    Rv = np.zeros((n + l, n + l))
    Rv[:n, :n] = R
    Rv[n:, n:] = QU
    P0 = np.zeros((r, r))
    P0[n:, n:] = np.kron(np.ones((2, 2)), QdU)
    out = np.zeros((H + 1, r, m))
    for c in range(m):
        mf = [np.concatenate([x0[:, c], u_prev[:, c], np.zeros(l)])]
        Pf = [P0]
        mp, Pp = [None], [None]
        for t in range(1, H + 1):
            m_ = A @ mf[-1]
            P_ = A @ Pf[-1] @ A.T + Qz
            S = Hz @ P_ @ Hz.T + Rv
            K = P_ @ Hz.T @ np.linalg.inv(S)
            y = np.concatenate([xref[t][:, c], uref[:, c]])
            mf.append(m_ + K @ (y - Hz @ m_))
            Pf.append(P_ - K @ S @ K.T)
            mp.append(m_)
            Pp.append(P_)
        ms = [None] * (H + 1)
        ms[H] = mf[H]
        for t in range(H - 1, -1, -1):
            C = Pf[t] @ A.T @ np.linalg.pinv(Pp[t + 1], rcond=1e-12, hermitian=True)
            ms[t] = mf[t] + C @ (ms[t + 1] - mp[t + 1])
        out[:, :, c] = np.stack(ms)
    return out


def dense_ls(F, G, QU, QdU, R, x0, u_prev, xref, uref=None):
    """Minimise, over U_k..U_{k+H} (columns independent), the cost
        sum_{t=k+1}^{k+H} [(x_t - xref_t)^T R^-1 (.) + (u_t - uref)^T Q_U^-1 (.)]
        + sum_{t=k}^{k+H} du_t^T Q_dU^-1 du_t,   du_t = u_t - u_{t-1}, u_{k-1} = u_prev,
    subject to x_{t+1} = F x_t + G u_t, by stacking weighted residuals and solving
    one dense least-squares problem per column.  Returns (H+1, n+2l, m)."""
    F = np.asarray(F, np.float64)
    G = np.asarray(G, np.float64)
    n, l = G.shape
    H = xref.shape[0] - 1
    m = x0.shape[1]
    uref = np.zeros((l, m)) if uref is None else uref
    Wr = np.linalg.cholesky(np.linalg.inv(R)).T      # Wr^T Wr = R^-1
    Wu = np.linalg.cholesky(np.linalg.inv(QU)).T
    Wd = np.linalg.cholesky(np.linalg.inv(QdU)).T
    nv = (H + 1) * l  # decision variables u_k..u_{k+H}
    out = np.zeros((H + 1, n + 2 * l, m))
    for c in range(m):
        # x_t = Phi_t x0 + sum_{s<t} Gam_{t,s} u_s  (affine in the decision vector)
        xs_lin = [np.zeros((n, nv))]
        xs_off = [x0[:, c].astype(np.float64)]
        for t in range(1, H + 1):
            lin = F @ xs_lin[-1]
            lin[:, (t - 1) * l:t * l] += G
            xs_lin.append(lin)
            xs_off.append(F @ xs_off[-1])
        rows, rhs = [], []
        for t in range(1, H + 1):
            rows.append(Wr @ xs_lin[t])
            rhs.append(Wr @ (xref[t][:, c] - xs_off[t]))
            sel = np.zeros((l, nv))
            sel[:, t * l:(t + 1) * l] = np.eye(l)
            rows.append(Wu @ sel)
            rhs.append(Wu @ uref[:, c])
        for t in range(0, H + 1):
            d = np.zeros((l, nv))
            d[:, t * l:(t + 1) * l] = np.eye(l)
            off = np.zeros(l)
            if t == 0:
                off = -u_prev[:, c]
            else:
                d[:, (t - 1) * l:t * l] -= np.eye(l)
            rows.append(Wd @ d)
            rhs.append(-(Wd @ off))
        Amat = np.vstack(rows)
        b = np.concatenate(rhs)
        u = np.linalg.lstsq(Amat, b, rcond=None)[0].reshape(H + 1, l)
        for t in range(H + 1):
            out[t, :n, c] = xs_lin[t] @ u.reshape(-1) + xs_off[t]
            out[t, n:n + l, c] = u[t]
            out[t, n + l:, c] = u[t] - (u_prev[:, c] if t == 0 else u[t - 1])
    return out


def conv_matrix(w2d, n, m) -> np.ndarray:
    """(n m) x (n m) matrix of a zero-padded 3x3 cross-correlation on an n x m field, vec
    index y m + x: (T vec(a))[y m + x] = sum_{dy,dx} w2d[dy][dx] a[y+dy-1, x+dx-1]."""
    T = np.zeros((n * m, n * m))
    for y in range(n):
        for x in range(m):
            for dy in range(3):
                for dx in range(3):
                    yy, xx = y + dy - 1, x + dx - 1
                    if 0 <= yy < n and 0 <= xx < m:
                        T[y * m + x, yy * m + xx] += w2d[dy][dx]
    return T


def pooled_recursion(w, B, QU, QdU, R, x0, u_prev, xref, uref=None, pooled=True):
    """The ensemble smoother's limit N -> infinity for one linear conv layer with a full
    3x3 kernel w (1, 2, 3, 3), which mixes columns so that the matrix-normal assumption
    no longer holds exactly.  Everything stays linear and Gaussian, so the stored
    trajectory (every slice [x; u; du], vectorised, index (slice, row, column)) has an
    exact Gaussian mean and covariance P; what the ensemble method changes is the gain:
    pooled over the m columns (Eqs. (13b,c) with the sample sums replaced by their
    expectations),
        K = (sum_c P_{zY}[c, c]) (sum_c P_{YY}[c, c] + m diag(R, Q_U))^{-1},
    where [c, c] takes the rows of column c on both sides, applied to every column
    (I_m kron K), and the perturbed-observation covariance update for an arbitrary gain
    (Joseph form),
        P+ = (I - KH) P (I - KH)^T + K (diag(R, Q_U) kron I_m) K^T.
    Process noise [0; w; w] with w ~ MN(0, Q_dU, I_m); observations [x_t; u_t] + v with
    v ~ MN(0, diag(R, Q_U), I_m) and observed value [xref_t; uref]; prior x_k fixed,
    u_k = u_prev + w_0, du_k = w_0.  Returns the smoothed means (H+1, n+2l, m).
    pooled=False: the exact Kalman smoother of the same vectorised system instead (gain
    P H^T (H P H^T + diag(R, Q_U) kron I_m)^{-1}, no pooling), from which the pooled limit
    departs when the conv mixes columns."""
    w = np.asarray(w, np.float64)
    B = np.asarray(B, np.float64)
    n, m = x0.shape
    l = B.shape[1]
    H = xref.shape[0] - 1
    r = n + 2 * l
    p = n + l
    S = r * m  # one slice, vectorised (row, column)
    uref = np.zeros((l, m)) if uref is None else uref
    Ax = conv_matrix(w[0, 0], n, m)
    Au = conv_matrix(w[0, 1], n, m) @ np.kron(B, np.eye(m))  # (n m) x (l m): B U per column, then the conv
    Qw = np.kron(QdU, np.eye(m))
    Rv = np.zeros((p * m, p * m))
    Rv[:n * m, :n * m] = np.kron(R, np.eye(m))
    Rv[n * m:, n * m:] = np.kron(QU, np.eye(m))
    Robs = np.zeros((p, p))
    Robs[:n, :n] = R
    Robs[n:, n:] = QU
    xs, us, ds = slice(0, n * m), slice(n * m, (n + l) * m), slice((n + l) * m, S)
    mu = np.concatenate([x0.reshape(-1), u_prev.reshape(-1), np.zeros(l * m)])
    P = np.zeros((S, S))
    P[us, us] = P[us, ds] = P[ds, us] = P[ds, ds] = Qw
    for t in range(1, H + 1):
        D = mu.size
        # forecast: the new slice from the last one
        T = np.zeros((S, D))
        last = D - S
        T[xs, last + xs.start:last + xs.stop] = Ax
        T[xs, last + us.start:last + us.stop] = Au
        T[us, last + us.start:last + us.stop] = np.eye(l * m)
        Qs = np.zeros((S, S))
        Qs[us, us] = Qs[us, ds] = Qs[ds, us] = Qs[ds, ds] = Qw
        mu = np.concatenate([mu, T @ mu])
        P = np.block([[P, P @ T.T], [T @ P, T @ P @ T.T + Qs]])
        D = mu.size
        # observation of the new slice's x and u rows
        Hm = np.zeros((p * m, D))
        Hm[:, D - S:D - S + p * m] = np.eye(p * m)
        PzY = P @ Hm.T
        PYY = Hm @ P @ Hm.T
        rows = (t + 1) * r
        Szy = np.zeros((rows, p))
        Syy = m * Robs
        for c in range(m):
            zc = np.arange(rows) * m + c  # (slice, row) at column c
            yc = np.arange(p) * m + c
            Szy += PzY[np.ix_(zc, yc)]
            Syy = Syy + PYY[np.ix_(yc, yc)]
        if pooled:
            K = Szy @ np.linalg.inv(Syy)
            Kf = np.zeros((D, p * m))
            for c in range(m):
                Kf[np.ix_(np.arange(rows) * m + c, np.arange(p) * m + c)] = K
        else:
            Kf = PzY @ np.linalg.inv(PYY + Rv)
        y = np.concatenate([xref[t].reshape(-1), uref.reshape(-1)])
        mu = mu + Kf @ (y - Hm @ mu)
        IKH = np.eye(D) - Kf @ Hm
        P = IKH @ P @ IKH.T + Kf @ Rv @ Kf.T
    return mu.reshape(H + 1, r, m)
