"""Kalman-MPC: the single-pass matrix-variate ensemble Kalman smoother (FP64).

Follows Algorithm 1 with the prediction of Eq. (15) and the update of
Eqs. (12)-(14) of the paper, on the virtual system of Eqs. (4)-(5):

    Xbar_t = [X_t; U_t; dU_t]            (r = n + 2l rows, m columns)
    Xbar_{t+1} = f_CNN(Xbar_t) + Wbar_t,  Wbar_t = [0; W_t; W_t]
    Ybar_t = H Xbar_t + Vbar_t,           H = [I 0 0; 0 I 0],  Ybar_t = [X^ref_t; U^ref]

The augmented trajectory of member i at horizon step t is the row-wise
concatenation of its slices k..t; every analysis updates all of them with the
same innovation, which is what makes one forward pass a smoother (Eq. (7)).

Readings where the paper is silent or garbled (each is listed in the design
notes): the sums of (13a) and (15a) carry 1/N like (11) and (14a); R is the
row covariance of V_X, Q_U of V_U and Q_dU of W, with identity column
covariance Psi = I_m so lambda = 1/m; the initial ensemble has X_k exact and
U_k = U_prev + W_0, dU_k = W_0; updates happen at t = k+1..k+H only; no bias
unless given; the optional covariances (lines 8 and 11) are returned on request.

This implementation keeps every row of the augmented state, forms anomalies
explicitly and inverts Sigma^Ybar through a Cholesky factorisation.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .cnn import cnn_forward


@dataclasses.dataclass
class SolveResult:
    U_mean: np.ndarray  # (H+1, l, m): smoothed control means U_hat_{k..k+H}
    X_mean: np.ndarray  # (H+1, n, m)
    dU_mean: np.ndarray  # (H+1, l, m)
    members: np.ndarray  # (N, H+1, r, m): final smoothed ensemble (slices k..k+H)
    gains: List[np.ndarray]  # gain K_t (j r x p) per horizon step
    syy: List[np.ndarray]  # Sigma^Ybar_{t|t-1} per horizon step (with lambda/N)
    post_cov: List[np.ndarray]  # Sigma^X_{t|t} (Eq. 14c) per step, if requested
    prior_cov: List[np.ndarray]  # Sigma^X_{t|t-1} (Eq. 15f, line 8) per step, if requested


@dataclasses.dataclass
class Constraint:
    """A constraint g(Xbar_t, Ubar_t) <= 0 observed through a barrier (section on
    extensions after Table 1): z_t = phi(g) + eps_t with the softplus barrier
    phi(x) = ln(1 + exp(beta x)) / alpha and eps_t ~ N(0, rz), appended to Ybar_t as one
    more row whose actual value is 0.  Reading: g is applied column by column, as the
    linear form g_c = aX . X[:, c] + aU . U[:, c] - b on the forecast (noise-free) state
    and control, so the extra row has the m columns of every other row; a scalar g of
    the whole matrix corresponds to repeating one value over the columns."""

    aX: np.ndarray  # (n,)
    aU: np.ndarray  # (l,)
    b: float
    alpha: float
    beta: float
    rz: float

    def g(self, X, U):
        """Per-column constraint values of (.., n, m) states and (.., l, m) controls."""
        return (np.einsum("r,...rm->...m", np.asarray(self.aX, np.float64), X)
                + np.einsum("a,...am->...m", np.asarray(self.aU, np.float64), U) - self.b)

    def barrier(self, x):
        """Softplus barrier ln(1 + e^{beta x}) / alpha, evaluated without overflow."""
        return np.logaddexp(0.0, self.beta * np.asarray(x, np.float64)) / self.alpha


def _chol_lower(a: np.ndarray) -> np.ndarray:
    return np.linalg.cholesky(np.asarray(a, dtype=np.float64))


def analysis(Xcal, Y, Ybar_t):
    """One ensemble analysis (Eqs. (11), (13a-c), (14b)).

    Xcal: (N, a, m) forecast trajectories (all stored slices, row-concatenated);
    Y: (N, p, m) perturbed virtual observations; Ybar_t: (p, m) actual virtual
    observation.  Returns the updated trajectories, the gain K (a x p) and
    Sigma^Ybar (p x p).  lambda = 1/tr(Psi) with Psi = I_m; it cancels in K.
    """
    N, _, m = Xcal.shape
    lam = 1.0 / m
    Xcal_mean = Xcal.mean(axis=0)      # Eq. (11)
    Ymean = Y.mean(axis=0)             # Eq. (13a), with 1/N
    A = Xcal - Xcal_mean
    D = Y - Ymean
    # Eqs. (13b), (13c): sum over members i and columns of A^i D^iT (a library contraction)
    Syy = (lam / N) * np.tensordot(D, D, axes=([0, 2], [0, 2]))
    Sxy = (lam / N) * np.tensordot(A, D, axes=([0, 2], [0, 2]))
    # Eq. (14b): gain Sigma^{XY} (Sigma^Y)^{-1}, through the Cholesky factor of Sigma^Y.
    Ly = _chol_lower(Syy)
    K = np.linalg.solve(Ly.T, np.linalg.solve(Ly, Sxy.T)).T
    Xcal_upd = Xcal + np.matmul(K, Ybar_t[None] - Y)  # Eq. (14b), every member
    return Xcal_upd, K, Syy


def solve(B, weights, act, X0, Xref, QU, QdU, R, N, H, Z_init, Z_W, Z_VX, Z_VU,
          U_prev=None, Uref=None, biases=None, want_cov=False, constraint=None,
          Z_VZ=None) -> SolveResult:
    """One MPC solve at time k (Algorithm 1, lines 4-13).

    Shapes: B (n,l); X0 (n,m); Xref (H+1,n,m) = X^ref_t for t=k..k+H; QU, QdU (l,l);
    R (n,n); Z_init (N,l,m); Z_W, Z_VU (H,N,l,m); Z_VX (H,N,n,m) standard normals.
    constraint: an optional Constraint, observed with the standard normals Z_VZ (H,N,1,m).
    """
    X0 = np.asarray(X0, dtype=np.float64)
    n, m = X0.shape
    l = np.asarray(B).shape[1]
    r = n + 2 * l
    p = n + l
    U_prev = np.zeros((l, m)) if U_prev is None else np.asarray(U_prev, dtype=np.float64)
    Uref = np.zeros((l, m)) if Uref is None else np.asarray(Uref, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    L_dU = _chol_lower(QdU)  # W ~ MN(0; Q_dU, I_m)
    L_U = _chol_lower(QU)    # V_U ~ MN(0; Q_U, I_m)
    L_R = _chol_lower(R)     # V_X ~ MN(0; R, I_m)

    # Line 4: initial ensemble Xbar^i_{k|k} = [X_k; U_prev + W_0^i; W_0^i].
    W0 = np.matmul(L_dU, np.asarray(Z_init, dtype=np.float64))  # (N, l, m)
    traj = np.zeros((N, H + 1, r, m))
    traj[:, 0, :n, :] = X0
    traj[:, 0, n:n + l, :] = U_prev + W0
    traj[:, 0, n + l:, :] = W0

    gains, syys, covs, priors = [], [], [], []
    for t in range(1, H + 1):  # Line 5: t = k+1..k+H
        j = t + 1  # slices k..t after the concatenation
        prev = traj[:, t - 1]
        # Line 6, Eq. (15b): Xbar^i_{t|t-1} = f_CNN(Xbar^i_{t-1|t-1}) + Wbar^i_{t-1}.
        Xn = cnn_forward(prev[:, :n], prev[:, n:n + l], B, weights, act, biases)
        W = np.matmul(L_dU, np.asarray(Z_W[t - 1], dtype=np.float64))
        traj[:, t, :n] = Xn
        traj[:, t, n:n + l] = prev[:, n:n + l] + W
        traj[:, t, n + l:] = W
        # Line 7, Eq. (15c): concatenation = the first j slices of traj.
        Xcal = traj[:, :j].reshape(N, j * r, m)
        # Line 9, Eq. (12): perturbed virtual observations Ybar^i = H Xbar^i + Vbar^i.
        VX = np.matmul(L_R, np.asarray(Z_VX[t - 1], dtype=np.float64))
        VU = np.matmul(L_U, np.asarray(Z_VU[t - 1], dtype=np.float64))
        Y = np.concatenate([traj[:, t, :n] + VX, traj[:, t, n:n + l] + VU], axis=1)  # (N, p, m)
        Ybar_t = np.concatenate([Xref[t], Uref], axis=0)  # (p, m)
        if constraint is not None:  # the barrier observation z_t, actual value 0
            g = constraint.g(traj[:, t, :n], traj[:, t, n:n + l])  # (N, m)
            z = constraint.barrier(g) + np.sqrt(constraint.rz) * np.asarray(Z_VZ[t - 1], np.float64)[:, 0]
            Y = np.concatenate([Y, z[:, None, :]], axis=1)
            Ybar_t = np.concatenate([Ybar_t, np.zeros((1, m))], axis=0)
        if want_cov:  # Line 8, Eqs. (15d)-(15f): the block matrix equals the pooled covariance
            Ap = Xcal - Xcal.mean(axis=0)
            priors.append((1.0 / (m * N)) * np.einsum("iam,ibm->ab", Ap, Ap))
        # Lines 9-10, Eqs. (13)-(14b): update every member's whole trajectory (all j slices).
        Xcal_upd, K, Syy = analysis(Xcal, Y, Ybar_t)
        traj[:, :j] = Xcal_upd.reshape(N, j, r, m)
        gains.append(K)
        syys.append(Syy)
        if want_cov:  # Line 11, Eq. (14c)
            Au = Xcal_upd - Xcal_upd.mean(axis=0)
            covs.append((1.0 / (m * N)) * np.einsum("iam,ibm->ab", Au, Au))

    # Line 13: extract the smoothed means of every slice.
    mean = traj.mean(axis=0)  # (H+1, r, m), Eq. (14a)
    return SolveResult(U_mean=mean[:, n:n + l].copy(), X_mean=mean[:, :n].copy(),
                       dU_mean=mean[:, n + l:].copy(), members=traj, gains=gains,
                       syy=syys, post_cov=covs, prior_cov=priors)


def forecast_cov(members_t: np.ndarray) -> np.ndarray:
    """Eq. (15d): Sigma^Xbar = (lambda/N) sum_i (Xbar^i - mean)(Xbar^i - mean)^T, lambda = 1/m."""
    N, _, m = members_t.shape
    A = members_t - members_t.mean(axis=0)
    return (1.0 / (m * N)) * np.einsum("iam,ibm->ab", A, A)


def plant_step(X, U, B, weights, act, biases=None) -> np.ndarray:
    """Closed loop (Algorithm 1, line 14): the nominal plant is the surrogate itself,
    X_{k+1} = CNN(X_k, U_hat_k), deterministic."""
    return cnn_forward(X, U, B, weights, act, biases)


def closed_loop(B, weights, act, X0, ref_fn, QU, QdU, R, N, H, steps, noise_fn,
                U_prev=None):
    """Receding-horizon loop of Algorithm 1 (lines 3-15).

    ref_fn(k) -> (H+1, n, m) reference window; noise_fn(k) -> (Z_init, Z_W, Z_VX, Z_VU).
    Returns the realised states X_0..X_steps and applied controls U_0..U_{steps-1}.
    """
    n, m = np.asarray(X0).shape
    l = np.asarray(B).shape[1]
    X = np.asarray(X0, dtype=np.float64)
    Up = np.zeros((l, m)) if U_prev is None else np.asarray(U_prev, dtype=np.float64)
    Xs, Us = [X], []
    for k in range(steps):
        z = noise_fn(k)
        res = solve(B, weights, act, X, ref_fn(k), QU, QdU, R, N, H, *z, U_prev=Up)
        Uk = res.U_mean[0]
        X = plant_step(X, Uk, B, weights, act)
        Up = Uk
        Xs.append(X)
        Us.append(Uk)
    return np.stack(Xs), np.stack(Us)
