"""Matrix-trace tracking cost of the MPC problem (section "Problem Setup").

Per time t the stage cost is
    tr[(X_t - X^ref)^T R^{-1} (X_t - X^ref) + (U_t - U^ref)^T Q_U^{-1} (U_t - U^ref)
       + dU_t^T Q_dU^{-1} dU_t],
and the paper shows it equals the vectorised form with (I kron R)^{-1} etc.
``stage_cost_trace`` is the trace form; ``stage_cost_vec`` builds the Kronecker
matrices explicitly (column-stacking vec) and is used to pin the former.
"""
from __future__ import annotations

import numpy as np


def stage_cost_trace(X, Xref, U, Uref, dU, R, QU, QdU) -> float:
    ex = np.asarray(X, np.float64) - np.asarray(Xref, np.float64)
    eu = np.asarray(U, np.float64) - np.asarray(Uref, np.float64)
    du = np.asarray(dU, np.float64)
    Ri = np.linalg.inv(np.asarray(R, np.float64))
    Qi = np.linalg.inv(np.asarray(QU, np.float64))
    Qdi = np.linalg.inv(np.asarray(QdU, np.float64))
    return float(np.trace(ex.T @ Ri @ ex) + np.trace(eu.T @ Qi @ eu) + np.trace(du.T @ Qdi @ du))


def _vec(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, np.float64).reshape(-1, order="F")  # column stacking


def stage_cost_vec(X, Xref, U, Uref, dU, R, QU, QdU) -> float:
    m = np.asarray(X).shape[1]
    I = np.eye(m)
    ex = _vec(np.asarray(X, np.float64) - Xref)
    eu = _vec(np.asarray(U, np.float64) - Uref)
    du = _vec(dU)
    return float(ex @ np.linalg.inv(np.kron(I, R)) @ ex + eu @ np.linalg.inv(np.kron(I, QU)) @ eu
                 + du @ np.linalg.inv(np.kron(I, QdU)) @ du)


def closed_loop_cost(Xs, Us, U_prev0, Xrefs, R, Q) -> float:
    """Cost of a realised closed loop: sum over applied steps k of the stage cost with
    X_k against its reference, U_k against U^ref = 0 and dU_k = U_k - U_{k-1}
    (U_{-1} = U_prev0).  Xs: (K+1, n, m) with Xs[0] the initial state; Us: (K, l, m);
    Xrefs: (K+1, n, m).  The states X_1..X_K reached under the applied controls are scored."""
    Xs = np.asarray(Xs, np.float64)
    Us = np.asarray(Us, np.float64)
    total = 0.0
    Uprev = np.asarray(U_prev0, np.float64)
    for k in range(Us.shape[0]):
        dU = Us[k] - Uprev
        total += stage_cost_trace(Xs[k + 1], Xrefs[k + 1], Us[k], np.zeros_like(Us[k]), dU, R, Q, Q)
        Uprev = Us[k]
    return total


def mse(X, Xref) -> float:
    """The tracking error printed in the experiments: ||X - X^ref||_F^2 / (number of cells)."""
    e = np.asarray(X, np.float64) - np.asarray(Xref, np.float64)
    return float(np.sum(e * e) / e.size)
