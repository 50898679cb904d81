"""Right transformation of the control (section on extensions, after Table 1).

Test infrastructure, not product code.  When the actual control u_t has q < m
columns, the method runs on U_t = u_t T with a q x m matrix T of full row rank
(T T^T > 0), and the smoothed control is mapped back by the least-squares right
inverse:  u_hat = U_hat T^T (T T^T)^{-1}.  For a column vector u (q = 1) the paper's
choice T = [1 ... 1] repeats u over the m columns.
"""
from __future__ import annotations

import numpy as np


def expand(u, T) -> np.ndarray:
    """U = u T for u (..., l, q) and T (q, m)."""
    return np.asarray(u, np.float64) @ np.asarray(T, np.float64)


def project(U, T) -> np.ndarray:
    """u = U T^T (T T^T)^{-1} for U (..., l, m) and T (q, m)."""
    T = np.asarray(T, np.float64)
    G = T @ T.T
    # U T^T G^{-1} = (G^{-1} T U^T)^T, G symmetric
    rhs = np.asarray(U, np.float64) @ T.T
    return np.linalg.solve(G, np.swapaxes(rhs, -1, -2)).swapaxes(-1, -2)
