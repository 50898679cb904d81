"""The matrix-trace cost equals its vectorised Kronecker form (problem setup)."""
import numpy as np

from oracle import cost
from paper_2410_09663_amd import workloads as wl


def test_trace_form_equals_vec_form():
    rng = np.random.default_rng(2)
    n, m, l = 5, 4, 3
    X, Xr = rng.standard_normal((2, n, m))
    U, Ur, dU = rng.standard_normal((3, l, m))
    R = wl.random_spd(n, 1).astype(np.float64)
    QU = wl.random_spd(l, 2).astype(np.float64)
    QdU = wl.random_spd(l, 3).astype(np.float64)
    a = cost.stage_cost_trace(X, Xr, U, Ur, dU, R, QU, QdU)
    b = cost.stage_cost_vec(X, Xr, U, Ur, dU, R, QU, QdU)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_closed_loop_cost_isotropic():
    rng = np.random.default_rng(3)
    n, m, l, K = 4, 3, 2, 3
    Xs = rng.standard_normal((K + 1, n, m))
    Xr = rng.standard_normal((K + 1, n, m))
    Us = rng.standard_normal((K, l, m))
    U0 = rng.standard_normal((l, m))
    r, q = 0.01, 0.1
    got = cost.closed_loop_cost(Xs, Us, U0, Xr, r * np.eye(n), q * np.eye(l))
    dU = np.diff(np.concatenate([U0[None], Us]), axis=0)
    ref = np.sum((Xs[1:] - Xr[1:]) ** 2) / r + np.sum(Us ** 2) / q + np.sum(dU ** 2) / q
    assert abs(got - ref) <= 1e-12 * ref
    assert abs(cost.mse(Xs[0], Xr[0]) - np.mean((Xs[0] - Xr[0]) ** 2)) < 1e-15
