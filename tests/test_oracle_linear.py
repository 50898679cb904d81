"""Pins the whole smoother in the linear-Gaussian case (spec check (i)).

A single linear conv layer whose kernel is nonzero only in its centre column acts
column by column, so the matrix-normal assumption holds exactly.  Then:
  * the per-column Kalman filter + RTS smoother equals the dense least-squares
    minimiser of the MPC cost (Theorem 1), to rounding;
  * the ensemble smoother's mean converges to both as N grows, at rate N^-1/2.
"""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import enks


def _case(seed=5, n=5, m=4, l=2, H=3):
    rng = np.random.default_rng(seed)
    f = np.array([0.2, 0.6, 0.15])
    g = np.array([0.3, 0.5, -0.2])
    B = rng.standard_normal((n, l)) * 0.5
    F = cf.tridiag(f, n)
    G = cf.tridiag(g, n) @ B
    QdU = np.array([[0.1, 0.03], [0.03, 0.2]])
    QU = np.array([[0.3, 0.0], [0.0, 0.25]])
    R = 0.05 * np.eye(n) + 0.01
    x0 = rng.standard_normal((n, m))
    up = rng.standard_normal((l, m)) * 0.3
    xref = rng.standard_normal((H + 1, n, m))
    return dict(f=f, g=g, B=B, F=F, G=G, QdU=QdU, QU=QU, R=R, x0=x0, up=up, xref=xref,
                n=n, m=m, l=l, H=H)


def test_tridiag_is_the_centre_column_conv():
    from oracle import cnn
    c = _case()
    w = cf.linear_weights(c["f"], c["g"])
    U = np.random.default_rng(1).standard_normal((c["l"], c["m"]))
    got = cnn.cnn_forward(c["x0"], U, c["B"], [w], cnn.ACT_TANH)
    assert np.allclose(got, c["F"] @ c["x0"] + c["G"] @ U, atol=1e-13)


def test_rts_equals_dense_least_squares():
    c = _case()
    a = cf.kalman_rts(c["F"], c["G"], c["QU"], c["QdU"], c["R"], c["x0"], c["up"], c["xref"])
    b = cf.dense_ls(c["F"], c["G"], c["QU"], c["QdU"], c["R"], c["x0"], c["up"], c["xref"])
    assert np.max(np.abs(a - b)) <= 1e-10 * np.abs(a).max()


def test_enks_mean_converges_to_rts():
    c = _case()
    n, m, l, H = c["n"], c["m"], c["l"], c["H"]
    rts = cf.kalman_rts(c["F"], c["G"], c["QU"], c["QdU"], c["R"], c["x0"], c["up"], c["xref"])
    w = [cf.linear_weights(c["f"], c["g"])]
    Ns = [32, 128, 512, 2048, 8192]
    errs = []
    for N in Ns:
        e = []
        for s in range(8):
            rng = np.random.default_rng(1000 + s)
            z = (rng.standard_normal((N, l, m)), rng.standard_normal((H, N, l, m)),
                 rng.standard_normal((H, N, n, m)), rng.standard_normal((H, N, l, m)))
            res = enks.solve(c["B"], w, 0, c["x0"], c["xref"], c["QU"], c["QdU"], c["R"], N, H,
                             *z, U_prev=c["up"])
            full = np.concatenate([res.X_mean, res.U_mean, res.dU_mean], axis=1)
            e.append(np.linalg.norm(full - rts) / np.linalg.norm(rts))
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert -0.62 <= slope <= -0.38, (slope, errs)
    assert errs[-1] < 0.02, errs
