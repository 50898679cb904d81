"""Pins the whole smoother in the linear-Gaussian case.

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


def test_closed_loop_converges_to_the_closed_form_loop():
    """Algorithm 1's receding-horizon loop (lines 3-16: solve, apply the smoothed U_k,
    step the plant, carry U_k as the next U_prev) driven by the ensemble smoother tends,
    as N grows, to the same loop driven by the closed-form Kalman filter + RTS smoother,
    at rate N^-1/2.  A loop that applied another slice, skipped the U_prev hand-over or
    stepped the plant with the wrong control would converge to something else."""
    c = _case(H=2)
    n, m, l, H = c["n"], c["m"], c["l"], c["H"]
    steps = 3
    xrefs = np.random.default_rng(7).standard_normal((steps + H + 1, n, m))
    ref_fn = lambda k: xrefs[k:k + H + 1]
    w = [cf.linear_weights(c["f"], c["g"])]
    # the loop with the closed-form smoother and the linear plant x' = F x + G u
    X, Up = c["x0"], c["up"]
    want_X, want_U = [], []
    for k in range(steps):
        sm = cf.kalman_rts(c["F"], c["G"], c["QU"], c["QdU"], c["R"], X, Up, ref_fn(k))
        Uk = sm[0, n:n + l]
        X = c["F"] @ X + c["G"] @ Uk
        Up = Uk
        want_X.append(X)
        want_U.append(Uk)
    want = np.concatenate([np.ravel(want_X), np.ravel(want_U)])
    Ns = [128, 1024, 8192]
    errs = []
    for N in Ns:
        e = []
        for s in range(8):
            def noise_fn(k, s=s, N=N):
                rng = np.random.default_rng(50_000 + 100 * s + k)
                return (rng.standard_normal((N, l, m)), rng.standard_normal((H, N, l, m)),
                        rng.standard_normal((H, N, n, m)), rng.standard_normal((H, N, l, m)))
            Xs, Us = enks.closed_loop(c["B"], w, 0, c["x0"], ref_fn, c["QU"], c["QdU"], c["R"], N, H,
                                      steps, noise_fn, U_prev=c["up"])
            assert np.array_equal(Xs[0], c["x0"])
            got = np.concatenate([np.ravel(Xs[1:]), np.ravel(Us)])
            e.append(np.linalg.norm(got - want) / np.linalg.norm(want))
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert -0.65 <= slope <= -0.35, (slope, errs)
    assert errs[-1] < 0.02, errs


def _full_conv_case(seed=7, n=5, m=4, l=2, H=3):
    """A linear layer with a full 3x3 kernel (2 -> 1 channels): it mixes columns, so the
    covariance is no longer of the matrix-normal form and the pooled gain differs from the
    vectorised Kalman gain."""
    c = _case(seed=seed, n=n, m=m, l=l, H=H)
    rng = np.random.default_rng(seed)
    c["w"] = rng.standard_normal((1, 2, 3, 3)) * 0.25
    return c


def test_conv_matrix_is_the_oracle_conv():
    from oracle import cnn
    c = _full_conv_case()
    n, m, l = c["n"], c["m"], c["l"]
    U = np.random.default_rng(2).standard_normal((l, m))
    got = cnn.cnn_forward(c["x0"], U, c["B"], [c["w"]], cnn.ACT_TANH)  # one layer: no activation
    Ax = cf.conv_matrix(c["w"][0, 0], n, m)
    Au = cf.conv_matrix(c["w"][0, 1], n, m)
    want = (Ax @ c["x0"].reshape(-1) + Au @ (c["B"] @ U).reshape(-1)).reshape(n, m)
    assert np.allclose(got, want, atol=1e-13)


def test_pooled_recursion_is_the_kalman_smoother_when_columns_do_not_mix():
    """With the centre-column kernel every column evolves alone with the same covariances:
    the pooled gain is the per-column Kalman gain, and both the pooled limit and the exact
    vectorised smoother equal the per-column Kalman filter + RTS smoother."""
    c = _case()
    w = cf.linear_weights(c["f"], c["g"])
    args = (c["QU"], c["QdU"], c["R"], c["x0"], c["up"], c["xref"])
    rts = cf.kalman_rts(c["F"], c["G"], *args)
    pooled = cf.pooled_recursion(w, c["B"], *args)
    exact = cf.pooled_recursion(w, c["B"], *args, pooled=False)
    scale = np.abs(rts).max()
    assert np.max(np.abs(pooled - rts)) <= 1e-10 * scale
    assert np.max(np.abs(exact - rts)) <= 1e-10 * scale


def test_enks_mean_converges_to_the_pooled_limit_for_a_full_conv():
    """A full 3x3 linear conv: the ensemble smoother's mean tends, at rate N^-1/2, to the
    pooled-gain limit (exact Gaussian propagation, gain pooled over columns, Joseph
    covariance update), and not to the exact vectorised Kalman smoother, which is far
    from it (the matrix-normal approximation error of this system)."""
    c = _full_conv_case()
    n, m, l, H = c["n"], c["m"], c["l"], c["H"]
    args = (c["QU"], c["QdU"], c["R"], c["x0"], c["up"], c["xref"])
    ref = cf.pooled_recursion(c["w"], c["B"], *args)
    exact = cf.pooled_recursion(c["w"], c["B"], *args, pooled=False)
    Ns = [32, 128, 512, 2048, 8192]
    errs = []
    for N in Ns:
        e = []
        for s in range(8):
            rng = np.random.default_rng(1000 + s)
            z = (rng.standard_normal((N, l, m)), rng.standard_normal((H, N, l, m)),
                 rng.standard_normal((H, N, n, m)), rng.standard_normal((H, N, l, m)))
            res = enks.solve(c["B"], [c["w"]], 0, c["x0"], c["xref"], c["QU"], c["QdU"], c["R"], N, H,
                             *z, U_prev=c["up"])
            full = np.concatenate([res.X_mean, res.U_mean, res.dU_mean], axis=1)
            e.append(np.linalg.norm(full - ref) / np.linalg.norm(ref))
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    gap = np.linalg.norm(exact - ref) / np.linalg.norm(ref)
    print(f"EnKS vs pooled limit: {errs}, slope {slope:.3f}; pooled vs exact smoother {gap:.3f}", flush=True)
    assert -0.62 <= slope <= -0.38, (slope, errs)
    assert errs[-1] < 0.06, errs
    assert gap > 5 * errs[-1], (gap, errs)
