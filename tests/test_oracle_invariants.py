"""Invariants and limits the method fixes: symmetric positive semi-definite covariances and
the sign of the covariance update, the lambda normalisation, and more."""
import numpy as np
import pytest

from oracle import cnn, enks
from paper_2410_09663_amd import workloads as wl


def _solve(p, seed=3, Up=None, QU=None, R=None, want_cov=False):
    prob = wl.make_problem(p)
    z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed)
    Q = prob.Q.astype(np.float64)
    res = enks.solve(prob.B, prob.weights, p.activation, prob.X0, wl.reference_window(p, 0),
                     Q if QU is None else QU, Q, prob.R if R is None else R, p.N, p.H,
                     z.Z_init, z.Z_W, z.Z_VX, z.Z_VU, U_prev=Up, want_cov=want_cov)
    return res, prob, z


def test_covariances_symmetric_psd():
    p = wl.small_preset(n=6, m=5, l=2, N=20, H=3)
    res, _, _ = _solve(p, want_cov=True)
    for S in res.syy + res.post_cov:
        S = np.asarray(S)
        assert np.max(np.abs(S - S.T)) <= 1e-14 * np.abs(S).max()
        ev = np.linalg.eigvalsh(0.5 * (S + S.T))
        assert ev.min() >= -1e-12 * np.abs(ev).max()
    for S in res.syy:  # Sigma^Y is positive definite ((N-1) m >= p)
        assert np.linalg.eigvalsh(S).min() > 0


def test_posterior_cov_has_the_conditional_minus_sign():
    """Eq. (14c) on the analysed ensemble matches the matrix-normal conditional of the
    appendix, Sigma_post = Sigma_prior - Sigma^{XY} (Sigma^Y)^{-1} Sigma^{XY}T, within
    Monte-Carlo error; the '+' printed in Eq. (10b) would not."""
    p = wl.small_preset(n=4, m=4, l=2, N=3000, H=2)
    res, _, _ = _solve(p, want_cov=True)
    for K, S, prior, post in zip(res.gains, res.syy, res.prior_cov, res.post_cov):
        Sxy = K @ S
        minus = prior - Sxy @ np.linalg.solve(S, Sxy.T)
        plus = prior + Sxy @ np.linalg.solve(S, Sxy.T)
        scale = np.linalg.norm(prior)
        assert np.linalg.norm(post - minus) < 0.05 * scale
        assert np.linalg.norm(post - plus) > 0.2 * scale


def test_dU_rows_are_increments():
    p = wl.small_preset(n=6, m=5, l=3, N=16, H=4)
    Up = 0.2 * np.random.default_rng(0).standard_normal((p.l, p.m))
    res, _, _ = _solve(p, Up=Up)
    mem = res.members  # (N, H+1, r, m)
    n, l = p.n, p.l
    U = mem[:, :, n:n + l]
    dU = mem[:, :, n + l:]
    assert np.max(np.abs(dU[:, 1:] - (U[:, 1:] - U[:, :-1]))) <= 1e-12
    assert np.max(np.abs(dU[:, 0] - (U[:, 0] - Up))) <= 1e-12


def test_zero_spread_rows_unchanged():
    p = wl.small_preset(n=6, m=5, l=2, N=16, H=4)
    res, prob, _ = _solve(p)
    # X_k has no spread in the initial ensemble, so its gain rows vanish
    assert np.max(np.abs(res.X_mean[0] - prob.X0)) <= 1e-12
    assert np.max(np.abs(res.members[:, 0, :p.n] - prob.X0)) <= 1e-12


def test_uninformative_observations_give_vanishing_gain():
    """With R, Q_U scaled by s -> infinity, the gain falls like s^-1/2 (the perturbed
    observations' spread grows like s^1/2), while the innovation grows like s^1/2."""
    p = wl.small_preset(n=5, m=4, l=2, N=12, H=3)
    norms = []
    for big in (1e6, 1e10):
        res, _, _ = _solve(p, QU=big * np.eye(p.l), R=big * np.eye(p.n))
        norms.append(max(np.abs(K).max() for K in res.gains))
    assert norms[1] < 1e-4
    assert 0.3e-2 < norms[1] / norms[0] < 3e-2  # ratio (1e10/1e6)^-1/2 = 1e-2


def test_lambda_normalisation_matches_appendix_identity():
    """E[(X - M)(X - M)^T] = tr(Psi) Sigma: with Psi = I_m the pooled estimator of
    Eq. (15d), (lambda/N) sum_i A^i A^iT with lambda = 1/m, estimates Sigma."""
    rng = np.random.default_rng(9)
    n, m, N = 5, 8, 20000
    Lq = np.linalg.cholesky(np.array(wl.random_spd(n, 3, scale=0.5), dtype=np.float64))
    X = np.matmul(Lq, rng.standard_normal((N, n, m))) + 2.0
    est = enks.forecast_cov(X)
    Sigma = Lq @ Lq.T
    se = np.sqrt((Sigma.diagonal()[:, None] * Sigma.diagonal()[None, :] + Sigma ** 2) / (N * m))
    assert np.all(np.abs(est - Sigma) <= 4 * se)
