"""Pins of the constraint extension of the oracle (a barrier-observed constraint appended
to the virtual observation as one more row with actual value 0):

* the softplus barrier's closed-form limits: 0 far inside, the line (beta/alpha) x far
  outside, ln(2)/alpha on the boundary;
* with an overwhelming observation noise (rz -> infinity) the extra row carries no
  information: what remains is a sampling effect that shrinks with the ensemble size;
* the analysis with the extra row equals dense vectorised brute force;
* a violated constraint on the control pulls the smoothed control toward feasibility."""
import numpy as np

from oracle import enks
from paper_2410_09663_amd import workloads as wl

from test_oracle_bruteforce import brute_analysis


def _problem(N=64, H=3, n=6, m=5, l=2):
    p = wl.small_preset(n=n, m=m, l=l, channels=(2, 3, 1), N=N, H=H)
    prob = wl.make_problem(p)
    z = wl.host_noise(n, m, l, N, H, seed=9)
    zz = np.random.default_rng(10).standard_normal((H, N, 1, m))
    return p, prob, z, zz


def _solve(p, prob, z, constraint=None, zz=None, Xref=None):
    Xref = wl.reference_window(p, 0) if Xref is None else Xref
    return enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, p.N,
                      p.H, z.Z_init, z.Z_W, z.Z_VX, z.Z_VU, constraint=constraint, Z_VZ=zz)


def test_barrier_limits():
    c = enks.Constraint(np.zeros(3), np.zeros(2), 0.0, alpha=2.0, beta=5.0, rz=1e-4)
    assert abs(c.barrier(0.0) - np.log(2.0) / 2.0) < 1e-15
    assert c.barrier(-50.0) < 1e-100
    assert abs(c.barrier(50.0) - 2.5 * 50.0) < 1e-12  # (beta / alpha) x, up to e^{-250}
    assert np.isfinite(c.barrier(1e6))


def test_overwhelming_noise_only_adds_sampling_error():
    # With rz -> infinity the extra row carries no information about the state; in a
    # finite ensemble it still acts as one sampled regressor (its sample correlation
    # with the other anomalies is O(1/sqrt(N)) and its scale cancels in the gain), so
    # the solve differs from the unconstrained one by an rz-independent amount that
    # shrinks as the ensemble grows.
    rel = {}
    for N in (64, 1024):
        p, prob, z, zz = _problem(N=N)
        base = _solve(p, prob, z)
        for rz in (1e10, 1e14):
            c = enks.Constraint(np.full(p.n, 1.0 / p.n), np.full(p.l, 0.5), 0.0, alpha=1.0, beta=4.0,
                                rz=rz)
            con = _solve(p, prob, z, c, zz)
            rel[N, rz] = np.linalg.norm(con.U_mean - base.U_mean) / np.linalg.norm(base.U_mean)
    assert abs(rel[64, 1e10] - rel[64, 1e14]) < 1e-3 * rel[64, 1e14]
    assert rel[1024, 1e14] < 0.5 * rel[64, 1e14]
    # a small noise makes the row informative: a much larger change
    p, prob, z, zz = _problem()
    base = _solve(p, prob, z)
    c = enks.Constraint(np.full(p.n, 1.0 / p.n), np.full(p.l, 0.5), 0.0, alpha=1.0, beta=4.0, rz=1e-4)
    con = _solve(p, prob, z, c, zz)
    assert np.linalg.norm(con.U_mean - base.U_mean) / np.linalg.norm(base.U_mean) > 10 * rel[64, 1e14]


def test_constrained_analysis_matches_bruteforce():
    rng = np.random.default_rng(11)
    N, a, n, l, m = 12, 7, 3, 2, 4
    Xcal = rng.standard_normal((N, a, m))
    c = enks.Constraint(rng.standard_normal(n), rng.standard_normal(l), 0.2, alpha=1.5, beta=3.0, rz=0.01)
    Xt, Ut = rng.standard_normal((N, n, m)), rng.standard_normal((N, l, m))
    z = c.barrier(c.g(Xt, Ut)) + 0.1 * rng.standard_normal((N, m))
    Y = np.concatenate([Xt + 0.1 * rng.standard_normal((N, n, m)), Ut, z[:, None, :]], axis=1)
    Ybar = np.concatenate([rng.standard_normal((n, m)), np.zeros((l + 1, m))], axis=0)
    got, K, _ = enks.analysis(Xcal, Y, Ybar)
    want, Kb = brute_analysis(Xcal, Y, Ybar)
    assert np.allclose(got, want, atol=1e-10)
    assert np.allclose(K, Kb, atol=1e-10)


def test_violated_control_constraint_pulls_toward_feasibility():
    # g_c = mean over the control rows of column c, minus b: keep the column means of U
    # below b, with b below what the unconstrained solve returns
    p, prob, z, zz = _problem(N=256, H=4)
    base = _solve(p, prob, z)
    gb = base.U_mean.mean(axis=1)  # (H+1, m): column means of U_hat
    b = float(np.median(gb)) - 0.05
    c = enks.Constraint(np.zeros(p.n), np.full(p.l, 1.0 / p.l), b, alpha=1.0, beta=20.0, rz=1e-3)
    con = _solve(p, prob, z, c, zz)
    viol = lambda U: np.maximum(U.mean(axis=1)[1:] - b, 0.0).sum()  # slices k+1..k+H
    assert viol(con.U_mean) < 0.5 * viol(base.U_mean)
