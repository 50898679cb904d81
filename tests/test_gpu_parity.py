"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (each both normwise, ||gpu - oracle||_F / ||oracle||_F, and element-wise,
max |gpu - oracle| / max |oracle|):
  * FP32 solve: 1e-5 on the smoothed control means U_hat_{k..k+H} and on X_hat;
  * CNN rollout alone: 1e-5 per field batch;
  * device normals: bitwise FP32 equality (both sides round the same FP64 value;
    a 1-ulp FP64 difference in log/cos may flip an FP32 rounding, so at most
    1 in 10^5 values may differ, by 1 ulp).
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import enks, philox
from paper_2410_09663_amd import oic
from paper_2410_09663_amd import workloads as wl
from parity_util import assert_parity, relerr

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def oracle_solve(prob, Xref, z, U_prev=None, Q=None, R=None, N=None, H=None):
    p = prob.preset
    Q = prob.Q if Q is None else Q
    R = prob.R if R is None else R
    return enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, Q, Q, R,
                      N or p.N, H or p.H, *z, U_prev=U_prev)


def tiny(n=6, m=5, l=2, channels=(2, 3, 1), act=wl.ACT_TANH, N=7, H=3):
    return wl.small_preset(n=n, m=m, l=l, channels=channels, activation=act, N=N, H=H)


@pytest.mark.parametrize("kind,count", [(0, 1), (1, 4097), (2, 100003), (3, 30001)])
def test_device_normals_match_oracle(kind, count):
    prob = wl.make_problem(wl.PRESETS["C1"])
    with oic.controller_for(prob, max_N=64, max_H=8) as c:
        seed = (123 << 32) | 77
        got = c.normals(seed, kind, count)
    ref = philox.normals(seed, kind, (count,))
    diff = got != ref
    assert diff.sum() <= max(1, count // 100000)
    if diff.any():
        assert np.all(np.abs(got[diff].view(np.int32) - ref[diff].view(np.int32)) <= 1)


@pytest.mark.parametrize("preset", ["C1", "C2", "tiny", "tiny_gelu", "wide", "deep_a", "deep_b",
                                    "c16_ragged", "c16_l16", "fold64", "fold32"])
def test_cnn_forward_matches_oracle(preset):
    if preset == "fold64":
        # 64 -> 64 -> 1: the last layer folded into the last hidden layer's epilogue; 9 rows
        # and 70 columns leave ragged row and column tiles
        p = wl.small_preset(n=9, m=70, l=4, channels=(2, 64, 64, 64, 1), activation=wl.ACT_GELU, N=3)
    elif preset == "fold32":
        p = wl.small_preset(n=7, m=67, l=3, channels=(2, 16, 32, 64, 1), N=4)
    elif preset == "tiny":
        p = tiny()
    elif preset == "c16_ragged":
        # 2-16-16-1 with ragged row (13) and column (70 = 64 + 6) tiles
        p = wl.small_preset(n=13, m=70, l=5, channels=(2, 16, 16, 1), activation=wl.ACT_GELU, N=3)
    elif preset == "c16_l16":
        p = wl.small_preset(n=17, m=20, l=16, channels=(2, 16, 16, 1), N=4)
    elif preset == "deep_a":
        # hidden pairs (64,64), (64,32), (32,16), (16,64): channel-chunked MFMA layers;
        # 9 rows and 70 columns leave ragged row and column tiles
        p = wl.small_preset(n=9, m=70, l=4, channels=(2, 64, 64, 32, 16, 64, 1),
                            activation=wl.ACT_GELU, N=3)
    elif preset == "deep_b":
        p = wl.small_preset(n=13, m=66, l=5, channels=(2, 16, 32, 64, 16, 1), N=3)
    elif preset == "tiny_gelu":
        p = tiny(n=5, m=7, l=3, channels=(2, 5, 4, 1), act=wl.ACT_GELU)
    elif preset == "wide":
        p = wl.small_preset(n=12, m=20, l=3, channels=(2, 40, 1), activation=wl.ACT_GELU, N=9)
    else:
        p = wl.PRESETS[preset]
    prob = wl.make_problem(p)
    rng = np.random.default_rng(0)
    b = min(p.N, 16)
    X = rng.standard_normal((b, p.n, p.m)).astype(np.float32)
    U = rng.standard_normal((b, p.l, p.m)).astype(np.float32)
    with oic.controller_for(prob, max_N=b) as c:
        got = c.cnn_forward(X, U)
        one = c.plant_step(X[0], U[0])
    ref = ocnn.cnn_forward(X, U, prob.B, prob.weights, p.activation)
    assert_parity(got, ref, TOL_FP32, 'got vs ref')
    assert np.array_equal(one, got[0])


@pytest.mark.parametrize("preset", ["C1", "tiny", "tiny_gelu", "tiny_l1", "C2", "p90", "p100", "p150",
                                    "p500", "fold64", "smallest", "l_eq_n", "N2"])
def test_solve_explicit_noise_matches_oracle(preset):
    if preset == "smallest":
        # the smallest configuration the library accepts: a 4 x 5 field, one control row,
        # two members ((N - 1) m = 5 = n + l observation rows), one horizon step
        p = tiny(n=4, m=5, l=1, channels=(2, 3, 1), N=2, H=1)
    elif preset == "l_eq_n":
        p = tiny(n=4, m=6, l=4, channels=(2, 3, 1), N=4, H=2)
    elif preset == "N2":
        # two members over a wide field
        p = tiny(n=6, m=40, l=2, channels=(2, 8, 1), N=2, H=3)
    elif preset == "fold64":
        # 64-channel hidden layers with the last layer folded, on a ragged 20 x 72 field
        p = tiny(n=20, m=72, l=5, channels=(2, 64, 64, 1), act=wl.ACT_GELU, N=12, H=3)
    elif preset == "tiny":
        p = tiny()
    elif preset == "p90":
        # p = n + l = 90: the largest one-workgroup Cholesky, padded to 96 (the most LDS)
        p = tiny(n=72, m=6, l=18, channels=(2, 4, 1), N=40, H=2)
    elif preset == "p100":
        # p = n + l = 100 > 90: blocked Cholesky (panels 64 + 36) and triangular-solve gain
        p = tiny(n=80, m=6, l=20, channels=(2, 4, 1), N=40, H=2)
    elif preset == "p150":
        p = tiny(n=120, m=8, l=30, channels=(2, 4, 1), N=64, H=3)
    elif preset == "p500":
        # p = 500: eight panels, the gain's 16-row blocks
        p = tiny(n=400, m=4, l=100, channels=(2, 4, 1), N=400, H=2)
    elif preset == "tiny_gelu":
        p = tiny(n=5, m=7, l=3, channels=(2, 5, 4, 1), act=wl.ACT_GELU, N=6, H=4)
    elif preset == "tiny_l1":
        p = tiny(n=9, m=4, l=1, channels=(2, 2, 1), N=5, H=2)
    else:
        p = wl.PRESETS[preset]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=11)
    Up = (0.1 * np.random.default_rng(1).standard_normal((p.l, p.m))).astype(np.float32)
    with oic.controller_for(prob) as c:
        U, X = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, U_prev=Up, noise=z)
        U_applied = c.get_u_prev()
    ref = oracle_solve(prob, Xref, (z.Z_init, z.Z_W, z.Z_VX, z.Z_VU), U_prev=Up)
    eu, eu_max = assert_parity(U, ref.U_mean, TOL_FP32, f"{preset} U")
    ex, ex_max = assert_parity(X, ref.X_mean, TOL_FP32, f"{preset} X")
    print(f"{preset}: relerr U {eu:.2e} (max {eu_max:.2e}) X {ex:.2e} (max {ex_max:.2e})", flush=True)
    assert_parity(U[0], ref.U_mean[0], TOL_FP32, 'U[0] vs ref.U_mean[0]')
    assert np.array_equal(U_applied, U[0])


def test_seeded_solve_matches_oracle_with_philox_noise():
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    seed = 2024
    z = philox.solve_noise(seed, p.n, p.m, p.l, p.N, p.H)
    with oic.controller_for(prob) as c:
        U, X = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed, want_X=True)
    ref = oracle_solve(prob, Xref, z)
    assert_parity(U, ref.U_mean, TOL_FP32, 'U vs ref.U_mean')
    assert_parity(X, ref.X_mean, TOL_FP32, 'X vs ref.X_mean')


def test_dense_Q_and_R():
    p = tiny(n=8, m=6, l=3, channels=(2, 4, 1), N=10, H=3)
    prob = wl.make_problem(p)
    Q = wl.random_spd(p.l, 5, scale=0.05, cond=3.0)
    R = wl.random_spd(p.n, 6, scale=0.01, cond=5.0)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=4)
    with oic.controller_for(prob) as c:
        U, X = c.solve_ex(prob.X0, Xref, Q, R, p.N, p.H, noise=z)
    ref = oracle_solve(prob, Xref, (z.Z_init, z.Z_W, z.Z_VX, z.Z_VU), Q=Q, R=R)
    assert_parity(U, ref.U_mean, TOL_FP32, 'U vs ref.U_mean')
    assert_parity(X, ref.X_mean, TOL_FP32, 'X vs ref.X_mean')


def test_device_memory_mode_matches_host_mode_bitwise():
    import torch
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    with oic.controller_for(prob) as c:
        U_h, X_h = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed=5, want_X=True)
    stream = torch.cuda.current_stream().cuda_stream
    with oic.controller_for(prob, mem_mode=oic.OIC_MEM_DEVICE, stream=stream) as c:
        U_d, X_d = c.solve(torch.from_numpy(prob.X0).cuda(), torch.from_numpy(Xref).cuda(),
                           prob.Q, prob.R, p.N, p.H, seed=5, want_X=True)
        torch.cuda.synchronize()
        U_d, X_d = U_d.cpu().numpy(), X_d.cpu().numpy()
    assert np.array_equal(U_h, U_d) and np.array_equal(X_h, X_d)


def test_repeat_solves_are_bitwise_identical():
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    with oic.controller_for(prob, max_N=64, max_H=8) as c:
        outs = []
        for _ in range(3):
            c.set_u_prev(np.zeros((p.l, p.m), np.float32))
            outs.append(c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed=9, want_X=True))
    for U, X in outs[1:]:
        assert np.array_equal(U, outs[0][0]) and np.array_equal(X, outs[0][1])


def test_smaller_solve_in_larger_handle():
    """A handle sized for (max_N, max_H) solves smaller N and H correctly, before and
    after a larger solve (no stale state leaks between solves)."""
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    with oic.controller_for(prob, max_N=48, max_H=7) as c:
        for N, H in [(48, 7), (9, 2), (33, 5)]:
            Xref = wl.reference_window(p, 0, H)
            z = wl.host_noise(p.n, p.m, p.l, N, H, seed=N)
            c.set_u_prev(np.zeros((p.l, p.m), np.float32))
            U, X = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, N, H, noise=z)
            ref = oracle_solve(prob, Xref, (z.Z_init, z.Z_W, z.Z_VX, z.Z_VU), N=N, H=H)
            assert_parity(U, ref.U_mean, TOL_FP32, (N, H))


def test_error_paths_leave_outputs_untouched():
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    with oic.controller_for(prob) as c:
        with pytest.raises(oic.OicError) as e:
            c.solve(prob.X0, Xref, prob.Q, prob.R, 1, p.H, 0)
        assert e.value.code == oic.OIC_EINVAL
        with pytest.raises(oic.OicError) as e:
            c.solve(prob.X0, Xref, prob.Q, prob.R, p.N + 1, p.H, 0)
        assert e.value.code == oic.OIC_ENOMEM
        with pytest.raises(oic.OicError) as e:
            c.solve(prob.X0, Xref, -prob.Q, prob.R, p.N, p.H, 0)
        assert e.value.code == oic.OIC_EINVAL
        bad = prob.X0.copy()
        bad[3, 3] = np.nan
        with pytest.raises(oic.OicError) as e:
            c.solve(bad, Xref, prob.Q, prob.R, p.N, p.H, 0)
        assert e.value.code == oic.OIC_EINVAL
        # zero noise: no spread anywhere, Sigma^Ybar = 0 -> not positive definite
        zero = wl.Noise(*(np.zeros_like(a) for a in wl.host_noise(p.n, p.m, p.l, p.N, p.H, 0).__dict__.values()))
        before = c.get_u_prev()
        with pytest.raises(oic.OicError) as e:
            c.solve_ex(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, noise=zero)
        assert e.value.code == oic.OIC_ENOTSPD
        assert np.array_equal(c.get_u_prev(), before)
        # the handle still works afterwards
        U, _ = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, 1)
        assert np.all(np.isfinite(U))


def test_device_mode_failed_solve_leaves_outputs_untouched():
    """Device memory mode: a solve whose Sigma^Ybar is not positive definite reports
    OIC_ENOTSPD and writes neither the caller's output buffers nor the carried U_prev."""
    import torch
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    with oic.controller_for(prob, mem_mode=oic.OIC_MEM_DEVICE, stream=stream) as c:
        c.solve(dev(prob.X0), dev(Xref), prob.Q, prob.R, p.N, p.H, seed=2)  # U_prev now non-zero
        before = c.get_u_prev().clone()
        U_out = torch.full((p.H + 1, p.l, p.m), 7.0, device="cuda")
        X_out = torch.full((p.H + 1, p.n, p.m), -3.0, device="cuda")
        z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, 0)
        zero = tuple(torch.zeros_like(dev(a)) for a in (z.Z_init, z.Z_W, z.Z_VX, z.Z_VU))
        with pytest.raises(oic.OicError) as e:
            c.solve_ex(dev(prob.X0), dev(Xref), prob.Q, prob.R, p.N, p.H, noise=zero, U_out=U_out, X_out=X_out)
        assert e.value.code == oic.OIC_ENOTSPD
        torch.cuda.synchronize()
        assert bool(torch.all(U_out == 7.0)) and bool(torch.all(X_out == -3.0))
        assert torch.equal(c.get_u_prev(), before)
        # and a good solve afterwards writes them
        U, X = c.solve_ex(dev(prob.X0), dev(Xref), prob.Q, prob.R, p.N, p.H, noise=tuple(dev(a) for a in (
            z.Z_init, z.Z_W, z.Z_VX, z.Z_VU)), U_out=U_out, X_out=X_out)
        torch.cuda.synchronize()
        assert bool(torch.all(torch.isfinite(U_out))) and not bool(torch.all(U_out == 7.0))


@pytest.mark.parametrize("preset", ["C2", "tiny"])
@pytest.mark.parametrize("own_stream", [False, True])
def test_device_mode_forward_matches_host_mode_bitwise(preset, own_stream):
    """The forward in device memory mode reads and writes the caller's buffers directly
    (tiled and generic layer paths; on the caller's stream and on a private one)."""
    import torch
    p = tiny() if preset == "tiny" else wl.PRESETS[preset]
    prob = wl.make_problem(p)
    rng = np.random.default_rng(4)
    b = 3
    X = rng.standard_normal((b, p.n, p.m)).astype(np.float32)
    U = rng.standard_normal((b, p.l, p.m)).astype(np.float32)
    with oic.controller_for(prob) as c:
        ref = c.cnn_forward(X, U)
        ref_plant = c.plant_step(X[0], U[0])
    kw = {} if own_stream else {"stream": torch.cuda.current_stream().cuda_stream}
    with oic.controller_for(prob, mem_mode=oic.OIC_MEM_DEVICE, **kw) as c:
        got = c.cnn_forward(torch.from_numpy(X).cuda(), torch.from_numpy(U).cuda())
        got_plant = c.plant_step(torch.from_numpy(X[0]).cuda(), torch.from_numpy(U[0]).cuda())
        torch.cuda.synchronize()
        got, got_plant = got.cpu().numpy(), got_plant.cpu().numpy()
    assert np.array_equal(ref, got) and np.array_equal(ref_plant, got_plant)


def test_closed_loop_teacher_forced():
    """Three closed-loop steps of C2-shaped dynamics at C1 size: at each step the
    oracle solves from the library's own state X_k and applied U_{k-1}."""
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    X = prob.X0.copy()
    Up = np.zeros((p.l, p.m), np.float32)
    with oic.controller_for(prob) as c:
        for k in range(3):
            Xref = wl.reference_window(p, k)
            z = philox.solve_noise(100 + k, p.n, p.m, p.l, p.N, p.H)
            U, _ = c.solve(X, Xref, prob.Q, prob.R, p.N, p.H, 100 + k)
            ref = enks.solve(prob.B, prob.weights, p.activation, X, Xref, prob.Q, prob.Q, prob.R,
                             p.N, p.H, *z, U_prev=Up)
            assert_parity(U, ref.U_mean, TOL_FP32, k)
            Up = c.get_u_prev()
            assert np.array_equal(Up, U[0])
            Xn = c.plant_step(X, Up)
            assert_parity(Xn, enks.plant_step(X, Up, prob.B, prob.weights, p.activation), TOL_FP32, 'Xn vs enks.plant_step(X, Up, prob.B, prob.weights, p.activation)')
            X = Xn


def test_graph_replay_matches_eager_bitwise():
    """The captured solve replays bitwise like the kernel-by-kernel launch, picks up a
    new seed on every replay, and is re-captured when N or H change."""
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    zero = np.zeros((p.l, p.m), np.float32)
    with oic.controller_for(prob, max_N=48, max_H=7) as c:
        c.set_graph(False)
        c.set_u_prev(zero)
        U_e, X_e = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, 3, want_X=True)
        c.set_graph(True)
        outs = []
        for seed in (3, 4, 3):
            c.set_u_prev(zero)
            outs.append(c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed, want_X=True))
        assert np.array_equal(outs[0][0], U_e) and np.array_equal(outs[0][1], X_e)
        assert np.array_equal(outs[2][0], U_e)
        assert not np.array_equal(outs[1][0], U_e)
        ref4 = oracle_solve(prob, Xref, philox.solve_noise(4, p.n, p.m, p.l, p.N, p.H))
        assert_parity(outs[1][0], ref4.U_mean, TOL_FP32, 'outs[1][0] vs ref4.U_mean')
        # a different shape forces a new capture; explicit noise too
        Xref2 = wl.reference_window(p, 0, 2)
        c.set_u_prev(zero)
        U2, _ = c.solve(prob.X0, Xref2, prob.Q, prob.R, 40, 2, 5)
        z2 = philox.solve_noise(5, p.n, p.m, p.l, 40, 2)
        assert_parity(U2, oracle_solve(prob, Xref2, z2, N=40, H=2).U_mean, TOL_FP32, 'U2 vs oracle_solve(prob, Xref2, z2, N=40, H=2).U_mean')
        c.set_u_prev(zero)
        U3, _ = c.solve_ex(prob.X0, Xref2, prob.Q, prob.R, 40, 2, noise=z2)
        assert relerr(U3, U2) < 1e-6  # device and host Philox normals agree (bitwise, up to rare 1-ulp)


@pytest.mark.parametrize("preset", ["tiny", "C1"])
def test_covariance_outputs_match_oracle(preset):
    """Optional outputs of Algorithm 1 (lines 8 and 11): the pooled covariance of the
    stored trajectory before (Eqs. 15d-15f) and after (Eq. 14c) every analysis, against
    the oracle's (whose slices also carry the Delta U rows, dropped here)."""
    p = tiny() if preset == "tiny" else wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=5)
    Up = np.zeros((p.l, p.m), np.float32)  # both solves start from the same U_prev
    with oic.controller_for(prob) as c:
        U, X, prior, post = c.solve_cov(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, U_prev=Up, noise=z)
        U2, X2 = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, U_prev=Up, noise=z)
    assert np.array_equal(U, U2) and np.array_equal(X, X2)  # the covariances change nothing
    ref = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, p.N,
                     p.H, z.Z_init, z.Z_W, z.Z_VX, z.Z_VU, want_cov=True)
    rows = p.n + 2 * p.l
    for t in range(1, p.H + 1):
        keep = np.concatenate([s * rows + np.arange(p.n + p.l) for s in range(t + 1)])
        for got, want in ((prior[t - 1], ref.prior_cov[t - 1]), (post[t - 1], ref.post_cov[t - 1])):
            want = want[np.ix_(keep, keep)]
            assert got.shape == want.shape
            assert_parity(got, want, TOL_FP32, (t, relerr(got, want)))
            assert np.allclose(got, got.T, rtol=0, atol=1e-12 * np.abs(got).max())


def _constraint(p, rng):
    c = enks.Constraint(aX=rng.standard_normal(p.n).astype(np.float32) / p.n,
                        aU=np.full(p.l, 1.0 / p.l, np.float32), b=float(np.float32(0.05)),
                        alpha=float(np.float32(2.0)), beta=float(np.float32(8.0)),
                        rz=float(np.float32(1e-3)))
    return c


@pytest.mark.parametrize("preset", ["tiny", "C1"])
def test_constrained_solve_matches_oracle(preset):
    """The barrier-observed constraint as one more row of Ybar (explicit noise), against
    the oracle; then removing it gives the unconstrained solve again."""
    p = tiny(N=12) if preset == "tiny" else wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    rng = np.random.default_rng(31)
    con = _constraint(p, rng)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=13)
    zz = rng.standard_normal((p.H, p.N, 1, p.m)).astype(np.float32)
    Up = np.zeros((p.l, p.m), np.float32)
    with oic.controller_for(prob) as c:
        c.set_constraint(con.aX, con.aU, con.b, con.alpha, con.beta, con.rz)
        U, X = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, U_prev=Up, noise=z, Z_VZ=zz)
        c.set_constraint()
        U0, _ = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, U_prev=Up, noise=z)
    ref = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, p.N, p.H,
                     z.Z_init, z.Z_W, z.Z_VX, z.Z_VU, constraint=con, Z_VZ=zz)
    ref0 = oracle_solve(prob, Xref, (z.Z_init, z.Z_W, z.Z_VX, z.Z_VU), U_prev=Up)
    eu, _ = assert_parity(U, ref.U_mean, TOL_FP32, "constrained U")
    ex, _ = assert_parity(X, ref.X_mean, TOL_FP32, "constrained X")
    print(f"{preset} constrained: relerr U {eu:.2e} X {ex:.2e}", flush=True)
    assert_parity(U0, ref0.U_mean, TOL_FP32, 'U0 vs ref0.U_mean')
    assert relerr(ref.U_mean, ref0.U_mean) > 1e-3  # the constraint did change the solve


def test_constrained_seeded_solve_uses_noise_kind_4():
    p = wl.PRESETS["C1"]
    prob = wl.make_problem(p)
    con = _constraint(p, np.random.default_rng(32))
    Xref = wl.reference_window(p, 0)
    seed = 77
    with oic.controller_for(prob) as c:
        c.set_constraint(con.aX, con.aU, con.b, con.alpha, con.beta, con.rz)
        U, _ = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed)
    z = philox.solve_noise(seed, p.n, p.m, p.l, p.N, p.H)
    zz = philox.normals(seed, 4, (p.H, p.N, 1, p.m))
    ref = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, p.N, p.H,
                     *z, constraint=con, Z_VZ=zz)
    assert_parity(U, ref.U_mean, TOL_FP32, 'U vs ref.U_mean')


def _graph_vs_eager(prob, p, steps):
    """Run the same sequence of (action, solve) steps on a graph-replaying handle and on
    an eager one; return both lists of (U_hat, X_hat)."""
    Xref = wl.reference_window(p, 0)
    zero = np.zeros((p.l, p.m), np.float32)
    outs = {}
    for graph in (False, True):
        with oic.controller_for(prob) as c:
            c.set_graph(graph)
            res = []
            for action, (Q, R) in steps:
                action(c)
                c.set_u_prev(zero)
                res.append(c.solve(prob.X0, Xref, Q, R, p.N, p.H, 3, want_X=True))
            outs[graph] = res
    return outs[False], outs[True]


def test_graph_recaptured_when_noise_factor_layout_changes():
    """A replayed solve must follow a switch between diagonal and dense Q or R at the
    same N and H (the noise kernels read a diagonal factor as scales, a dense one as a
    triangle): graph and eager results agree bitwise, and the dense solve matches the
    oracle."""
    p = tiny(n=8, m=6, l=3, channels=(2, 4, 1), N=10, H=3)
    prob = wl.make_problem(p)
    Qd, Rd = prob.Q, prob.R
    Qf = wl.random_spd(p.l, 5, scale=0.05, cond=3.0)
    Rf = wl.random_spd(p.n, 6, scale=0.01, cond=5.0)
    keep = lambda c: None
    seq = [(keep, (Qd, Rd)), (keep, (Qf, Rd)), (keep, (Qf, Rf)), (keep, (Qd, Rf)), (keep, (Qd, Rd))]
    eager, graph = _graph_vs_eager(prob, p, seq)
    for k, ((Ue, Xe), (Ug, Xg)) in enumerate(zip(eager, graph)):
        assert np.array_equal(Ue, Ug) and np.array_equal(Xe, Xg), k
    z = philox.solve_noise(3, p.n, p.m, p.l, p.N, p.H)
    Xref = wl.reference_window(p, 0)
    for k, (Q, R) in ((1, (Qf, Rd)), (2, (Qf, Rf)), (3, (Qd, Rf))):
        ref = oracle_solve(prob, Xref, z, Q=Q, R=R)
        assert_parity(graph[k][0], ref.U_mean, TOL_FP32, f"step {k} U")
    assert not np.array_equal(graph[0][0], graph[1][0])


def test_graph_recaptured_when_bias_changes():
    """Setting weights with biases, then without, then with again on a graph-replaying
    handle gives the eager results bitwise (the bias buffers are allocated and freed
    between the solves), and the biased solve matches the oracle with the same biases."""
    p = tiny(n=7, m=9, l=2, channels=(2, 5, 1), N=12, H=3)
    prob = wl.make_problem(p)
    rng = np.random.default_rng(8)
    biases = [(0.1 * rng.standard_normal(co)).astype(np.float32) for co in p.channels[1:]]
    with_b = lambda c: c.set_weights(prob.B, prob.weights, biases)
    without = lambda c: c.set_weights(prob.B, prob.weights)
    QR = (prob.Q, prob.R)
    eager, graph = _graph_vs_eager(prob, p, [(with_b, QR), (without, QR), (with_b, QR)])
    for k, ((Ue, Xe), (Ug, Xg)) in enumerate(zip(eager, graph)):
        assert np.array_equal(Ue, Ug) and np.array_equal(Xe, Xg), k
    z = philox.solve_noise(3, p.n, p.m, p.l, p.N, p.H)
    Xref = wl.reference_window(p, 0)
    ref_b = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R,
                       p.N, p.H, *z, biases=biases)
    assert_parity(graph[0][0], ref_b.U_mean, TOL_FP32, "biased U")
    assert_parity(graph[1][0], oracle_solve(prob, Xref, z).U_mean, TOL_FP32, "unbiased U")
    assert np.array_equal(graph[0][0], graph[2][0])


@pytest.mark.parametrize("shape", ["fp32_tanh", "bf16_fold64"])
def test_new_weights_in_the_same_buffers_reach_a_replayed_solve(shape):
    """oic_set_weights with a new surrogate of the same shape and no change of biases keeps
    the captured solve (its buffers are rewritten in place): graph replays give the eager
    results bitwise for both surrogates, in both orders, and the FP32 replays match the
    oracle with the weights of their own step. The BF16 case covers the re-laid-out BF16
    weights and the folded last layer's BF16 pair."""
    if shape == "fp32_tanh":
        p = tiny(n=8, m=7, l=2, channels=(2, 6, 1), N=9, H=3)
    else:
        p = dataclasses.replace(wl.small_preset(n=12, m=70, l=3, channels=(2, 64, 64, 64, 1),
                                                activation=wl.ACT_GELU, N=6, H=2), precision=wl.PREC_BF16)
    prob = wl.make_problem(p)
    W2 = wl.he_weights(p.channels, seed=1234)
    B2 = wl.lift_matrix(p.n, p.l, seed=4321)
    first = lambda c: c.set_weights(prob.B, prob.weights)
    second = lambda c: c.set_weights(B2, W2)
    QR = (prob.Q, prob.R)
    eager, graph = _graph_vs_eager(prob, p, [(first, QR), (second, QR), (first, QR)])
    for k, ((Ue, Xe), (Ug, Xg)) in enumerate(zip(eager, graph)):
        assert np.array_equal(Ue, Ug) and np.array_equal(Xe, Xg), k
    assert np.array_equal(graph[0][0], graph[2][0])
    assert not np.array_equal(graph[0][0], graph[1][0])
    if shape == "fp32_tanh":
        z = philox.solve_noise(3, p.n, p.m, p.l, p.N, p.H)
        Xref = wl.reference_window(p, 0)
        ref2 = enks.solve(B2, W2, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, p.N, p.H, *z)
        assert_parity(graph[1][0], ref2.U_mean, TOL_FP32, "second surrogate U")
        assert_parity(graph[0][0], oracle_solve(prob, Xref, z).U_mean, TOL_FP32, "first surrogate U")
