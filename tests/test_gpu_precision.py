"""BF16 rollout (BF16 activations and weights on MFMA, FP32 accumulation; statistics FP64,
gain FP64): errors against the FP64 oracle and against the FP32 GPU path.

Bars (relative, Frobenius): 2e-2 on the smoothed control mean, 2e-2 on the state mean,
and 2% on the closed-loop tracking cost."""
import dataclasses

import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import cost as ocost
from oracle import enks, philox
from paper_2410_09663_amd import oic
from paper_2410_09663_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_BF16 = 2e-2


def relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("preset", ["C2", "C3"])
def test_bf16_rollout_vs_oracle(preset):
    p = wl.PRESETS[preset]
    prob = wl.make_problem(p)
    rng = np.random.default_rng(0)
    b = 8
    X = rng.standard_normal((b, p.n, p.m)).astype(np.float32)
    U = (0.3 * rng.standard_normal((b, p.l, p.m))).astype(np.float32)
    with oic.controller_for(prob, max_N=b, precision=oic.OIC_PREC_BF16) as c:
        got = c.cnn_forward(X, U)
        plant = c.plant_step(X[0], U[0])
    ref = ocnn.cnn_forward(X, U, prob.B, prob.weights, p.activation)
    e = relerr(got, ref)
    print(f"{preset} bf16 rollout relerr {e:.2e}", flush=True)
    assert e < TOL_BF16
    assert e > 1e-6  # it really ran in BF16
    assert relerr(plant, ref[0]) < 1e-5  # the plant stays FP32


@pytest.mark.parametrize("preset,N,H", [("C2", 128, 10), ("C3", 32, 3)])
def test_bf16_solve_vs_oracle(preset, N, H):
    p = dataclasses.replace(wl.PRESETS[preset], N=N, H=H)
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, N, H, seed=21)
    with oic.controller_for(prob, precision=oic.OIC_PREC_BF16) as c:
        U, X = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, N, H, noise=z)
    ref = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, N, H,
                     z.Z_init, z.Z_W, z.Z_VX, z.Z_VU)
    eu, ex = relerr(U, ref.U_mean), relerr(X, ref.X_mean)
    print(f"{preset} N={N} H={H} bf16: relerr U {eu:.2e} X {ex:.2e}", flush=True)
    assert eu < TOL_BF16
    assert ex < TOL_BF16


def test_bf16_vs_fp32_gpu_full_c3():
    p = wl.PRESETS["C3"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    outs = {}
    for prec in (oic.OIC_PREC_FP32, oic.OIC_PREC_BF16):
        with oic.controller_for(prob, precision=prec) as c:
            outs[prec] = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed=7, want_X=True)
    eu = relerr(outs[oic.OIC_PREC_BF16][0], outs[oic.OIC_PREC_FP32][0])
    ex = relerr(outs[oic.OIC_PREC_BF16][1], outs[oic.OIC_PREC_FP32][1])
    print(f"C3 full size bf16 vs fp32 GPU: relerr U {eu:.2e} X {ex:.2e}", flush=True)
    assert eu < TOL_BF16 and ex < TOL_BF16


def closed_loop(prob, precision, steps):
    p = prob.preset
    X = prob.X0.copy()
    Xs, Us = [X], []
    with oic.controller_for(prob, precision=precision) as c:
        for k in range(steps):
            U, _ = c.solve(X, wl.reference_window(p, k), prob.Q, prob.R, p.N, p.H, 5000 + k)
            X = c.plant_step(X, U[0])
            Xs.append(X)
            Us.append(U[0])
    Xrefs = np.stack([wl.reference_at(p, k) for k in range(steps + 1)])
    return ocost.closed_loop_cost(np.stack(Xs), np.stack(Us), np.zeros((p.l, p.m)), Xrefs,
                                  prob.R.astype(np.float64), prob.Q.astype(np.float64))


@pytest.mark.parametrize("preset,steps", [("C2", 20), ("C3", 10)])
def test_bf16_closed_loop_tracking_cost_within_2pct(preset, steps):
    prob = wl.make_problem(wl.PRESETS[preset])
    j32 = closed_loop(prob, oic.OIC_PREC_FP32, steps)
    j16 = closed_loop(prob, oic.OIC_PREC_BF16, steps)
    print(f"{preset} closed-loop cost fp32 {j32:.6e} bf16 {j16:.6e} rel {abs(j16 - j32) / j32:.2e}",
          flush=True)
    assert abs(j16 - j32) / j32 < 0.02
