"""BF16 rollout (BF16 activations and weights on MFMA, FP32 accumulation; statistics and
update as three BF16 matrix-core products of split operands, about 2^-16 per product, with
FP32 sums folded into FP64; gain FP64): errors against the FP64 oracle and against the FP32
GPU path.

Bars: 2e-2 on the smoothed control mean and on the state mean (normwise, and element-wise
relative to the largest magnitude), and 2% on the closed-loop tracking cost."""
import dataclasses

import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import cost as ocost
from oracle import enks, philox
from paper_2410_09663_amd import oic
from paper_2410_09663_amd import workloads as wl
from parity_util import assert_parity, max_relerr, relerr

pytestmark = pytest.mark.gpu

TOL_BF16 = 2e-2


FOLD64 = wl.small_preset(n=20, m=72, l=5, channels=(2, 64, 64, 64, 1), activation=wl.ACT_GELU, N=8, H=3)
FOLD32 = wl.small_preset(n=13, m=66, l=4, channels=(2, 32, 64, 1), N=8, H=3)
# odd p = n + l = 97 (> 80: strip update with its gain split into BF16 planes, gain rows not
# 16-byte aligned; statistics with a partial right tile)
RAGGED_P = wl.small_preset(n=90, m=20, l=7, channels=(2, 16, 16, 1), N=12, H=3)


@pytest.mark.parametrize("preset", ["C2", "C3", "fold64", "fold32", "ragged_p"])
def test_bf16_rollout_vs_oracle(preset):
    # fold64 / fold32: the last layer folded into the last BF16 hidden layer (64 outputs)
    p = {"fold64": FOLD64, "fold32": FOLD32, "ragged_p": RAGGED_P}.get(preset) or wl.PRESETS[preset]
    prob = wl.make_problem(p)
    rng = np.random.default_rng(0)
    b = 8
    X = rng.standard_normal((b, p.n, p.m)).astype(np.float32)
    U = (0.3 * rng.standard_normal((b, p.l, p.m))).astype(np.float32)
    with oic.controller_for(prob, max_N=b, precision=oic.OIC_PREC_BF16) as c:
        got = c.cnn_forward(X, U)
        plant = c.plant_step(X[0], U[0])
    ref = ocnn.cnn_forward(X, U, prob.B, prob.weights, p.activation)
    e, e_max = assert_parity(got, ref, TOL_BF16, "rollout")
    print(f"{preset} bf16 rollout relerr {e:.2e} (max {e_max:.2e})", flush=True)
    assert e > 1e-6  # it really ran in BF16
    assert_parity(plant, ref[0], 1e-5, "plant")  # the plant stays FP32


@pytest.mark.parametrize("preset,N,H", [("C2", 128, 10), ("C3", 32, 3), ("fold64", 12, 3), ("ragged_p", 32, 3)])
def test_bf16_solve_vs_oracle(preset, N, H):
    base = {"fold64": FOLD64, "ragged_p": RAGGED_P}.get(preset) or wl.PRESETS[preset]
    p = dataclasses.replace(base, N=N, H=H)
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    z = wl.host_noise(p.n, p.m, p.l, N, H, seed=21)
    with oic.controller_for(prob, precision=oic.OIC_PREC_BF16) as c:
        U, X = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, N, H, noise=z)
    ref = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R, N, H,
                     z.Z_init, z.Z_W, z.Z_VX, z.Z_VU)
    eu, eu_max = assert_parity(U, ref.U_mean, TOL_BF16, "U")
    ex, ex_max = assert_parity(X, ref.X_mean, TOL_BF16, "X")
    print(f"{preset} N={N} H={H} bf16: relerr U {eu:.2e} (max {eu_max:.2e}) X {ex:.2e} "
          f"(max {ex_max:.2e})", flush=True)


def test_bf16_vs_fp32_gpu_full_c3():
    p = wl.PRESETS["C3"]
    prob = wl.make_problem(p)
    Xref = wl.reference_window(p, 0)
    outs = {}
    for prec in (oic.OIC_PREC_FP32, oic.OIC_PREC_BF16):
        with oic.controller_for(prob, precision=prec) as c:
            outs[prec] = c.solve(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, seed=7, want_X=True)
    eu, _ = assert_parity(outs[oic.OIC_PREC_BF16][0], outs[oic.OIC_PREC_FP32][0], TOL_BF16, "U")
    ex, _ = assert_parity(outs[oic.OIC_PREC_BF16][1], outs[oic.OIC_PREC_FP32][1], TOL_BF16, "X")
    print(f"C3 full size bf16 vs fp32 GPU: relerr U {eu:.2e} X {ex:.2e}", flush=True)


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


# ---- FP8 (OCP e4m3) hidden layers: per-output-channel weight scales, per-layer
# activation scales from the ensemble's largest magnitude, BF16 storage between layers.
#
# e4m3 keeps 3 mantissa bits (BF16: 8), so every FP8 layer perturbs its output by a few
# per cent, about 16x the BF16 error; measured on these workloads the FP8 path does NOT
# reach the 2e-2 / 2% bars that BF16 meets.  These tests pin the FP8 path to the error
# bands it does reach (regression guards), each with the measured value beside it.

TOL_FP8_ROLLOUT = 9e-2   # three FP8 layers, white-noise inputs: measured 6.5e-2 .. 7.5e-2
TOL_FP8_U = 3.5e-2       # smoothed control mean, 40x40 solve: measured 2.6e-2
TOL_FP8_COST = 6e-2      # closed-loop tracking cost, 10 steps: measured 3.7e-2


def fp8_preset(n=40, l=10, channels=(2, 32, 32, 32, 1), N=64, H=5):
    return dataclasses.replace(wl.PRESETS["C3"], name="f8", n=n, m=n, l=l, channels=list(channels),
                               N=N, H=H, grf_length=4.0, ref_sigma=4.0, ref_center=(n / 2, n / 4),
                               precision=wl.PREC_FP8)


@pytest.mark.parametrize("channels", [(2, 32, 32, 32, 1), (2, 64, 64, 64, 1), (2, 32, 64, 16, 1)])
def test_fp8_rollout_vs_oracle(channels):
    p = fp8_preset(channels=channels)
    prob = wl.make_problem(p)
    rng = np.random.default_rng(0)
    b = 8
    X = rng.standard_normal((b, p.n, p.m)).astype(np.float32)
    U = (0.3 * rng.standard_normal((b, p.l, p.m))).astype(np.float32)
    with oic.controller_for(prob, max_N=b, precision=oic.OIC_PREC_FP8) as c:
        got = c.cnn_forward(X, U)
        plant = c.plant_step(X[0], U[0])
    with oic.controller_for(prob, max_N=b, precision=oic.OIC_PREC_BF16) as c:
        got16 = c.cnn_forward(X, U)
    ref = ocnn.cnn_forward(X, U, prob.B, prob.weights, p.activation)
    e, e16 = relerr(got, ref), relerr(got16, ref)
    print(f"{channels} fp8 rollout relerr {e:.2e} (bf16 {e16:.2e})", flush=True)
    assert e < TOL_FP8_ROLLOUT
    assert e > 2 * e16  # it really ran in FP8
    assert_parity(plant, ref[0], 1e-5, "plant")  # the plant stays FP32


TOL_FP8_BAR_U = 2e-2     # the stated bar on the smoothed control mean
TOL_FP8_BAR_COST = 0.02  # and on the closed-loop tracking cost
_cache = {}


def _fp8_solve_errors():
    if "solve" not in _cache:
        p = fp8_preset()
        prob = wl.make_problem(p)
        Xref = wl.reference_window(p, 0)
        z = wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=23)
        with oic.controller_for(prob, precision=oic.OIC_PREC_FP8) as c:
            U, X = c.solve_ex(prob.X0, Xref, prob.Q, prob.R, p.N, p.H, noise=z)
        ref = enks.solve(prob.B, prob.weights, p.activation, prob.X0, Xref, prob.Q, prob.Q, prob.R,
                         p.N, p.H, z.Z_init, z.Z_W, z.Z_VX, z.Z_VU)
        _cache["solve"] = (relerr(U, ref.U_mean), relerr(X, ref.X_mean), max_relerr(U, ref.U_mean))
    return _cache["solve"]


def _fp8_cost_error():
    if "cost" not in _cache:
        prob = wl.make_problem(fp8_preset())
        j32 = closed_loop(prob, oic.OIC_PREC_FP32, 10)
        j8 = closed_loop(prob, oic.OIC_PREC_FP8, 10)
        _cache["cost"] = (j32, j8, abs(j8 - j32) / j32)
    return _cache["cost"]


def test_fp8_solve_vs_oracle():
    eu, ex, eu_max = _fp8_solve_errors()
    print(f"fp8 solve: relerr U {eu:.2e} (max {eu_max:.2e}) X {ex:.2e}", flush=True)
    assert eu < TOL_FP8_U
    assert ex < TOL_BF16


@pytest.mark.xfail(strict=True, reason="FP8 e4m3 misses the 2e-2 bar on U_hat (measured 2.6e-2 at 40x40)")
def test_fp8_solve_meets_the_bar():
    eu, _, eu_max = _fp8_solve_errors()
    assert eu < TOL_FP8_BAR_U and eu_max < TOL_FP8_BAR_U


def test_fp8_closed_loop_tracking_cost():
    j32, j8, rel = _fp8_cost_error()
    print(f"fp8 closed-loop cost fp32 {j32:.6e} fp8 {j8:.6e} rel {rel:.2e}", flush=True)
    assert rel < TOL_FP8_COST


@pytest.mark.xfail(strict=True, reason="FP8 e4m3 misses the 2% cost bar at 40x40 (measured 3.7%)")
def test_fp8_closed_loop_cost_meets_the_bar():
    assert _fp8_cost_error()[2] < TOL_FP8_BAR_COST


def _full_size_256():
    """256x256 field, 5-layer 64-channel GELU CNN, N = 512, H = 20: FP32, BF16 and FP8
    closed loops of 3 steps (the FP64 oracle takes minutes per solve here, so the
    reduced precisions are compared with the FP32 GPU path): the first solve's smoothed
    control mean and the closed-loop tracking cost."""
    if "256" in _cache:
        return _cache["256"]
    p = dataclasses.replace(wl.PRESETS["C4"], closed_loop_steps=3)
    prob = wl.make_problem(p)
    costs, first = {}, {}
    for prec in (oic.OIC_PREC_FP32, oic.OIC_PREC_BF16, oic.OIC_PREC_FP8):
        X = prob.X0.copy()
        Xs, Us = [X], []
        with oic.controller_for(prob, precision=prec) as c:
            for k in range(3):
                U, _ = c.solve(X, wl.reference_window(p, k), prob.Q, prob.R, p.N, p.H, 7000 + k)
                if k == 0:
                    first[prec] = U
                X = c.plant_step(X, U[0])
                Xs.append(X)
                Us.append(U[0])
        Xrefs = np.stack([wl.reference_at(p, k) for k in range(4)])
        costs[prec] = ocost.closed_loop_cost(np.stack(Xs), np.stack(Us), np.zeros((p.l, p.m)), Xrefs,
                                             prob.R.astype(np.float64), prob.Q.astype(np.float64))
    out = {}
    j32 = costs[oic.OIC_PREC_FP32]
    for prec, name in ((oic.OIC_PREC_BF16, "bf16"), (oic.OIC_PREC_FP8, "fp8")):
        eu = relerr(first[prec], first[oic.OIC_PREC_FP32])
        eu_max = max_relerr(first[prec], first[oic.OIC_PREC_FP32])
        rel = abs(costs[prec] - j32) / j32
        print(f"256x256 {name}: U relerr vs fp32 {eu:.2e} (max {eu_max:.2e}), cost {costs[prec]:.6e} "
              f"vs {j32:.6e} rel {rel:.2e}", flush=True)
        out[name] = (eu, eu_max, rel)
    _cache["256"] = out
    return out


@pytest.mark.slow
def test_full_size_256_bf16():
    eu, eu_max, rel = _full_size_256()["bf16"]
    assert eu < TOL_BF16 and eu_max < TOL_BF16
    assert rel < 0.02


@pytest.mark.slow
def test_full_size_256_fp8_band():
    """Regression band of the FP8 path (measured U 1.7e-1, cost 1.5e-2)."""
    eu, _, rel = _full_size_256()["fp8"]
    assert eu < 0.25
    assert rel < 0.02


@pytest.mark.slow
@pytest.mark.xfail(strict=True, reason="FP8 e4m3 misses the 2e-2 bar on U_hat at 256x256 (measured 1.7e-1)")
def test_full_size_256_fp8_meets_the_bar():
    eu, eu_max, rel = _full_size_256()["fp8"]
    assert eu < TOL_FP8_BAR_U and eu_max < TOL_FP8_BAR_U and rel < TOL_FP8_BAR_COST
