"""Host-side checks of the benchmark's accounting: algorithmic FLOPs and bytes per
kernel class, the roofline classification, and the one-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2410_09663_amd import workloads as wl  # noqa: E402


def test_hidden_layer_work_is_the_convolution_count():
    p = wl.PRESETS["C2"]
    work = bench.algorithmic_work(p, p.H, "fp32")
    f, b = work["conv_mid"]
    px = p.n * p.m * p.N
    # one 16 -> 16 hidden layer per horizon step: 9 taps x cin x cout multiply-adds per pixel,
    # FP32 activations read once and written once
    assert f == pytest.approx(p.H * 2.0 * 9 * 16 * 16 * px)
    assert b == pytest.approx(p.H * 4.0 * (16 + 16) * px)
    # BF16 activations halve the bytes, not the FLOPs
    fb, bb = bench.algorithmic_work(p, p.H, "bf16")["conv_mid"]
    assert fb == pytest.approx(f) and bb == pytest.approx(b / 2)


def test_folded_last_layer_keeps_the_network_flops():
    """With the last layer folded into the last hidden layer's epilogue (FP32, 64-channel
    hidden layers) the conv FLOPs per step are the network's, and the last layer's class
    moves the nine FP32 tap planes and the state instead of the activations."""
    p = wl.PRESETS["C4"]
    assert all(bench.last_layer_folded(p, prec) for prec in ("fp32", "bf16", "fp8"))
    assert not bench.last_layer_folded(wl.PRESETS["C3"], "fp32")  # 32 -> 32 last hidden layer
    px = p.n * p.m * p.N
    ch = p.channels
    net = sum(2.0 * 9 * a * b * px for a, b in zip(ch[:-1], ch[1:]))
    for prec in ("fp32", "bf16", "fp8"):
        work = bench.algorithmic_work(p, 1, prec)
        conv = sum(work[c][0] for c in ("conv_first", "conv_mid")) + (
            0.0 if bench.last_layer_folded(p, prec) else work["conv_last"][0])
        assert conv == pytest.approx(net)
    f, b = bench.algorithmic_work(p, 1, "fp32")["conv_last"]
    assert b == pytest.approx(4.0 * 10 * px)


def test_precomputed_lift_moves_its_bytes_and_flops():
    """A 64-channel first layer reads X and the precomputed lift channel B U; the lift
    class reads U and writes B U and does the l multiply-adds per pixel.  Narrower first
    layers form the lift themselves and read X and U."""
    p = wl.PRESETS["C4"]
    px = p.n * p.m * p.N
    work = bench.algorithmic_work(p, 1, "fp32")
    f, b = work["lift"]
    assert f == pytest.approx(2.0 * p.l * px)
    assert b == pytest.approx(4.0 * (p.l * p.m * p.N + px))
    _, bf = work["conv_first"]
    assert bf == pytest.approx(4.0 * 2 * px + 4.0 * 64 * px)
    q = wl.PRESETS["C2"]
    work = bench.algorithmic_work(q, 1, "fp32")
    assert "lift" not in work
    _, bq = work["conv_first"]
    assert bq == pytest.approx(4.0 * (q.n + q.l) * q.m * q.N + 4.0 * 16 * q.n * q.m * q.N)


def test_statistics_peak_lies_between_the_two_matrix_core_peaks():
    p = wl.PRESETS["C2"]
    for prec, lo, hi in (("fp32", bench.PEAK["fp64"], bench.PEAK["fp32"]),
                         ("bf16", bench.PEAK["fp32"], bench.PEAK["fp32"])):
        work = bench.algorithmic_work(p, p.H, prec)
        f, _ = work["stats"]
        t, _ = work["stats_t_peak"]
        eff = f / t
        assert lo * (1 - 1e-12) <= eff <= hi * (1 + 1e-12), (prec, eff)
    # in the FP32 mode the FP64 share is Sigma^Y's p x p block against Sigma^{XY}'s Ma x p
    work = bench.algorithmic_work(p, p.H, "fp32")
    f, _ = work["stats"]
    t, _ = work["stats_t_peak"]
    assert bench.PEAK["fp64"] < f / t < bench.PEAK["fp32"]


def test_roofline_classification():
    # 1 GFLOP and 1 GB in 1 ms: bytes take longer at peak, so the launch is HBM-bound
    r = bench.roofline_for("update", 1e9, 1e9, 1.0, 10, "fp32")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1e9 / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["avg_launch_us"] == pytest.approx(100.0)
    # 1 TFLOP and 1 MB: the matrix cores bound it, against the FP32 peak
    r = bench.roofline_for("conv_mid", 1e12, 1e6, 10.0, 1, "fp32")
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(157.3)
    # an explicit time at peak overrides the class's peak
    r = bench.roofline_for("stats", 1e12, 1e6, 10.0, 1, "fp32", None, 1e12 / 100e12)
    assert r["peak"] == pytest.approx(100.0)


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode != 0
    assert "one GPU" in res.stdout + res.stderr
