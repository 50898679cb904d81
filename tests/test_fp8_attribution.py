"""Where the FP8 rollout's error comes from, on the CPU (no GPU, no library).

An FP64 emulation of the FP8 rollout, written from the OCP FP8 e4m3 definition (bias 7,
3 mantissa bits, subnormal spacing 2^-9, largest finite 448, round to nearest even,
saturating), quantises the hidden layers of a network shaped like the 256x256 workload's
(2-64-64-64-64-1, GELU, He-normal x 0.9) the way the library's FP8 mode does: weights per
output channel with each tap's rounding error carried into the next tap of the same
kernel, activations per layer by their largest magnitude, BF16 storage between layers.
Variants switch off one source at a time, and one scales every 32-channel block of an
activation by its own power of two (the block scales the gfx950 FP8 matrix instruction
accepts).  The tests pin the emulation and record the attribution:

  * e4m3's relative rounding error is bounded by 2^-4 whatever the scale, so block scales
    cannot reduce it for values inside the normal range: the block-scaled rollout error
    stays within a small factor of the per-layer-scaled one;
  * weight and activation rounding both contribute, each at several per cent per layer,
    an order of magnitude above BF16's.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn
from paper_2410_09663_amd import workloads as wl

E4M3_MAX = 448.0


def e4m3(x):
    """Round to the nearest OCP e4m3 value (ties to even), saturating at +-448."""
    x = np.asarray(x, np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)  # below 2^-6 the spacing stays 2^-9 (subnormals)
    q = np.exp2(e - 3.0)
    r = np.round(a / q) * q  # numpy rounds halves to even
    return np.sign(x) * np.minimum(r, E4M3_MAX)


def bf16(x):
    """Round FP64 values to BF16 (via FP32, ties to even)."""
    f = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) >> 16 << 16
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def quantise_weights(W, carry=True):
    """Per-output-channel e4m3 weights (FP64 values of the codes times the scale); with
    carry, each tap's rounding error is added to the next tap of the same (o, c) kernel."""
    W = np.asarray(W, np.float64)
    out = np.empty_like(W)
    for o in range(W.shape[0]):
        s = np.max(np.abs(W[o])) / E4M3_MAX
        for c in range(W.shape[1]):
            taps = W[o, c].reshape(-1) / s
            res = np.empty(9)
            err = 0.0
            for t in range(9):
                target = taps[t] + (err if carry else 0.0)
                res[t] = e4m3(target)
                err = target - res[t]
            out[o, c] = (res * s).reshape(3, 3)
    return out


def quantise_acts(h, block=None):
    """e4m3 activations: one scale per layer (largest magnitude / 448), or per block of
    `block` channels of each pixel with a power-of-two scale."""
    if block is None:
        s = np.max(np.abs(h)) / E4M3_MAX
        return e4m3(h / s) * s
    N, C, n, m = h.shape
    hb = h.reshape(N, C // block, block, n, m)
    mx = np.max(np.abs(hb), axis=2, keepdims=True)
    s = np.exp2(np.ceil(np.log2(np.where(mx > 0, mx, 1.0) / E4M3_MAX)))
    return (e4m3(hb / s) * s).reshape(N, C, n, m)


def act(x):
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def rollout(X, U, B, weights, mode):
    """The network with the hidden layers in the given arithmetic.  mode: 'fp64', 'bf16',
    'fp8', 'fp8_w' (weights only), 'fp8_a' (activations only), 'fp8_block' (activations
    with 32-channel power-of-two block scales)."""
    h = np.concatenate([X[:, None], (B @ U)[:, None]], axis=1)
    L = len(weights)
    for k, W in enumerate(weights):
        W = np.asarray(W, np.float64)
        if 0 < k < L - 1 and mode != "fp64":
            if mode == "bf16":
                Wq, hq = bf16(W), h
            else:
                Wq = W if mode == "fp8_a" else quantise_weights(W)
                if mode == "fp8_w":
                    hq = h
                else:
                    hq = quantise_acts(h, 32 if mode == "fp8_block" else None)
            h = ocnn.conv3x3(hq, Wq)
        else:
            h = ocnn.conv3x3(h, W)
        if k < L - 1:
            h = act(h)
            if mode != "fp64":
                h = bf16(h)  # BF16 storage between layers
    return h[:, 0]


@pytest.fixture(scope="module")
def net():
    p = wl.small_preset(n=20, m=20, l=5, channels=(2, 64, 64, 64, 64, 1), activation=wl.ACT_GELU, N=2)
    prob = wl.make_problem(p)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((2, p.n, p.m))
    U = 0.3 * rng.standard_normal((2, p.l, p.m))
    ref = rollout(X, U, prob.B.astype(np.float64), prob.weights, "fp64")
    return p, prob, X, U, ref


def test_e4m3_rounding_matches_the_format():
    # exact codes, the largest finite value, saturation, subnormal spacing, ties to even
    assert e4m3(448.0) == 448.0 and e4m3(1e6) == 448.0 and e4m3(-500.0) == -448.0
    assert e4m3(1.0) == 1.0 and e4m3(1.0625) == 1.0 and e4m3(1.1875) == 1.25  # spacing 1/8 in [1, 2)
    assert e4m3(2.0 ** -9) == 2.0 ** -9 and e4m3(3 * 2.0 ** -10) == 2.0 ** -8  # tie -> even code
    assert e4m3(2.0 ** -10) == 0.0  # half the smallest subnormal: tie to even (zero)
    x = np.random.default_rng(0).uniform(2.0 ** -6, 448, 10000)
    assert np.max(np.abs(e4m3(x) - x) / x) <= 2.0 ** -4 + 1e-12


def test_weight_quantisation_with_carry_keeps_kernel_sums():
    W = np.random.default_rng(1).standard_normal((4, 3, 3, 3))
    Wq = quantise_weights(W)
    s = np.max(np.abs(W.reshape(4, -1)), axis=1) / E4M3_MAX
    # the sum over a kernel's taps differs from the exact one by at most the last rounding
    d = np.abs(Wq.sum(axis=(2, 3)) - W.sum(axis=(2, 3)))
    assert np.all(d <= (2.0 ** -4) * (s[:, None] * E4M3_MAX) + 1e-12)


def test_fp8_error_attribution(net):
    p, prob, X, U, ref = net
    B = prob.B.astype(np.float64)
    err = {}
    for mode in ("bf16", "fp8", "fp8_w", "fp8_a", "fp8_block"):
        got = rollout(X, U, B, prob.weights, mode)
        err[mode] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("rollout relerr vs FP64: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    # FP8 is an order of magnitude above BF16, and each source contributes
    assert err["fp8"] > 5 * err["bf16"]
    assert err["fp8_w"] > 0.2 * err["fp8"] and err["fp8_a"] > 0.2 * err["fp8"]
    # power-of-two block scales do not remove the 3-bit mantissa's rounding error
    assert err["fp8_block"] > 0.5 * err["fp8"]
