"""Seeded synthetic inputs for the Kalman-MPC solve.

This module only draws inputs: the CNN weights, the lift matrix B, the initial
field, the reference fields and the standard-normal noise arrays.  It holds
none of the smoother's arithmetic, so both the FP64 oracle and the HIP library
can be fed from it without sharing any part of the method.

The paper's workload (a trained CNN surrogate of 2-D Burgers' flow, section
"Numerical Experiments") is not available, so every preset below is synthetic:
a He-initialised conv3x3 CNN scaled by 0.9, a Gaussian random field as the
initial state, and Gaussian-bump references.  All draws use
``numpy.random.default_rng(seed)`` with ``standard_normal`` in C order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ACT_TANH = 0
ACT_GELU = 1

PREC_FP32 = 0
PREC_BF16 = 1
PREC_FP8 = 2


@dataclasses.dataclass
class Preset:
    """One synthetic workload.  Sizes: state n x m, control l x m."""

    name: str
    n: int
    m: int
    l: int
    channels: List[int]  # [2, c1, ..., 1]
    activation: int
    N: int
    H: int
    q: float  # Q = q * I (l x l)
    r: float  # R = r * I (n x n)
    grf_length: float
    ref_kind: str  # "bump", "moving", "twobump"
    ref_sigma: float
    ref_center: tuple  # (row, col) of the (first) bump at absolute time 0
    closed_loop_steps: int = 1
    precision: int = PREC_FP32
    seed_B: int = 0
    seed_W: int = 1
    seed_X0: int = 2
    noise_seed_base: int = 1000

    @property
    def n_layers(self) -> int:
        return len(self.channels) - 1


PRESETS = {
    # 16x16 field, one solve; small enough for the FP64 oracle in well under a second.
    "C1": Preset("C1", 16, 16, 4, [2, 8, 1], ACT_TANH, 32, 5, 0.1, 0.01, 3.0,
                 "bump", 3.0, (7.5, 7.5), closed_loop_steps=1, noise_seed_base=3),
    # 64x64 field, N=128, H=10, 20 closed-loop steps, moving bump reference.
    "C2": Preset("C2", 64, 64, 8, [2, 16, 16, 1], ACT_TANH, 128, 10, 0.1, 0.01, 6.0,
                 "moving", 6.0, (32.0, 16.0), closed_loop_steps=20),
    # 128x128 field, GELU CNN, N=256, H=10, 50 closed-loop steps.
    "C3": Preset("C3", 128, 128, 32, [2, 32, 32, 32, 1], ACT_GELU, 256, 10, 0.05, 0.005, 8.0,
                 "moving", 8.0, (64.0, 32.0), closed_loop_steps=50, precision=PREC_BF16),
    # 256x256 field, 5-layer GELU CNN, N=512, H=20, two-bump reference.
    "C4": Preset("C4", 256, 256, 64, [2, 64, 64, 64, 64, 1], ACT_GELU, 512, 20, 0.05, 0.005, 12.0,
                 "twobump", 12.0, (256 / 3.0, 256 / 3.0), closed_loop_steps=50, precision=PREC_FP8),
}


# Serving mix: per controller a grid side from SERVE_GRIDS, l = side/4, N and H drawn
# from the lists below, and the CNN of matching size.
SERVE_GRIDS = (32, 64, 128, 256)
SERVE_N = (64, 128, 256)
SERVE_H = (5, 10, 20)
SERVE_CNN = {32: ([2, 16, 16, 1], ACT_TANH), 64: ([2, 16, 16, 1], ACT_TANH),
             128: ([2, 32, 32, 32, 1], ACT_GELU), 256: ([2, 64, 64, 64, 64, 1], ACT_GELU)}


def serving_mix(count: int, seed: int = 7, precision: int = PREC_BF16) -> List[Preset]:
    """`count` independent controllers drawn uniformly from the serving mix, each with its
    own seeds for B, the weights and X0; GRF length and bump width 0.75 sqrt(n), the bump
    drifting one column per step from (n/2, m/4); Q = 0.05 I, R = 0.005 I."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        g = int(rng.choice(SERVE_GRIDS))
        N = int(rng.choice(SERVE_N))
        H = int(rng.choice(SERVE_H))
        ch, act = SERVE_CNN[g]
        ell = 0.75 * math.sqrt(g)
        out.append(Preset(f"serve{c}", g, g, g // 4, list(ch), act, N, H, 0.05, 0.005, ell, "moving",
                          ell, (g / 2.0, g / 4.0), closed_loop_steps=1, precision=precision,
                          seed_B=10 * c + 100, seed_W=10 * c + 101, seed_X0=10 * c + 102,
                          noise_seed_base=10 * c + 103))
    return out


def small_preset(n=8, m=8, l=2, channels=(2, 4, 1), activation=ACT_TANH, N=16, H=3,
                 q=0.1, r=0.01, name="tiny") -> Preset:
    """A hand-sized preset for unit tests (ragged sizes allowed)."""
    return Preset(name, n, m, l, list(channels), activation, N, H, q, r, max(1.0, n / 5),
                  "bump", max(1.0, n / 5), ((n - 1) / 2, (m - 1) / 2))


def he_weights(channels: Sequence[int], seed: int, gain: float = 0.9) -> List[np.ndarray]:
    """He-normal conv3x3 weights, OIHW, std sqrt(2 / (9 C_in)) times `gain`, float32."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        w = rng.standard_normal((cout, cin, 3, 3)) * math.sqrt(2.0 / (9.0 * cin)) * gain
        out.append(w.astype(np.float32))
    return out


def lift_matrix(n: int, l: int, seed: int) -> np.ndarray:
    """B in R^{n x l} with entries N(0, 1/4), float32."""
    rng = np.random.default_rng(seed)
    return (0.5 * rng.standard_normal((n, l))).astype(np.float32)


def gaussian_random_field(n: int, m: int, length: float, seed: int) -> np.ndarray:
    """White noise smoothed by a Gaussian of std length/sqrt(2) (zero padding), so that the
    correlation at lag d is close to exp(-d^2 / (2 length^2)); standardised to zero mean and
    unit sample std; float32."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, m))
    f = gaussian_filter(w, sigma=length / math.sqrt(2.0), mode="constant", cval=0.0)
    f = f - f.mean()
    f = f / f.std()
    return f.astype(np.float32)


def bump(n: int, m: int, center, sigma: float, amplitude: float = 1.0) -> np.ndarray:
    y = np.arange(n, dtype=np.float64)[:, None]
    x = np.arange(m, dtype=np.float64)[None, :]
    cy, cx = center
    return amplitude * np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2.0 * sigma ** 2))


def reference_at(p: Preset, t: int) -> np.ndarray:
    """X^ref at absolute time t (float32, n x m)."""
    if p.ref_kind == "bump":
        f = bump(p.n, p.m, p.ref_center, p.ref_sigma)
    elif p.ref_kind == "moving":
        cy, cx = p.ref_center
        f = bump(p.n, p.m, (cy, cx + t), p.ref_sigma)
    elif p.ref_kind == "twobump":
        f = bump(p.n, p.m, (p.n / 3.0, p.m / 3.0), p.ref_sigma) + \
            bump(p.n, p.m, (2.0 * p.n / 3.0, 2.0 * p.m / 3.0), p.ref_sigma)
    else:
        raise ValueError(p.ref_kind)
    return f.astype(np.float32)


def reference_window(p: Preset, k: int, H: Optional[int] = None) -> np.ndarray:
    """X^ref_t for t = k..k+H, shape (H+1, n, m), float32."""
    H = p.H if H is None else H
    return np.stack([reference_at(p, k + s) for s in range(H + 1)]).astype(np.float32)


@dataclasses.dataclass
class Noise:
    """Standard normals, float32, member-major:
    Z_init (N, l, m); Z_W (H, N, l, m); Z_VX (H, N, n, m); Z_VU (H, N, l, m).
    Index t-1 of the H-long arrays belongs to horizon step t = 1..H."""

    Z_init: np.ndarray
    Z_W: np.ndarray
    Z_VX: np.ndarray
    Z_VU: np.ndarray


def host_noise(n: int, m: int, l: int, N: int, H: int, seed: int) -> Noise:
    rng = np.random.default_rng(seed)
    f = np.float32
    z0 = rng.standard_normal((N, l, m)).astype(f)
    zw = rng.standard_normal((H, N, l, m)).astype(f)
    zx = rng.standard_normal((H, N, n, m)).astype(f)
    zu = rng.standard_normal((H, N, l, m)).astype(f)
    return Noise(z0, zw, zx, zu)


@dataclasses.dataclass
class Problem:
    """Everything one solve needs, as float32 arrays."""

    preset: Preset
    B: np.ndarray
    weights: List[np.ndarray]
    X0: np.ndarray
    Q: np.ndarray
    R: np.ndarray


def make_problem(p: Preset) -> Problem:
    B = lift_matrix(p.n, p.l, p.seed_B)
    W = he_weights(p.channels, p.seed_W)
    X0 = gaussian_random_field(p.n, p.m, p.grf_length, p.seed_X0)
    Q = (p.q * np.eye(p.l)).astype(np.float32)
    R = (p.r * np.eye(p.n)).astype(np.float32)
    return Problem(p, B, W, X0, Q, R)


def random_spd(k: int, seed: int, scale: float = 0.1, cond: float = 4.0) -> np.ndarray:
    """A seeded dense SPD matrix with eigenvalues spread over [scale, scale*cond], float32."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    ev = scale * np.exp(np.linspace(0.0, math.log(cond), k))
    a = (q * ev) @ q.T
    a = 0.5 * (a + a.T)
    return a.astype(np.float32)
