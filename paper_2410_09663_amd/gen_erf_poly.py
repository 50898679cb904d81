"""Coefficients of the polynomial GELU used by the BF16 / FP8 rollout kernels.

erf(z) on [0, ZMAX] is fitted by z (c0 + c1 z + ... + c8 z^8) with iteratively reweighted
least squares on Chebyshev nodes (weights grow where the residual is large, which moves
the fit toward the minimax one); beyond ZMAX the kernels take erf = 1 (1 - erf(3.5) =
7.4e-7).  The kernels evaluate GELU(x) = x/2 + |x| erf(|x|/sqrt2)/2 (erf is odd) with the
argument scaling and the factor 1/2 folded into the coefficients:

    a = min(|x|, ZMAX sqrt2),  GELU(x) = fma(|x| a, Q(a), x/2),
    Q(a) = sum_k q_k a^k,  q_k = c_k / (2 sqrt2^(k+1)),

twelve instructions per value and no transcendental ones.  Prints q as C++ float literals,
the maximum absolute error of the erf fit on a fine grid (4.9e-5, well below BF16's
rounding of the activations, 2^-9 relative) and that of the GELU evaluated in FP32 on
[-10, 10] (3.5e-4, at |x| = 10: |x|/2 times the erf error plus the FP32 rounding of the
Horner sum, 3.5e-5 relative).

Usage: python -m paper_2410_09663_amd.gen_erf_poly
"""
import numpy as np
from scipy.special import erf

ZMAX = 3.5
DEG = 9


def fit():
    z = np.cos(np.linspace(0.0, np.pi, 6000)) * ZMAX / 2 + ZMAX / 2
    A = np.stack([z ** (k + 1) for k in range(DEG)], axis=1)
    w = np.ones_like(z)
    c = None
    for _ in range(30):
        c, *_ = np.linalg.lstsq(A * w[:, None], erf(z) * w, rcond=None)
        r = np.abs(A @ c - erf(z))
        w = w * (1.0 + 5.0 * r / np.max(r))
    return c


def gelu_coefficients(c):
    return np.array([c[k] / (2.0 * np.sqrt(2.0) ** (k + 1)) for k in range(DEG)]).astype(np.float32)


def gelu_fp32(x, q):
    """The kernels' evaluation, operation by operation in FP32."""
    x = np.asarray(x, np.float32)
    a = np.abs(x)
    ac = np.minimum(a, np.float32(ZMAX * np.sqrt(2.0)))
    p = np.full_like(x, q[-1])
    for k in range(DEG - 2, -1, -1):
        p = (p * ac + q[k]).astype(np.float32)
    return ((a * ac).astype(np.float32) * p + np.float32(0.5) * x).astype(np.float32)


def main():
    c = fit().astype(np.float32)
    zz = np.linspace(0.0, ZMAX, 400001)
    p = zz * np.polyval(c[::-1].astype(np.float64), zz)
    q = gelu_coefficients(c.astype(np.float64))
    xx = np.linspace(-10.0, 10.0, 800001)
    exact = 0.5 * xx * (1.0 + erf(xx / np.sqrt(2.0)))
    print(f"// max |p(z) - erf(z)| on [0, {ZMAX}]: {np.max(np.abs(p - erf(zz))):.2e}")
    print(f"// max |GELU_fp32(x) - GELU(x)| on [-10, 10]: {np.max(np.abs(gelu_fp32(xx, q) - exact)):.2e}")
    print("constexpr float kGeluPoly[%d] = {%s};" % (DEG, ", ".join(f"{v:.9e}f" for v in q)))


if __name__ == "__main__":
    main()
