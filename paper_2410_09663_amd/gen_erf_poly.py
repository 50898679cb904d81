"""Coefficients of the polynomial erf used by the BF16 / FP8 rollout kernels' GELU.

erf(z) on [0, ZMAX] is fitted by z (c0 + c1 z + ... + c8 z^8) with iteratively reweighted
least squares on Chebyshev nodes (weights grow where the residual is large, which moves
the fit toward the minimax one); beyond ZMAX the kernels take erf = 1 (1 - erf(3.5) =
7.4e-7).  Prints the coefficients as C++ float literals and the maximum absolute error on
a fine grid (4.2e-5, well below BF16's rounding of the activations, 2^-9 relative).

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


def main():
    c = fit().astype(np.float32)
    zz = np.linspace(0.0, ZMAX, 400001)
    p = zz * np.polyval(c[::-1].astype(np.float64), zz)
    print(f"// max |p(z) - erf(z)| on [0, {ZMAX}]: {np.max(np.abs(p - erf(zz))):.2e}")
    print("constexpr float kErfPoly[%d] = {%s};" % (DEG, ", ".join(f"{v:.9e}f" for v in c)))


if __name__ == "__main__":
    main()
