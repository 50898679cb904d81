"""The BF16/FP8 rollouts' GELU constants (CPU only): the table compiled into the kernels is
the one the committed generator writes, and the kernels' operation order, emulated in FP32,
stays within the fit's bound of the exact erf-form GELU."""
import os
import re

import numpy as np
from scipy.special import erf

from paper_2410_09663_amd import gen_erf_poly as gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_table():
    src = open(os.path.join(ROOT, "paper_2410_09663_amd", "csrc", "rollout.hip")).read()
    body = re.search(r"kGeluPoly\[9\]\s*=\s*\{([^}]*)\}", src).group(1)
    return np.array([float(v.strip().rstrip("f")) for v in body.split(",")], np.float32)


def test_kernel_table_is_the_generators():
    c = gen.fit().astype(np.float32)
    q = gen.gelu_coefficients(c.astype(np.float64))
    assert np.array_equal(kernel_table(), q)


def test_folded_form_matches_exact_gelu():
    q = kernel_table()
    x = np.linspace(-10.0, 10.0, 400001)
    exact = 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))
    got = gen.gelu_fp32(x, q).astype(np.float64)
    # |x|/2 times the erf fit's error (< 5e-5), plus the FP32 rounding of the Horner sum, whose
    # terms reach about 40 before cancelling (|x| a times a few 1e-6): 3.5e-4 at |x| = 10,
    # 3.5e-5 relative, far below BF16's 2^-9 rounding of the stored value
    assert np.all(np.abs(got - exact) <= 4e-5 * np.abs(x) + 2e-6)
    # odd-erf identity used by the folded form: GELU(x) - GELU(-x) = x
    assert np.max(np.abs(gen.gelu_fp32(x, q) - gen.gelu_fp32(-x, q) - x.astype(np.float32))) < 1e-5 * 10
