"""Error measures shared by the GPU parity tests.

Every parity check is made twice, on the same pair of arrays:
  * normwise:     ||got - ref||_F / ||ref||_F;
  * element-wise: max_e |got_e - ref_e| / max_e |ref_e|,
so that one wrong entry (an edge tile, a member column) cannot hide inside a norm
over thousands of correct ones.  Both must be within the stated tolerance.
"""
import numpy as np


def relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def assert_parity(got, ref, tol, what=""):
    """Assert both error measures are within tol; return (normwise, element-wise)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    e, emax = relerr(got, ref), max_relerr(got, ref)
    assert e < tol and emax < tol, f"{what}: normwise {e:.3e}, element-wise {emax:.3e}, tolerance {tol:.1e}"
    return e, emax
