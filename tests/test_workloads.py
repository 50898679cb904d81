"""Checks on the seeded synthetic inputs (shapes, statistics, determinism)."""
import math

import numpy as np

from paper_2410_09663_amd import workloads as wl


def test_grf_correlation_and_variance():
    ell = 4.0
    acc = {1: [], 2: [], 4: []}
    for s in range(6):
        f = wl.gaussian_random_field(96, 96, ell, seed=s).astype(np.float64)
        assert abs(f.std() - 1) < 1e-5 and abs(f.mean()) < 1e-5
        c = f[16:-16, 16:-16]
        for d in acc:
            acc[d].append(np.mean(c[:, :-d] * c[:, d:]) / np.mean(c * c))
    for d, v in acc.items():
        assert abs(np.mean(v) - math.exp(-d * d / (2 * ell * ell))) < 0.08, (d, np.mean(v))


def test_he_init_and_lift_statistics():
    ws = wl.he_weights([2, 64, 64, 1], seed=1)
    assert [w.shape for w in ws] == [(64, 2, 3, 3), (64, 64, 3, 3), (1, 64, 3, 3)]
    w = ws[1].astype(np.float64)
    assert abs(w.std() - 0.9 * math.sqrt(2 / (9 * 64))) < 0.03 * w.std()
    B = wl.lift_matrix(256, 64, 0).astype(np.float64)
    assert abs(B.std() - 0.5) < 0.01
    assert all(w.dtype == np.float32 for w in ws)


def test_bump_reference():
    p = wl.PRESETS["C1"]
    r = wl.reference_at(p, 0)
    assert r.shape == (16, 16)
    assert abs(r.max() - math.exp(-0.25 / 9)) < 1e-6  # centre (7.5, 7.5) falls between cells
    p2 = wl.PRESETS["C2"]
    a, b = wl.reference_at(p2, 0), wl.reference_at(p2, 1)
    assert np.allclose(np.roll(a, 1, axis=1)[:, 1:-1], b[:, 1:-1], atol=1e-6)  # drifts one column


def test_noise_is_deterministic():
    a = wl.host_noise(4, 5, 2, 3, 2, seed=7)
    b = wl.host_noise(4, 5, 2, 3, 2, seed=7)
    assert np.array_equal(a.Z_VX, b.Z_VX) and a.Z_W.shape == (2, 3, 2, 5)
