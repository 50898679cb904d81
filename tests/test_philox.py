"""Pins for the oracle's counter-based generator: published known-answer vectors and moments."""
import os

import numpy as np
import pytest

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(v, 16) for v in line.split()]
        rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_known_answer_vectors_scalar():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(philox.philox4x32_10_scalar(ctr, key)) == out


def test_known_answer_vectors_vectorised():
    for ctr, key, out in _kat():
        got = philox.philox4x32_10(*[np.array([c], dtype=np.uint64) for c in ctr], key[0], key[1])
        assert [int(g[0]) for g in got] == out


def test_vectorised_equals_scalar_on_many_counters():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2 ** 32, size=(4, 50), dtype=np.uint64)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    got = philox.philox4x32_10(c[0], c[1], c[2], c[3], k0, k1)
    for j in range(50):
        ref = philox.philox4x32_10_scalar([int(v) for v in c[:, j]], (k0, k1))
        assert [int(g[j]) for g in got] == list(ref)


def test_normals_element_order_and_counter():
    """Element e of kind k uses counter (e lo, e hi, k, 0) and key (seed lo, seed hi)."""
    seed = (7 << 32) | 99
    z = philox.normals(seed, 2, (3, 4, 5))
    for e in [0, 1, 17, 59]:
        w = philox.philox4x32_10_scalar((e, 0, 2, 0), (99, 7))
        a = (((w[1] << 32) | w[0]) >> 11)
        b = (((w[3] << 32) | w[2]) >> 11)
        u1 = (a + 1) * 2.0 ** -53
        u2 = b * 2.0 ** -53
        ref = np.float32(np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2))
        assert z.reshape(-1)[e] == ref


def test_normal_moments():
    z = philox.normals(2024, 1, (1 << 20,)).astype(np.float64)
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(z ** 3)) < 5 * np.sqrt(15 / n)
    assert abs(np.mean(z ** 4) - 3) < 5 * np.sqrt(96 / n)
    # kinds and seeds give different streams
    assert not np.array_equal(philox.normals(2024, 0, (64,)), philox.normals(2024, 1, (64,)))
    assert not np.array_equal(philox.normals(1, 0, (64,)), philox.normals(2, 0, (64,)))
