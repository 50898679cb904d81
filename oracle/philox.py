"""Philox4x32-10 counter-based generator and the normals the seeded solve draws.

Generator: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as
1, 2, 3" (SC'11).  A 128-bit counter (four 32-bit words) and a 64-bit key (two
words) go through ten rounds; each round multiplies words 0 and 2 by the
constants 0xD2511F53 and 0xCD9E8D57, keeps the 64-bit products' high and low
halves, and mixes the high halves with words 1 and 3 and the round key.  The key
advances by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.

Normals (the noise of Eqs. (12) and (15b)): for element index e of noise kind
``kind``, the counter is (e mod 2^32, e div 2^32, kind, 0) and the key is
(seed mod 2^32, seed div 2^32).  The output words w0..w3 give two 53-bit
uniforms, u1 = (((w1:w0) >> 11) + 1) 2^-53 in (0, 1] and
u2 = ((w3:w2) >> 11) 2^-53 in [0, 1); the normal is the Box-Muller cosine
branch sqrt(-2 ln u1) cos(2 pi u2), computed in FP64 and rounded to FP32.

Noise kinds and element order, for a solve with N members and horizon H:
kind 0 = initial control spread, shape (N, l, m);
kind 1 = process noise W_t,  kind 2 = V_X,t,  kind 3 = V_U,t, each (H, N, rows, m)
with rows l, n, l; e is the C-order linear index in that shape.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

KIND_INIT = 0
KIND_W = 1
KIND_VX = 2
KIND_VU = 3


def philox4x32_10_scalar(ctr, key):
    """Reference form on Python ints: ctr is 4 words, key is 2 words."""
    x0, x1, x2, x3 = (int(c) & MASK32 for c in ctr)
    k0, k1 = (int(k) & MASK32 for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised form: arrays of counter words (any broadcastable shape) as uint64."""
    x0 = np.asarray(c0, dtype=np.uint64) & np.uint64(MASK32)
    x1 = np.asarray(c1, dtype=np.uint64) & np.uint64(MASK32)
    x2 = np.asarray(c2, dtype=np.uint64) & np.uint64(MASK32)
    x3 = np.asarray(c3, dtype=np.uint64) & np.uint64(MASK32)
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    x0, x1, x2, x3 = (a.copy() for a in (x0, x1, x2, x3))
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m32 = np.uint64(MASK32)
    s32 = np.uint64(32)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = np.uint64(M0) * x0
        p1 = np.uint64(M1) * x2
        hi0, lo0 = p0 >> s32, p0 & m32
        hi1, lo1 = p1 >> s32, p1 & m32
        x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0
    return x0, x1, x2, x3


def normals(seed: int, kind: int, shape) -> np.ndarray:
    """The FP32 standard normals of one noise kind, in C order of `shape`."""
    count = int(np.prod(shape))
    e = np.arange(count, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    w0, w1, w2, w3 = philox4x32_10(e & np.uint64(MASK32), e >> np.uint64(32),
                                   np.uint64(kind), np.uint64(0),
                                   seed & MASK32, seed >> 32)
    s32 = np.uint64(32)
    s11 = np.uint64(11)
    a = ((w1 << s32) | w0) >> s11
    b = ((w3 << s32) | w2) >> s11
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.astype(np.float32).reshape(shape)


def solve_noise(seed: int, n: int, m: int, l: int, N: int, H: int):
    """The four noise arrays a seeded solve draws: (Z_init, Z_W, Z_VX, Z_VU)."""
    return (normals(seed, KIND_INIT, (N, l, m)),
            normals(seed, KIND_W, (H, N, l, m)),
            normals(seed, KIND_VX, (H, N, n, m)),
            normals(seed, KIND_VU, (H, N, l, m)))
