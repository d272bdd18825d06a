"""Philox4x32-10 counter-based generator, uniforms and normals (FP64).

The paper leaves the random-number generator unspecified (section 2.6,
white noise drawn from N(0, sigma); Timmer-Koenig pink noise).  This
project fixes it so that a noise realisation is reproducible from its key
alone: Philox4x32-10 of Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11), written here from that definition.

  key      (seed mod 2^32, seed >> 32)
  counter  (c0, c1, c2, c3) = (time or frequency index, channel, pixel,
           stream) with stream 0 = white noise, 1 = pink noise
  uniform  u = ((o >> 9) + 1/2) * 2^-23, exact in FP32 and FP64, in (0, 1)
  normal   Box-Muller: r = sqrt(-2 ln u0); z = r cos(2 pi u1)
           (pink noise also takes r sin(2 pi u1) as the imaginary part)

Oracle -- test infrastructure only.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# multipliers and Weyl key increments of Philox4x32 (Salmon et al. 2011)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def key_of(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def philox4x32_10(c0, c1, c2, c3, key):
    """Ten Philox rounds on counters (arrays of equal shape, values < 2^32)
    under key (k0, k1).  Returns the four 32-bit output words as uint32
    arrays.

    One round: the products M0*x0 and M1*x2 are split into high and low
    words; the new state is (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2),
    hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)).  The key advances by the Weyl
    increments between rounds."""
    x0 = np.asarray(c0, dtype=np.uint64) & MASK32
    x1 = np.asarray(c1, dtype=np.uint64) & MASK32
    x2 = np.asarray(c2, dtype=np.uint64) & MASK32
    x3 = np.asarray(c3, dtype=np.uint64) & MASK32
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = np.uint64(key[0]) & MASK32
    k1 = np.uint64(key[1]) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return (x0.astype(np.uint32), x1.astype(np.uint32),
            x2.astype(np.uint32), x3.astype(np.uint32))


def to_uniform(o):
    """23 high bits mapped to the open interval: ((o >> 9) + 0.5) * 2^-23."""
    o = np.asarray(o, dtype=np.uint32)
    return ((o >> np.uint32(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def box_muller(o0, o1):
    """(r cos(2 pi u1), r sin(2 pi u1)) with r = sqrt(-2 ln u0)."""
    u0 = to_uniform(o0)
    u1 = to_uniform(o1)
    r = np.sqrt(-2.0 * np.log(u0))
    ang = 2.0 * np.pi * u1
    return r * np.cos(ang), r * np.sin(ang)


def white_normal(seed, n, k, p):
    """Standard normal for detector sample (time n, channel k, pixel p)."""
    o = philox4x32_10(n, k, p, 0, key_of(seed))
    return box_muller(o[0], o[1])[0]


def pink_normals(seed, j, k, p):
    """(z_re, z_im) for frequency index j of series (pixel p, channel k)."""
    o = philox4x32_10(j, k, p, 1, key_of(seed))
    return box_muller(o[0], o[1])
