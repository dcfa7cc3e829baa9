"""Philox-4x32-10 counter-based random number generator, written from its published
definition (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): ten rounds of two 32x32->64 multiplications with the constants 0xD2511F53 and
0xCD9E8D57, a Weyl key schedule with increments 0x9E3779B9 and 0xBB67AE85.

The method draws two kinds of random numbers, both fixed functions of (seed, counter) so
that a run can be replayed and the noise "treated as an input" of the differentiable model
(Sec. 2.4.2):
  * white noise for the Gaussian initial field: one normal per cell by Box-Muller;
  * one uniform u in (0,1) per cell and step for the star-formation draw, giving the
    logistic difference g0 - g1 = ln u - ln(1-u) of two Gumbel(0,1) variables.
Counter layout (word 0..3): (cell index, step, stream tag, 0); key = (seed low, seed high).
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)

TAG_WHITE = 0x574E0000      # stream tag for the white-noise field
TAG_STARFORM = 0x53460000   # stream tag for the star-formation uniforms


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox-4x32-10.  Counters are uint32-valued arrays (broadcast together),
    keys are python ints.  Returns four uint32 arrays."""
    c0, c1, c2, c3 = [np.asarray(c, dtype=np.uint64) & MASK for c in (c0, c1, c2, c3)]
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(k0 & 0xFFFFFFFF)
    k1 = np.uint64(k1 & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0          # exact: both factors < 2^32
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniform_open(bits):
    """Map 32 random bits to u in (0,1): the top 24 bits plus one half, times 2^-24.
    Every value is exactly representable in float32 and float64."""
    b = np.asarray(bits, dtype=np.uint64) >> np.uint64(8)
    return (b.astype(np.float64) + 0.5) * (1.0 / 16777216.0)


def white_noise(seed, n):
    """Unit normal per cell of an n^3 grid, indexed [z, y, x] (x fastest)."""
    idx = np.arange(n ** 3, dtype=np.uint64)
    r0, r1, _, _ = philox4x32_10(idx, 0, TAG_WHITE, 0, seed & 0xFFFFFFFF, seed >> 32)
    u1 = uniform_open(r0)
    u2 = uniform_open(r1)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.reshape(n, n, n)


def starform_uniform(seed, step, n):
    """Uniform u in (0,1) per cell for the star-formation draw of a given step."""
    idx = np.arange(n ** 3, dtype=np.uint64)
    r0, _, _, _ = philox4x32_10(idx, step, TAG_STARFORM, 0, seed & 0xFFFFFFFF, seed >> 32)
    return uniform_open(r0).reshape(n, n, n)
