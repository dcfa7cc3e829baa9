"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Random fields only: this module holds none of the method's arithmetic.  Every function
returns numpy float32 arrays (exactly representable in float64, so the FP64 oracle and the
FP32 GPU path start from identical values)."""

import math

import numpy as np


def white_noise(n, seed):
    """Unit normal per cell, (n, n, n) indexed [z, y, x]."""
    return np.random.default_rng(seed).standard_normal((n, n, n)).astype(np.float32)


def smooth_gas_state(n, a, seed, amp=0.2, speed=0.5, energy=0.8):
    """A positive, smooth-plus-noise gas state Q = (rho, a rho U, a^2 rho E) of shape
    (5, n, n, n): density around 1, velocities of order `speed`, specific internal energy
    around `energy` (code units)."""
    rng = np.random.default_rng(seed)
    r = np.arange(n)
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    ph = rng.uniform(0, 2 * math.pi, size=8)
    k = 2 * math.pi / n

    def wave(i):
        return (np.sin(k * (x + 2 * y) + ph[i]) + np.cos(k * (3 * z - y) + ph[i + 1])) * 0.5

    rho = 1.0 + amp * wave(0) + 0.05 * rng.random((n, n, n))
    u = np.stack([speed * wave(1), -0.6 * speed * wave(2), 0.8 * speed * wave(3)])
    u += 0.05 * speed * rng.standard_normal(u.shape)
    e = energy * (1.0 + amp * wave(4)) + 0.02 * energy * rng.random((n, n, n))
    q = np.concatenate([rho[None], a * rho * u, (a * a * rho * (e + 0.5 * (u * u).sum(0)))[None]])
    return q.astype(np.float32)


def random_positions(n, seed, count=None):
    """Particle positions (3, count) uniform in [0, n)."""
    count = n ** 3 if count is None else count
    return np.random.default_rng(seed).uniform(0, n, size=(3, count)).astype(np.float32)


def random_field(shape, seed, scale=1.0):
    return (scale * np.random.default_rng(seed).standard_normal(shape)).astype(np.float32)
