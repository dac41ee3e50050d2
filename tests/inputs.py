"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds none of the method's arithmetic: it only draws random numbers into arrays whose scale the
caller chooses.
"""
import numpy as np


def random_populations(dims, seed, scale, amp=0.2):
    """Positive populations of shape (19, nz, ny, nx): scale[i] * (1 + amp * U(-1, 1))."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    s = np.asarray(scale, dtype=np.float64).reshape(19, 1, 1, 1)
    return s * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(19, nz, ny, nx)))


def random_field(shape, seed, lo, hi):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)
