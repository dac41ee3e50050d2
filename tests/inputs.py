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


def batched_boxes(seed=2105, count=64, lmin=48, lmax=160, rmin=0.15, rmax=0.35, gmin=1.05,
                  gmax=1.8):
    """The batched workload: `count` cubic boxes with L ~ U{lmin..lmax}, radius ~ U[rmin, rmax] L,
    G/G_c ~ U[gmin, gmax], droplet or bubble with probability 1/2, each with its own noise seed."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        L = int(rng.integers(lmin, lmax + 1))
        out.append(dict(L=L, radius=float(rng.uniform(rmin, rmax) * L),
                        g_over_gc=float(rng.uniform(gmin, gmax)),
                        bubble=bool(rng.integers(0, 2)), seed=seed * 1000 + k))
    return out


def served_requests(seed=8772, count=32, rate=1.0, lmin=32, lmax=192, rmin_abs=6.0, rmax_abs=60.0,
                    rmin=0.15, rmax=0.35, gmin=1.05, gmax=1.8):
    """Poisson arrivals (exponential gaps of mean 1/rate seconds) of requests with L ~
    U{lmin..lmax}, radius ~ U[max(rmin_abs, rmin L), min(rmax_abs, rmax L)], G/G_c ~ U[gmin, gmax],
    droplet or bubble with probability 1/2. Returns dicts in arrival order."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        L = int(rng.integers(lmin, lmax + 1))
        lo, hi = max(rmin_abs, rmin * L), min(rmax_abs, rmax * L)
        out.append(dict(rid=k, L=L, radius=float(rng.uniform(lo, hi)),
                        g_over_gc=float(rng.uniform(gmin, gmax)), bubble=bool(rng.integers(0, 2)),
                        seed=seed * 1000 + k, arrival=t))
    return out
