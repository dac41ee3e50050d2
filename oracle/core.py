"""ctypes binding of the plain C oracle (oracle/lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg; never by the product package.

Arrays are numpy float64, C-contiguous. Populations: shape (19, nz, ny, nx) in the D3Q19 order
rest, +-x, +-y, +-z, then the twelve face diagonals, each followed by its opposite.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

PSI_EXP = 0       # psi = exp(-1/n)
PSI_ONEMINUS = 1  # psi = 1 - exp(-n)

DROPLET, BUBBLE, SLAB = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc: plain -O2, OpenMP over z-planes, no FMA contraction."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        i, d, u64, ll = ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_longlong
        L.ora_psi.argtypes = [d, i]
        L.ora_psi.restype = d
        L.ora_tables.argtypes = [_I, _D, _D]
        L.ora_density.argtypes = [_D, i, i, i, i, _D, _D]
        L.ora_force.argtypes = [_D, i, i, i, d, _D]
        L.ora_step.argtypes = [_D, _D, i, i, i, d, d, i]
        L.ora_collide_at.argtypes = [_D, i, i, i, d, d, i, i, i, i, _D]
        L.ora_pressure_tensor.argtypes = [_D, i, i, i, d, i, _D]
        L.ora_noise.argtypes = [u64, u64, d]
        L.ora_noise.restype = d
        L.ora_init_density.argtypes = [i, i, i, i, i, d, d, d, d, d, u64, _D]
        L.ora_init_populations.argtypes = [_D, i, i, i, d, i, _D]
        L.ora_velocity.argtypes = [_D, i, i, i, d, i, _D, _D]
        L.ora_run.argtypes = [_D, i, i, i, d, d, i, ll]
        L.ora_threads.argtypes = []
        L.ora_threads.restype = i
        L.ora_set_threads.argtypes = [i]
        L.ora_set_threads.restype = None
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _dims(f):
    assert f.ndim == 4 and f.shape[0] == 19, f.shape
    nz, ny, nx = f.shape[1:]
    return nx, ny, nz


def tables():
    """(xi[19,3] int, w[19], W[19]) as the oracle holds them (W[0] = 0: the rest vector has no
    forcing weight)."""
    xi = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    W = np.zeros(19)
    lib().ora_tables(xi.ctypes.data_as(_I), _p(w), _p(W))
    return xi.reshape(19, 3), w, W


def threads():
    """OpenMP threads the oracle's loops use."""
    return lib().ora_threads()


def set_threads(n):
    """Set the OpenMP threads of the oracle's loops."""
    lib().ora_set_threads(int(n))


def psi(n, kind):
    return lib().ora_psi(float(n), int(kind))


def density(f, kind=PSI_EXP):
    nx, ny, nz = _dims(f)
    n = np.empty((nz, ny, nx))
    ps = np.empty((nz, ny, nx))
    lib().ora_density(_p(f), nx, ny, nz, kind, _p(n), _p(ps))
    return n, ps


def force(psi_field, G):
    nz, ny, nx = psi_field.shape
    F = np.empty((3, nz, ny, nx))
    lib().ora_force(_p(np.ascontiguousarray(psi_field)), nx, ny, nz, float(G), _p(F))
    return F


def step(f, G, tau=1.0, kind=PSI_EXP):
    """One time step from the pre-collision state f(t); returns f(t+1)."""
    nx, ny, nz = _dims(f)
    out = np.empty_like(f)
    lib().ora_step(_p(f), _p(out), nx, ny, nz, float(G), float(tau), int(kind))
    return out


def run(f, G, tau=1.0, kind=PSI_EXP, nsteps=1):
    """nsteps time steps; returns a new array."""
    nx, ny, nz = _dims(f)
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    lib().ora_run(_p(g), nx, ny, nz, float(G), float(tau), int(kind), int(nsteps))
    return g


def collide_at(f, G, tau, kind, x, y, z):
    """Post-collision populations f*_i at node (x, y, z), computed from f without whole-box
    fields; after streaming they land at (x, y, z) + xi_i in f(t+1)."""
    nx, ny, nz = _dims(f)
    out = np.empty(19)
    lib().ora_collide_at(_p(f), nx, ny, nz, float(G), float(tau), int(kind), int(x), int(y),
                         int(z), _p(out))
    return out


def pressure_tensor(f, G, kind=PSI_EXP):
    """Eq. (sm:pt) at every node: array (6, nz, ny, nx) for xx, yy, zz, xy, xz, yz."""
    nx, ny, nz = _dims(f)
    P = np.empty((6, nz, ny, nx))
    lib().ora_pressure_tensor(_p(f), nx, ny, nz, float(G), int(kind), _p(P))
    return P


def velocity(f, G, kind=PSI_EXP):
    """(j, u): momentum density sum xi f and physical velocity (sum xi f + F/2)/n, each (3,nz,ny,nx)."""
    nx, ny, nz = _dims(f)
    j = np.empty((3, nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    lib().ora_velocity(_p(f), nx, ny, nz, float(G), int(kind), _p(j), _p(u))
    return j, u


def noise(seed, index, amp):
    return lib().ora_noise(int(seed) & (2**64 - 1), int(index), float(amp))


def init_density(nx, ny, nz, geom, R, w, n_in, n_out, noise_amp=0.0, seed=0, slab_axis=2):
    n = np.empty((nz, ny, nx))
    lib().ora_init_density(nx, ny, nz, int(geom), int(slab_axis), float(R), float(w), float(n_in),
                           float(n_out), float(noise_amp), int(seed) & (2**64 - 1), _p(n))
    return n


def init_populations(n, G, kind=PSI_EXP):
    nz, ny, nx = n.shape
    f = np.empty((19, nz, ny, nx))
    lib().ora_init_populations(_p(np.ascontiguousarray(n)), nx, ny, nz, float(G), int(kind), _p(f))
    return f
