"""Two time steps per kernel pass (lbm_sc_launch.steps_per_pass = 2; FP32 storage and arithmetic,
tau = 1). The kernel keeps the first step's post-collision populations of its region in LDS and
applies the second step to them; it collides through the same routines as the single-step
kernels, so every result must be bitwise that of the same number of single steps: on tiny,
ragged and multi-tile boxes, for both pseudopotentials, with z chunks that do and do not divide
the box, odd step counts (the last step single), graph replays, packed rows, a caller's stream
capture, and the FP32 dither's step count carried across calls. Boxes it cannot step (FP64 or
FP64 arithmetic, tau != 1) reject the option.
"""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm
from oracle import core
from tests import inputs

pytestmark = pytest.mark.gpu

XI, W, _ = core.tables()
RHO_REF = 1.5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fp32_state(dims, seed):
    f = inputs.random_populations(dims, seed, W * RHO_REF, amp=0.3)
    g = (f - W.reshape(19, 1, 1, 1) * RHO_REF).astype(np.float32).astype(np.float64)
    return g + W.reshape(19, 1, 1, 1) * RHO_REF


def box(dims, psi=0, packed=0, prec=lbm.LBM_SC_FP32_SHIFTED, tau=1.0):
    nx, ny, nz = dims
    return lbm.Box(lbm.config(nx, ny, nz, psi=psi, geom=lbm.LBM_SC_FROM_HOST, prec=prec, tau=tau,
                              g_over_gc=1.4, rho_ref=RHO_REF, packed_rows=packed))


# two-step shapes (rows, waves, prefetch)
SHAPES2 = [(1, 8, 1, 64), (1, 8, 0, 64), (2, 16, 0, 64), (2, 8, 0, 32), (2, 8, 1, 32),
           (2, 4, 0, 32)]


def set_two(b, shape=(1, 8, 1, 64), zc=None, graph_steps=64):
    rows, waves, pf, tx = shape
    b.set_launch(rows, zc or b.dims[2], 1, pf, waves, tx, graph_steps, 2)


def run(dims, f, counts, psi=0, packed=0, two=False, zc=None, graph_steps=64, shape=(1, 8, 1, 64)):
    with box(dims, psi, packed) as b:
        b.set(f)
        if two:
            set_two(b, shape, zc, graph_steps)
        else:
            b.set_launch(2, zc or dims[2], 1, 0, 8, 64, graph_steps, 1)   # single steps
        out = []
        for n in counts:
            b.step(n)
            out.append(b.get())
        return out


DIMS = [(4, 4, 4), (1, 1, 8), (3, 5, 7), (5, 4, 1), (9, 7, 2), (37, 29, 11), (64, 8, 9),
        (65, 9, 10), (130, 17, 13), (100, 37, 21), (200, 3, 5)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("psi", [0, 1])
def test_two_steps_per_pass_equal_single_steps(dims, psi):
    say(f"two steps per pass dims={dims} psi={psi}")
    f = fp32_state(dims, 31 + sum(dims))
    counts = (2, 1, 3, 4)              # 2, 3, 6, 10 steps: pairs and single last steps
    want = run(dims, f, counts, psi)
    for shape in SHAPES2:
        for zc in (None, 1, 3, 5):
            got = run(dims, f, counts, psi, two=True, zc=zc, shape=shape)
            for k, (a, b) in enumerate(zip(got, want)):
                assert np.array_equal(a, b), (shape, zc, k)


@pytest.mark.parametrize("packed", [0, 1])
def test_two_steps_per_pass_graph_replay_and_packed_rows(packed):
    dims = (101, 45, 40)
    f = fp32_state(dims, 5)
    say(f"two steps per pass, graphs, packed={packed}")
    want = run(dims, f, (128, 70, 1), packed=0)
    for gs in (64, 4, 6, 0):          # 6: not a multiple of 4, so plain launches
        got = run(dims, f, (128, 70, 1), packed=packed, two=True, graph_steps=gs)
        for a, b in zip(got, want):
            assert np.array_equal(a, b), gs


def test_two_steps_per_pass_droplet_observables_and_dither():
    """A droplet created on the device (FP32 dither seeded from the step count): after 2050
    steps the populations and every observable equal those of single steps; a state saved and
    resumed with its step count continues identically."""
    cfg = dict(psi=0, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP32_SHIFTED, g_over_gc=1.3,
               radius=9.0, width=2.0, noise_amp=1e-6, seed=9)
    res = []
    for two in (False, True):
        with lbm.Box(lbm.config(48, 40, 44, **cfg)) as b:
            if two:
                set_two(b, zc=22)
            b.step(2050)
            o, p = b.observables()
            f = b.get()
            b.step(7)
            g = b.get()
        res.append((o, p, f, g))
    (o1, p1, f1, g1), (o2, p2, f2, g2) = res
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2) and np.array_equal(p1, p2)
    for k, v in o1.items():
        w = o2[k]
        if isinstance(v, float) and np.isnan(v):
            assert np.isnan(w), k
        else:
            assert np.array_equal(np.asarray(v), np.asarray(w)), k
    with lbm.Box(lbm.config(48, 40, 44, **cfg)) as b:
        set_two(b, (2, 8, 0, 32), zc=11)
        b.set(f1)
        b.set_step(2050)
        b.step(7)
        assert np.array_equal(b.get(), g1)


def test_two_steps_per_pass_in_a_caller_capture():
    import torch
    dims = (70, 33, 21)
    f = fp32_state(dims, 8)
    want = run(dims, f, (8, 6, 6))
    s = torch.cuda.Stream()
    cfg = lbm.config(*dims, psi=0, geom=lbm.LBM_SC_FROM_HOST, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.4, rho_ref=RHO_REF, stream=s.cuda_stream)
    with lbm.Box(cfg) as b:
        b.set(f)
        set_two(b)
        outs = []
        for n in (8, 6):                # 8: two-step launches; 6 (4k + 2): single steps
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                b.step(n)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            outs.append(b.get())
            if n == 6:
                g.replay()
                torch.cuda.synchronize()
                outs.append(b.get())
    for a, c in zip(outs, want):
        assert np.array_equal(a, c)


def test_two_steps_per_pass_is_refused_where_it_does_not_apply():
    for prec, tau in ((lbm.LBM_SC_FP64, 1.0), (lbm.LBM_SC_FP32_SHIFTED_MATH64, 1.0),
                      (lbm.LBM_SC_FP32_SHIFTED, 0.8)):
        with box((16, 16, 16), prec=prec, tau=tau) as b:
            with pytest.raises(lbm.LbmScError):
                set_two(b)
            with pytest.raises(lbm.LbmScError):
                b.set_launch(1, 16, 1, 1, 8, 64, 64, 3)
    with box((16, 16, 16)) as b:
        for bad in ((2, 8, 1, 64), (1, 4, 0, 64), (2, 16, 1, 64), (4, 8, 0, 64), (3, 12, 0, 64),
                    (1, 8, 0, 32), (2, 16, 0, 32), (2, 4, 1, 32), (1, 4, 0, 32)):
            with pytest.raises(lbm.LbmScError):
                set_two(b, bad)
        set_two(b, (2, 8, 0, 32), zc=5)
        assert b.launch() == dict(rows=2, z_chunk=5, xcd_remap=1, prefetch=0, waves=8, tile_x=32,
                                  graph_steps=64, steps_per_pass=2)
