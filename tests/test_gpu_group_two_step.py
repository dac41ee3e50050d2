"""Groups with two time steps per launch (lbm_sc_group_launch.steps_per_pass = 2; every box FP32
storage and arithmetic at tau = 1). The multi-box launch marches each (box, tile, z chunk) item
with the two-step tile kernel and an odd last step runs box by box in single steps, so every box
must end bitwise equal to the same box advanced by single steps alone: for every two-step tile
shape, fixed and per-box z chunks, graph replays and plain launches, odd step counts, packed and
padded rows, both pseudopotentials, a box that steps alone in between, the FP32 dither's step
count over thousands of steps, and the full 64-box batched mix against the single-step group.
Groups that cannot take it (FP64 storage or arithmetic, tau != 1, the persistent grid) reject it,
and so does the allocation-free entry point for such boxes.
"""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm
from tests import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def box_configs(stream, packed=(0, 0, 0, 0, 0, 0, 0)):
    """FP32-shifted boxes at tau = 1: ragged sizes, both psi, droplet, bubble and slab."""
    F32 = lbm.LBM_SC_FP32_SHIFTED
    c = [lbm.config(20, 20, 20, psi=0, geom=lbm.LBM_SC_DROPLET, prec=F32, g_over_gc=1.3,
                    radius=5.0, width=2.0, noise_amp=1e-6, seed=11, stream=stream),
         lbm.config(33, 17, 25, psi=1, geom=lbm.LBM_SC_BUBBLE, prec=F32, g_over_gc=1.2,
                    radius=5.0, width=1.5, noise_amp=1e-6, seed=12, stream=stream),
         lbm.config(70, 45, 12, psi=0, geom=lbm.LBM_SC_SLAB, prec=F32, g_over_gc=1.5,
                    slab_thickness=22.0, width=2.0, slab_axis=0, stream=stream),
         lbm.config(3, 5, 7, psi=0, geom=lbm.LBM_SC_DROPLET, prec=F32, g_over_gc=1.1,
                    radius=1.0, width=1.0, noise_amp=1e-3, seed=13, stream=stream),
         lbm.config(131, 9, 40, psi=0, geom=lbm.LBM_SC_DROPLET, prec=F32, g_over_gc=1.7,
                    radius=6.0, width=2.0, noise_amp=1e-6, seed=14, stream=stream),
         lbm.config(49, 49, 2, psi=1, geom=lbm.LBM_SC_DROPLET, prec=F32, g_over_gc=1.4,
                    radius=8.0, width=2.0, noise_amp=1e-6, seed=15, stream=stream),
         lbm.config(1, 2, 3, psi=1, geom=lbm.LBM_SC_DROPLET, prec=F32, g_over_gc=1.2,
                    radius=1.0, width=1.0, noise_amp=1e-3, seed=16, stream=stream)]
    for cfg, p in zip(c, packed):
        cfg.packed_rows = p
    return c


def alone_single(cfgs, counts):
    """Each box alone in single steps; its populations after each count of `counts`."""
    out = []
    for c in cfgs:
        with lbm.Box(c) as b:
            b.set_launch(2, c.nz, 1, 0, 8, 64, 64, 1)
            res = []
            for n in counts:
                b.step(n)
                res.append(b.get())
            out.append(res)
    return out


# two-step tile shapes (rows, waves, prefetch, tile_x)
SHAPES2 = [(1, 8, 1, 64), (1, 8, 0, 64), (2, 16, 0, 64), (2, 8, 0, 32), (2, 8, 1, 32),
           (2, 4, 0, 32)]
CHUNKS = [dict(z_chunk=3), dict(z_chunk=16), dict(z_chunk=0, items_per_cu=1),
          dict(z_chunk=0, items_per_cu=8)]
GRAPHS = [4, 6, 0, 8]       # 6: not a multiple of 4, so plain launches
COUNTS = (3, 8, 1, 12)      # 3, 11, 12, 24 steps: odd counts end in single steps


def launch2(shape, chunk, graph_steps, remap=1):
    rows, waves, pf, tx = shape
    return dict(rows=rows, waves=waves, prefetch=pf, tile_x=tx, xcd_remap=remap, persistent=0,
                workers=0, graph_steps=graph_steps, steps_per_pass=2, **chunk)


@pytest.mark.parametrize("si", range(len(SHAPES2)))
def test_two_step_group_equals_single_steps_alone(si):
    import torch
    s = torch.cuda.Stream()
    cfgs = box_configs(s.cuda_stream)
    want = alone_single(cfgs, COUNTS)
    for ci, chunk in enumerate(CHUNKS):
        launch = launch2(SHAPES2[si], chunk, GRAPHS[ci], remap=ci % 2)
        say(f"two-step group {launch}")
        boxes = [lbm.Box(c) for c in cfgs]
        with lbm.Group(s.cuda_stream) as g:
            g.set_launch(**launch)
            g.set(boxes)
            assert g.launch()["steps_per_pass"] == 2
            for k, n in enumerate(COUNTS):
                g.step(n)
                for j, b in enumerate(boxes):
                    assert np.array_equal(b.get(), want[j][k]), (launch, j, k)
        for b in boxes:
            b.close()


def test_two_step_group_packed_rows_resync_and_reorder():
    """Packed and padded rows in one group; a box that steps alone puts the group's work list
    out of phase (rebuilt before the next launch); the box order changes between calls."""
    import torch
    s = torch.cuda.Stream()
    cfgs = box_configs(s.cuda_stream, packed=(1, 0, 1, 1, 0, 1, 1))
    want = alone_single(box_configs(s.cuda_stream), (15,))
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(s.cuda_stream) as g:
        g.set_launch(**launch2((2, 8, 0, 32), dict(z_chunk=0, items_per_cu=4), 4))
        g.set(boxes)
        g.step(4)
        boxes[1].step(1)             # box 1 runs ahead alone ...
        g.step(9)                    # ... the group realigns: two graph replays, a single step
        for j, b in enumerate(boxes):
            if j != 1:
                b.step(1)            # every box has now taken 14 steps
        g.set(boxes[::-1])
        g.step(1)                    # the 15th: single steps of each box, in the new order
        for j, b in enumerate(boxes):
            assert np.array_equal(b.get(), want[j][0]), j
    for b in boxes:
        b.close()


def test_two_step_group_dither_and_observables_over_many_steps():
    """Droplets created on the device (the FP32 dither seeded from each box's step count):
    after 2051 group steps (graph chunks of 64 steps = 32 launches, then an odd single step),
    populations and observables equal those of the boxes stepped alone in single steps."""
    import torch
    s = torch.cuda.Stream()
    cfgs = [lbm.config(L, psi=p, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP32_SHIFTED,
                       g_over_gc=1.3, radius=0.3 * L, width=2.0, noise_amp=1e-6, seed=20 + L,
                       stream=s.cuda_stream) for L, p in ((24, 0), (37, 1), (50, 0))]
    want, wobs = [], []
    for c in cfgs:
        with lbm.Box(c) as b:
            b.set_launch(2, c.nz, 1, 0, 8, 64, 64, 1)
            b.step(2051)
            want.append(b.get())
            wobs.append(b.observables(profile=False)[0])
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(s.cuda_stream) as g:
        g.set_launch(**launch2((2, 8, 0, 32), dict(z_chunk=0, items_per_cu=8), 64))
        g.set(boxes)
        g.step(2051)
        for b, f, o in zip(boxes, want, wobs):
            assert np.array_equal(b.get(), f)
            got = b.observables(profile=False)[0]
            assert got["step"] == 2051
            for k, v in o.items():
                w = got[k]
                if isinstance(v, float) and np.isnan(v):
                    assert np.isnan(w), k
                else:
                    assert np.array_equal(np.asarray(v), np.asarray(w)), k
    for b in boxes:
        b.close()


def test_full_size_batched_mix_two_step_group_equals_single_step_group():
    """The 64-box batched mix (seed 2105, L ~ U{48..160}, rows packed) in two groups: two steps
    per launch in 32 x 16 tiles with per-box z chunks, against the single-step group with the
    full-row tiles the benchmark's tuner picks (checked against the oracle on sampled nodes in
    the parity tests). Every box bitwise equal after 2 steps (one launch) and after 66 (graph
    chunks of 64 steps)."""
    import torch
    say("batched 64-box mix: two-step group against the single-step group")
    st = torch.cuda.Stream()
    spec = inputs.batched_boxes()

    def make():
        return [lbm.Box(lbm.config(b["L"], psi=0,
                                   geom=lbm.LBM_SC_BUBBLE if b["bubble"] else lbm.LBM_SC_DROPLET,
                                   prec=lbm.LBM_SC_FP32_SHIFTED, tau=1.0, g_over_gc=b["g_over_gc"],
                                   radius=b["radius"], width=2.0, noise_amp=1e-6, seed=b["seed"],
                                   stream=st.cuda_stream, packed_rows=1)) for b in spec]
    one, two = make(), make()
    g1, g2 = lbm.Group(st.cuda_stream), lbm.Group(st.cuda_stream)
    g1.set_launch(rows=4, waves=8, tile_x=0, z_chunk=6, prefetch=0, xcd_remap=1, persistent=0,
                  workers=0, graph_steps=64, steps_per_pass=1)
    g2.set_launch(**launch2((2, 8, 0, 32), dict(z_chunk=0, items_per_cu=8), 64))
    g1.set(one)
    g2.set(two)
    for n in (2, 64):
        g1.step(n)
        g2.step(n)
        bad = [k for k in range(len(spec)) if not np.array_equal(one[k].get(), two[k].get())]
        say(f"after {n} more steps: {len(bad)} boxes differ")
        assert not bad, bad
    g1.close()
    g2.close()
    for b in one + two:
        b.close()


def test_two_step_group_is_refused_where_it_does_not_apply():
    import torch
    s = torch.cuda.Stream()
    good = lbm.Box(lbm.config(16, 16, 16, radius=4.0, prec=lbm.LBM_SC_FP32_SHIFTED,
                              stream=s.cuda_stream))
    bad_boxes = [lbm.Box(lbm.config(16, 16, 16, radius=4.0, prec=p, tau=t, stream=s.cuda_stream))
                 for p, t in ((lbm.LBM_SC_FP64, 1.0), (lbm.LBM_SC_FP32_SHIFTED_MATH64, 1.0),
                              (lbm.LBM_SC_FP32_SHIFTED, 0.8))]
    two = launch2((1, 8, 1, 64), dict(z_chunk=8), 4)
    with lbm.Group(s.cuda_stream) as g:
        for bb in bad_boxes:
            g.set([bb])
            with pytest.raises(lbm.LbmScError):
                g.set_launch(**two)          # a listed box cannot take it
            g.set([])
            g.set_launch(**two)
            with pytest.raises(lbm.LbmScError):
                g.set([good, bb])            # nor can a box added later
            g.set([])
            g.set_launch(steps_per_pass=1, prefetch=0, waves=4, tile_x=64, rows=2)
        for bad in (dict(persistent=1, workers=64), dict(rows=2, prefetch=1, tile_x=64),
                    dict(rows=1, tile_x=32, prefetch=0), dict(waves=4), dict(steps_per_pass=3),
                    dict(steps_per_pass=-1)):
            with pytest.raises(lbm.LbmScError):
                g.set_launch(**dict(two, **bad))
        g.set_launch(**two)
        g.set([good])
        assert g.launch()["steps_per_pass"] == 2
        g.step(3)
    # the allocation-free step takes two steps per launch for the boxes a group takes them for,
    # and refuses the others and the persistent grid
    lbm.lbm_sc_step_boxes_noalloc([good.h], 2, **two)
    for bb in bad_boxes:
        with pytest.raises(lbm.LbmScError):
            lbm.lbm_sc_step_boxes_noalloc([bb.h], 2, **two)
    with pytest.raises(lbm.LbmScError):
        lbm.lbm_sc_step_boxes_noalloc([good.h], 2, **dict(two, persistent=1, workers=64))
    for b in bad_boxes + [good]:
        b.close()
