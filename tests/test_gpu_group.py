"""Groups: many boxes advanced by one multi-box launch per step.

A box stepped in a group must end bitwise equal to the same box stepped alone (the per-node
arithmetic does not depend on the launch), for every group launch shape, with and without the
persistent work-queue kernel and with hipGraph replays of step chunks.
"""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def box_configs(prec, stream):
    c = []
    c.append(lbm.config(20, 20, 20, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.3,
                        radius=5.0, width=2.0, noise_amp=1e-6, seed=11, stream=stream))
    c.append(lbm.config(33, 17, 25, psi=1, geom=lbm.LBM_SC_BUBBLE, prec=prec, g_over_gc=1.2,
                        radius=5.0, width=1.5, tau=0.8, noise_amp=1e-6, seed=12, stream=stream))
    c.append(lbm.config(70, 45, 12, psi=0, geom=lbm.LBM_SC_SLAB, prec=prec, g_over_gc=1.5,
                        slab_thickness=22.0, width=2.0, slab_axis=0, stream=stream))
    c.append(lbm.config(3, 5, 7, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.1,
                        radius=1.0, width=1.0, noise_amp=1e-3, seed=13, stream=stream))
    c.append(lbm.config(131, 9, 40, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.7,
                        radius=6.0, width=2.0, noise_amp=1e-6, seed=14, stream=stream))
    return c


def alone(cfgs, nsteps):
    out = []
    for c in cfgs:
        with lbm.Box(c) as b:
            b.step(nsteps)
            out.append(b.get())
    return out


LAUNCHES = [
    dict(rows=2, z_chunk=32, xcd_remap=1, prefetch=1, persistent=0, workers=0, graph_steps=4),
    dict(rows=1, z_chunk=5, xcd_remap=0, prefetch=0, persistent=0, workers=0, graph_steps=0),
    dict(rows=4, z_chunk=9, xcd_remap=1, prefetch=1, persistent=1, workers=64, graph_steps=6),
    dict(rows=2, z_chunk=64, xcd_remap=1, prefetch=0, persistent=1, workers=8, graph_steps=2),
    dict(rows=2, z_chunk=7, xcd_remap=1, prefetch=0, persistent=1, workers=24, graph_steps=4,
         waves=8, tile_x=64),
    dict(rows=1, z_chunk=16, xcd_remap=1, prefetch=1, persistent=0, workers=0, graph_steps=0,
         tile_x=32),
    dict(rows=2, z_chunk=3, xcd_remap=0, prefetch=0, persistent=1, workers=40, graph_steps=2,
         waves=8, tile_x=32),
    dict(rows=4, z_chunk=6, xcd_remap=1, prefetch=0, persistent=0, workers=0, graph_steps=4,
         waves=8, tile_x=0),
    dict(rows=4, z_chunk=16, xcd_remap=1, prefetch=0, persistent=1, workers=16, graph_steps=0,
         waves=8, tile_x=0),
    dict(rows=2, z_chunk=5, xcd_remap=1, prefetch=0, persistent=0, workers=0, graph_steps=2,
         waves=8, tile_x=0),
    dict(rows=4, z_chunk=7, xcd_remap=0, prefetch=0, persistent=1, workers=24, graph_steps=4,
         waves=4, tile_x=0),
    dict(rows=4, z_chunk=0, items_per_cu=1, xcd_remap=1, prefetch=0, persistent=0, workers=0,
         graph_steps=4, waves=8, tile_x=0),
    dict(rows=2, z_chunk=0, items_per_cu=0, xcd_remap=1, prefetch=1, persistent=1, workers=24,
         graph_steps=2, waves=4, tile_x=64),
]


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP64,
                                  lbm.LBM_SC_FP32_SHIFTED_MATH64])
@pytest.mark.parametrize("li", range(len(LAUNCHES)))
def test_group_equals_boxes_alone(prec, li):
    import torch
    launch = LAUNCHES[li]
    say(f"group prec={prec} launch={launch}")
    s = torch.cuda.Stream()
    cfgs = box_configs(prec, s.cuda_stream)
    want = alone(cfgs, 11)
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(s.cuda_stream) as g:
        g.set_launch(**launch)
        g.set(boxes)
        g.step(3)
        g.step(8)   # 11 in total: graph replays plus single launches
        got = [b.get() for b in boxes]
        info = g.info()
    assert info["nbox"] == len(cfgs)
    assert info["nodes"] == sum(c.nx * c.ny * c.nz for c in cfgs)
    for k, (a, b) in enumerate(zip(got, want)):
        assert np.array_equal(a, b), f"box {k} differs from the same box stepped alone"
    for b in boxes:
        b.close()


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP64,
                                  lbm.LBM_SC_FP32_SHIFTED_MATH64])
@pytest.mark.parametrize("li", [7, 8, 9, 10, 11, 4])
def test_packed_rows_in_a_group_equal_padded_boxes_alone(prec, li):
    """Boxes with packed rows (pitch nx) mixed with padded ones in one group: every box ends
    bitwise equal to the same box with padded rows stepped alone, under full-row tiles (whose
    lane window is then aligned to the line grid per tile) and under x-y tiles."""
    import torch
    launch = LAUNCHES[li]
    say(f"packed rows in a group prec={prec} launch={launch}")
    s = torch.cuda.Stream()
    cfgs = box_configs(prec, s.cuda_stream)
    want = alone(cfgs, 11)
    for k, c in enumerate(cfgs):
        c.packed_rows = k % 2 == 0 or c.nx % 32 != 0
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(s.cuda_stream) as g:
        g.set_launch(**launch)
        g.set(boxes)
        g.step(3)
        g.step(8)
        got = [b.get() for b in boxes]
    for k, (a, b) in enumerate(zip(got, want)):
        assert np.array_equal(a, b), f"box {k} (packed {cfgs[k].packed_rows}) differs"
    for b in boxes:
        b.close()


def test_group_full_row_tiles_8_nodes_per_thread():
    """8 nodes per thread (FP32 arithmetic only): bitwise equal to the boxes stepped alone;
    groups of FP64 boxes or of boxes with FP64 arithmetic reject the shape."""
    import torch
    s = torch.cuda.Stream()
    launch = dict(rows=8, z_chunk=8, xcd_remap=1, prefetch=0, persistent=1, workers=64,
                  graph_steps=4, waves=8, tile_x=0)
    cfgs = box_configs(lbm.LBM_SC_FP32_SHIFTED, s.cuda_stream)
    want = alone(cfgs, 9)
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(s.cuda_stream) as g:
        g.set_launch(**launch)
        g.set(boxes)
        g.step(9)
        got = [b.get() for b in boxes]
    for k, (a, b) in enumerate(zip(got, want)):
        assert np.array_equal(a, b), f"box {k} differs from the same box stepped alone"
    for b in boxes:
        b.close()
    for prec in (lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED_MATH64):
        b64 = lbm.Box(box_configs(prec, s.cuda_stream)[0])
        with lbm.Group(s.cuda_stream) as g:
            g.set([b64])
            with pytest.raises(lbm.LbmScError):
                g.set_launch(**launch)
            g.set([])
            g.set_launch(**launch)
            with pytest.raises(lbm.LbmScError):
                g.set([b64])
        b64.close()


def test_group_resyncs_after_a_box_steps_alone_and_after_resets():
    import torch
    s = torch.cuda.Stream()
    cfgs = box_configs(lbm.LBM_SC_FP32_SHIFTED, s.cuda_stream)[:3]
    want = alone(cfgs, 9)
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(s.cuda_stream) as g:
        g.set_launch(graph_steps=2, persistent=1, workers=16)
        g.set(boxes)
        g.step(4)
        boxes[1].step(1)         # box 1 runs ahead alone ...
        g.step(4)                # ... the group realigns its work list
        boxes[0].step(1)
        boxes[2].step(1)         # boxes 0 and 2 catch up
        got = [b.get() for b in boxes]
        g.set(boxes[::-1])       # reorder
        g.step(0)
        g.set([])                # empty group is valid
        g.step(5)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    assert [b.get() is not None for b in boxes]
    for b in boxes:
        b.close()


def test_destroying_a_box_removes_it_from_its_groups():
    """A box destroyed while groups still list it leaves them: the next group step rebuilds the
    work list without it (no launch reaches its freed buffers) and the remaining boxes go on
    bitwise as if stepped alone; a group destroyed first leaves its boxes usable."""
    import torch
    s = torch.cuda.Stream()
    cfgs = box_configs(lbm.LBM_SC_FP32_SHIFTED, s.cuda_stream)[:3]
    want0, want2 = alone([cfgs[0], cfgs[2]], 13)
    boxes = [lbm.Box(c) for c in cfgs]
    g1, g2 = lbm.Group(s.cuda_stream), lbm.Group(s.cuda_stream)
    g1.set_launch(graph_steps=2)
    g1.set(boxes)
    g2.set(boxes[1:])
    g1.step(4)                   # graph chunks captured over all three boxes
    boxes[1].close()             # listed by both groups
    assert g1.info()["nbox"] == 2 and g2.info()["nbox"] == 1
    g1.step(6)
    g2.step(3)                   # box 2 runs ahead in the other group ...
    boxes[0].step(3)             # ... and box 0 alone
    assert np.array_equal(boxes[0].get(), want0) and np.array_equal(boxes[2].get(), want2)
    g2.close()                   # box 2 stays usable without the group
    boxes[2].step(1)
    g1.step(2)
    g1.close()
    boxes[0].close()
    boxes[2].close()


def test_group_rejects_mixed_precision_and_foreign_streams():
    import torch
    s = torch.cuda.Stream()
    other = torch.cuda.Stream()
    a = lbm.Box(lbm.config(8, 8, 8, radius=2.0, prec=lbm.LBM_SC_FP64, stream=s.cuda_stream))
    b = lbm.Box(lbm.config(8, 8, 8, radius=2.0, prec=lbm.LBM_SC_FP32_SHIFTED, stream=s.cuda_stream))
    c = lbm.Box(lbm.config(8, 8, 8, radius=2.0, prec=lbm.LBM_SC_FP64, stream=other.cuda_stream))
    d = lbm.Box(lbm.config(8, 8, 8, radius=2.0, prec=lbm.LBM_SC_FP32_SHIFTED_MATH64,
                           stream=s.cuda_stream))
    with lbm.Group(s.cuda_stream) as g:
        for bad in ([a, b], [a, c], [a, a], [b, d]):
            with pytest.raises(lbm.LbmScError) as e:
                g.set(bad)
            assert e.value.code == lbm.LBM_SC_EINVAL
        with pytest.raises(lbm.LbmScError):
            g.set_launch(workers=12)
        with pytest.raises(lbm.LbmScError):
            g.set_launch(z_chunk=-1)
        with pytest.raises(lbm.LbmScError):
            g.set_launch(z_chunk=0, items_per_cu=-1)
        with pytest.raises(lbm.LbmScError):
            g.set_launch(waves=8, prefetch=1)
        with pytest.raises(lbm.LbmScError):
            g.set_launch(rows=4, tile_x=32)
        with pytest.raises(lbm.LbmScError):
            g.set_launch(graph_steps=3)
    for x in (a, b, c, d):
        x.close()
