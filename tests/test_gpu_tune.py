"""The autotuner on the GPU: it times real steps, skips shapes a box cannot take, leaves the
fastest shape set, and - since shapes change only the schedule - the boxes it stepped end
bitwise equal to the same boxes stepped alone for the same number of steps."""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm
from paper_2105_08772_amd import tune

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cfgs(stream):
    return [lbm.config(24, 20, 18, psi=0, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP32_SHIFTED,
                       g_over_gc=1.3, radius=5.0, width=2.0, noise_amp=1e-6, seed=31, stream=stream),
            lbm.config(700, 3, 4, psi=1, geom=lbm.LBM_SC_SLAB, prec=lbm.LBM_SC_FP32_SHIFTED,
                       g_over_gc=1.2, slab_thickness=300.0, width=2.0, slab_axis=0, stream=stream)]


def test_tune_group_keeps_results_and_sets_the_fastest_shape():
    import torch
    s = torch.cuda.Stream()
    cands = [dict(waves=8, rows=2, prefetch=0, tile_x=64, z_chunk=8, items_per_cu=0, xcd_remap=1,
                  persistent=0, workers=0),
             dict(waves=4, rows=1, prefetch=1, tile_x=32, z_chunk=0, items_per_cu=4, xcd_remap=1,
                  persistent=1, workers=256),
             # rows of 700 nodes do not fit full-row tiles: skipped
             dict(waves=8, rows=4, prefetch=0, tile_x=0, z_chunk=8, items_per_cu=0, xcd_remap=1,
                   persistent=0, workers=0)]
    boxes = [lbm.Box(c) for c in cfgs(s.cuda_stream)]
    steps = 4
    with lbm.Group(s.cuda_stream) as g:
        g.set(boxes)
        best = tune.tune_group(g, steps=steps, candidates=cands, log=say)
        assert best["seconds_per_step"] > 0
        assert {k: best[k] for k in cands[0]} in cands[:2]
        launch = g.launch()
        assert all(launch[k] == best[k] for k in cands[0])
        g.step(3)
        g.set([])
    total = 2 * 2 * steps + 3      # two usable candidates, a warm-up and a timed run each
    for b, c in zip(boxes, cfgs(s.cuda_stream)):
        with lbm.Box(c) as ref:
            ref.step(total)
            assert np.array_equal(b.get(), ref.get())
        b.close()


def test_tune_box_keeps_results_and_sets_the_fastest_shape():
    import torch
    s = torch.cuda.Stream()
    cfg = cfgs(s.cuda_stream)[0]
    cands = [dict(waves=8, rows=2, prefetch=0, tile_x=64, z_chunk=8, xcd_remap=1),
             dict(waves=4, rows=2, prefetch=1, tile_x=32, z_chunk=16, xcd_remap=0),
             dict(waves=8, rows=4, prefetch=0, tile_x=0, z_chunk=8, xcd_remap=1)]
    steps = 4
    with lbm.Box(cfg) as b, lbm.Box(cfg) as ref:
        best = tune.tune_box(b, steps=steps, candidates=cands, log=say)
        assert {k: best[k] for k in cands[0]} in cands
        launch = b.launch()
        assert all(launch[k] == best[k] for k in ("rows", "waves", "prefetch", "tile_x", "xcd_remap"))
        b.step(5)
        ref.step(len(cands) * (2 + steps) + 5)
        assert np.array_equal(b.get(), ref.get())
