"""The allocation-free multi-box step (lbm_sc_step_boxes_noalloc) against the group step: the same
boxes stepped by both end bitwise equal, on two calls in a row (the second with fewer and smaller
boxes, so the fixed device array still holds the first call's longer work list), with and without
the persistent work-queue kernel, with two steps per launch (odd counts ending in single steps),
and when recorded into a caller's graph and replayed."""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def configs(prec, stream):
    return [
        lbm.config(20, 20, 20, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.3,
                   radius=5.0, width=2.0, noise_amp=1e-6, seed=11, stream=stream),
        lbm.config(33, 17, 25, psi=1, geom=lbm.LBM_SC_BUBBLE, prec=prec, g_over_gc=1.2,
                   radius=5.0, width=1.5, tau=0.8, noise_amp=1e-6, seed=12, stream=stream),
        lbm.config(70, 45, 12, psi=0, geom=lbm.LBM_SC_SLAB, prec=prec, g_over_gc=1.5,
                   slab_thickness=22.0, width=2.0, slab_axis=0, stream=stream),
        lbm.config(3, 5, 7, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.1,
                   radius=1.0, width=1.0, noise_amp=1e-3, seed=13, stream=stream),
        lbm.config(131, 9, 40, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.7,
                   radius=6.0, width=2.0, noise_amp=1e-6, seed=14, stream=stream),
    ]


BASE = dict(rows=2, z_chunk=32, xcd_remap=1, prefetch=0, persistent=0, workers=0, graph_steps=0,
            waves=4, tile_x=64, items_per_cu=0)
LAUNCHES = [
    dict(BASE),
    dict(BASE, rows=4, z_chunk=9, prefetch=1, persistent=1, workers=64),
    dict(BASE, rows=4, z_chunk=6, waves=8, tile_x=0),
    dict(BASE, rows=4, z_chunk=0, items_per_cu=2, waves=8, tile_x=0, persistent=1, workers=24),
]


def by_group(cfgs, launch, nsteps, stream):
    boxes = [lbm.Box(c) for c in cfgs]
    with lbm.Group(stream) as g:
        g.set_launch(**launch)
        g.set(boxes)
        g.step(nsteps)
        out = [b.get() for b in boxes]
    for b in boxes:
        b.close()
    return out


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP64])
@pytest.mark.parametrize("li", range(len(LAUNCHES)))
def test_noalloc_step_equals_group_step(prec, li):
    import torch
    launch = LAUNCHES[li]
    say(f"allocation-free step prec={prec} launch={launch}")
    s = torch.cuda.Stream()
    first = configs(prec, s.cuda_stream)
    second = [first[3], first[0]]          # fewer and smaller boxes on the second call
    for cfgs, nsteps in ((first, 11), (second, 7)):
        want = by_group(cfgs, launch, nsteps, s.cuda_stream)
        boxes = [lbm.Box(c) for c in cfgs]
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], 3, **launch)
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], nsteps - 3, **launch)
        got = [b.get() for b in boxes]
        steps = [b.observables(profile=False)[0]["step"] for b in boxes]
        for b in boxes:
            b.close()
        assert steps == [nsteps] * len(cfgs)
        for k, (a, w) in enumerate(zip(got, want)):
            assert np.array_equal(a, w), f"box {k} of {len(cfgs)} differs from the group step"


def test_noalloc_steps_recorded_into_a_caller_graph():
    """Recorded inside a caller's capture (even step count), each replay advances the boxes
    like the same number of eager allocation-free steps; an odd count is refused there."""
    import torch
    say("allocation-free steps inside a caller's graph capture")
    s = torch.cuda.Stream()
    launch = LAUNCHES[1]
    cfgs = configs(lbm.LBM_SC_FP32_SHIFTED, s.cuda_stream)[:3]
    boxes = [lbm.Box(c) for c in cfgs]
    refs = [lbm.Box(c) for c in cfgs]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        with pytest.raises(lbm.LbmScError) as odd:
            lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], 3, **launch)
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], 4, **launch)
    assert odd.value.code == lbm.LBM_SC_EINVAL
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in refs], 4, **launch)
        torch.cuda.synchronize()
        for b, r in zip(boxes, refs):
            assert np.array_equal(b.get(), r.get())
    for b in boxes + refs:
        b.close()


def test_noalloc_rejects_bad_calls_before_any_device_work():
    import torch
    say("allocation-free step: argument checks")
    s = torch.cuda.Stream()
    c32 = configs(lbm.LBM_SC_FP32_SHIFTED, s.cuda_stream)[0]
    c64 = configs(lbm.LBM_SC_FP64, s.cuda_stream)[3]
    with lbm.Box(c32) as a, lbm.Box(c64) as b:
        before = a.get()
        cases = {
            "too many boxes": ([a.h] * (lbm.LBM_SC_NOALLOC_MAX_BOXES + 1), BASE),
            "mixed precision": ([a.h, b.h], BASE),
            "twice": ([a.h, a.h], BASE),
            "bad shape": ([a.h], dict(BASE, rows=3)),
            "odd workers": ([a.h], dict(BASE, persistent=1, workers=12)),
        }
        for why, (hs, launch) in cases.items():
            with pytest.raises(lbm.LbmScError) as e:
                lbm.lbm_sc_step_boxes_noalloc(hs, 2, **launch)
            say(f"{why}: {lbm.lbm_sc_last_error()}")
            assert e.value.code == lbm.LBM_SC_EINVAL, why
        assert "at most 1024" in str(pytest.raises(
            lbm.LbmScError, lbm.lbm_sc_step_boxes_noalloc,
            [a.h] * (lbm.LBM_SC_NOALLOC_MAX_BOXES + 1), 2, **BASE).value)
        assert np.array_equal(a.get(), before)
        assert a.observables(profile=False)[0]["step"] == 0


# two steps per launch: FP32-shifted boxes at tau = 1 only
TWO = [dict(BASE, rows=2, waves=8, tile_x=32, z_chunk=0, items_per_cu=4, steps_per_pass=2),
       dict(BASE, rows=1, waves=8, tile_x=64, prefetch=1, z_chunk=9, steps_per_pass=2)]


def configs_tau1(stream):
    return [c for c in configs(lbm.LBM_SC_FP32_SHIFTED, stream) if c.tau == 1.0]


@pytest.mark.parametrize("li", range(len(TWO)))
def test_noalloc_two_steps_per_launch_equal_group_step(li):
    import torch
    launch = TWO[li]
    say(f"allocation-free step, two steps per launch: {launch}")
    s = torch.cuda.Stream()
    first = configs_tau1(s.cuda_stream)
    second = [first[2], first[0]]          # fewer and smaller boxes on the second call
    for cfgs, nsteps in ((first, 11), (second, 7)):
        want = by_group(cfgs, launch, nsteps, s.cuda_stream)
        boxes = [lbm.Box(c) for c in cfgs]
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], 3, **launch)
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], nsteps - 3, **launch)
        got = [b.get() for b in boxes]
        steps = [b.observables(profile=False)[0]["step"] for b in boxes]
        for b in boxes:
            b.close()
        assert steps == [nsteps] * len(cfgs)
        for k, (a, w) in enumerate(zip(got, want)):
            assert np.array_equal(a, w), f"box {k} of {len(cfgs)} differs from the group step"


@pytest.mark.parametrize("nsteps", [4, 6])
def test_noalloc_two_steps_per_launch_recorded_into_a_caller_graph(nsteps):
    """Recorded inside a caller's capture, 4 steps (two launches) and 6 (two launches and a pair
    of single steps, so that the replays find every box where they expect it): each replay
    advances the boxes like the same number of eager allocation-free steps."""
    import torch
    say(f"allocation-free two-step launches inside a caller's graph capture, {nsteps} steps")
    s = torch.cuda.Stream()
    launch = TWO[0]
    cfgs = configs_tau1(s.cuda_stream)[:3]
    boxes = [lbm.Box(c) for c in cfgs]
    refs = [lbm.Box(c) for c in cfgs]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in boxes], nsteps, **launch)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        lbm.lbm_sc_step_boxes_noalloc([b.h for b in refs], nsteps, **launch)
        torch.cuda.synchronize()
        for b, r in zip(boxes, refs):
            assert np.array_equal(b.get(), r.get())
    for b in boxes + refs:
        b.close()
