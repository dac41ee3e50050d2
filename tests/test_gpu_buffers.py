"""Boxes on caller-supplied population buffers (lbm_sc_create_with_buffers).

The two ping-pong population buffers come from a tensor allocator instead of the library. The
arithmetic does not depend on where the state lives, so such a box must end bitwise equal to
the same box on library allocations: stepped alone, replayed from a graph, and inside a group.
Bad buffers (too small, misaligned, overlapping, host memory) are rejected before any kernel
touches them.
"""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cfgs(stream):
    return [lbm.config(37, 29, 23, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.3,
                       radius=7.0, width=2.0, noise_amp=1e-6, seed=21, stream=stream)
            for prec in (lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP64)]


def torch_buffers(torch, cfg, extra=0):
    n = lbm.lbm_sc_population_bytes(cfg) + extra
    return (torch.empty(n, dtype=torch.uint8, device="cuda"),
            torch.empty(n, dtype=torch.uint8, device="cuda"))


def test_caller_buffers_step_like_library_buffers():
    import torch
    s = torch.cuda.Stream()
    for cfg in cfgs(s.cuda_stream):
        say(f"caller buffers, prec {cfg.prec}")
        with lbm.Box(cfg) as ref, lbm.Box(cfg, buffers=torch_buffers(torch, cfg)) as b:
            assert np.array_equal(b.get(), ref.get())
            # the library holds only the observation scratch of this box
            assert b.info()["device_bytes"] == (ref.info()["device_bytes"]
                                                - 2 * lbm.lbm_sc_population_bytes(cfg))
            for n in (1, 5, 64, 3):          # plain launches and graph replays
                b.step(n)
                ref.step(n)
                assert np.array_equal(b.get(), ref.get())
            o, _ = b.observables(profile=False)
            o_ref, _ = ref.observables(profile=False)
            assert o["mass"] == o_ref["mass"] and o["dP"] == o_ref["dP"]


def test_caller_buffers_inside_a_group():
    import torch
    s = torch.cuda.Stream()
    cfg = cfgs(s.cuda_stream)[0]
    with lbm.Box(cfg) as ref:
        ref.step(9)
        want = ref.get()
    bufs = torch_buffers(torch, cfg)
    boxes = [lbm.Box(cfg, buffers=bufs), lbm.Box(cfg)]
    with lbm.Group(s.cuda_stream) as g:
        g.set(boxes)
        g.step(9)
        g.set([])
    for b in boxes:
        assert np.array_equal(b.get(), want)
        b.close()


def test_bad_caller_buffers_are_rejected():
    import torch
    s = torch.cuda.Stream()
    cfg = cfgs(s.cuda_stream)[0]
    need = lbm.lbm_sc_population_bytes(cfg)
    a, b = torch_buffers(torch, cfg, extra=512)
    # host buffers on a 256-byte boundary, so that they fail the memory-type check, not alignment
    host = torch.empty(need + 256, dtype=torch.uint8)
    pinned = torch.empty(need + 256, dtype=torch.uint8, pin_memory=True)
    host_p = (host.data_ptr() + 255) // 256 * 256
    pinned_p = (pinned.data_ptr() + 255) // 256 * 256
    bad = [
        (a.data_ptr(), b.data_ptr(), need - 256, "too few bytes", "at least"),
        (a.data_ptr() + 4, b.data_ptr(), need, "misaligned", "aligned"),
        (a.data_ptr(), a.data_ptr() + 256, need, "overlapping", "overlap"),
        (a.data_ptr(), a.data_ptr(), need, "the same buffer twice", "overlap"),
        (host_p, b.data_ptr(), need, "pageable host memory", "device memory"),
        (a.data_ptr(), pinned_p, need, "pinned host memory", "device memory"),
    ]
    for pa, pb, n, why, msg in bad:
        with pytest.raises(lbm.LbmScError) as e:
            lbm.lbm_sc_create_with_buffers(cfg, pa, pb, n)
        assert e.value.code == lbm.LBM_SC_EINVAL, why
        say(f"{why}: {lbm.lbm_sc_last_error()}")
        assert msg in lbm.lbm_sc_last_error(), why
    # the good pair still works afterwards
    h = lbm.lbm_sc_create_with_buffers(cfg, a.data_ptr(), b.data_ptr(), need)
    lbm.lbm_sc_step(h, 2)
    lbm.lbm_sc_destroy(h)


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP64])
def test_no_stale_reads_with_poisoned_buffers(prec):
    """Poison check: both buffers are filled with NaN bytes before the box is created (the
    initial state then overwrites the nodes of the first, leaving its padding poisoned); after
    each of several steps the state must be finite and bitwise equal to a box on clean library
    buffers, so the step reads nothing it did not write (row padding, pitch padding and halo
    wrap included)."""
    import torch
    s = torch.cuda.Stream()
    cfg = lbm.config(37, 29, 23, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.3,
                     radius=7.0, width=2.0, noise_amp=1e-6, seed=21, stream=s.cuda_stream)
    a, b = torch_buffers(torch, cfg)
    a.fill_(0xFF)
    b.fill_(0xFF)
    torch.cuda.synchronize()
    with lbm.Box(cfg) as ref, lbm.Box(cfg, buffers=(a, b)) as box:
        for n in (1, 1, 3):
            box.step(n)
            ref.step(n)
            got = box.get()
            assert np.isfinite(got).all()
            assert np.array_equal(got, ref.get())
