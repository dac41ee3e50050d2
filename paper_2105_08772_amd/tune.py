"""Autotuner of launch shapes: times candidate shapes on the real boxes and keeps the fastest.

Every candidate is measured with real steps of the boxes it is given (they advance the
simulation), after one untimed step that absorbs graph capture. The shapes change only the
schedule, never the results, so tuning on a running simulation is safe.
"""
import itertools
import time


def _sync():
    import torch
    torch.cuda.synchronize()


SHAPES = [dict(waves=4, rows=r, prefetch=pf, tile_x=64) for r in (1, 2, 4) for pf in (0, 1)] + \
         [dict(waves=4, rows=r, prefetch=pf, tile_x=32) for r in (1, 2) for pf in (0, 1)] + \
         [dict(waves=8, rows=r, prefetch=0, tile_x=bx) for r in (1, 2) for bx in (64, 32)] + \
         [dict(waves=8, rows=r, prefetch=0, tile_x=0) for r in (2, 4, 8)] + \
         [dict(waves=4, rows=4, prefetch=0, tile_x=0)]   # full-row tiles
# two steps per pass (single boxes, FP32 storage and arithmetic, tau = 1)
SHAPES2 = [dict(waves=8, rows=1, prefetch=pf, tile_x=64) for pf in (0, 1)] + \
          [dict(waves=16, rows=2, prefetch=0, tile_x=64)] + \
          [dict(waves=8, rows=2, prefetch=pf, tile_x=32) for pf in (0, 1)] + \
          [dict(waves=4, rows=2, prefetch=0, tile_x=32)]


def group_candidates(two_step=True):
    """Every compiled single-step shape with z chunks of 6..64 planes or per-box chunks (z_chunk
    0) of 4, 8 or 16 items per CU, one workgroup per item or persistent workers; and (two_step:
    groups of FP32 boxes at tau = 1, refused by other groups) every two-steps-per-pass shape with
    z chunks of 16..128 planes or per-box chunks, one workgroup per item."""
    out = []
    chunks = [dict(z_chunk=zc, items_per_cu=0) for zc in (6, 8, 16, 32, 64)]
    chunks += [dict(z_chunk=0, items_per_cu=k) for k in (4, 8, 16)]
    for shape, ch in itertools.product(SHAPES, chunks):
        out.append(dict(shape, **ch, xcd_remap=1, persistent=0, workers=0, steps_per_pass=1))
        for workers in (256, 512):
            out.append(dict(shape, **ch, xcd_remap=1, persistent=1, workers=workers,
                            steps_per_pass=1))
    if two_step:
        chunks2 = [dict(z_chunk=zc, items_per_cu=0) for zc in (16, 32, 64, 96, 128)]
        chunks2 += [dict(z_chunk=0, items_per_cu=k) for k in (4, 8, 16)]
        for shape, ch in itertools.product(SHAPES2, chunks2):
            out.append(dict(shape, **ch, xcd_remap=1, persistent=0, workers=0, steps_per_pass=2))
    return out


def tune_group(group, steps=8, candidates=None, log=None):
    """Try each candidate on `group` (a paper_2105_08772_amd.Group) for `steps` steps; set and
    return the fastest as a dict with its seconds per step. The group keeps its own graph chunk
    length (candidates are timed with chunks of `steps`)."""
    from . import LbmScError
    graph_steps = group.launch()["graph_steps"]
    best = None
    for cand in candidates or group_candidates():
        try:
            group.set_launch(graph_steps=steps, **cand)
        except LbmScError:
            continue               # shape not available for these boxes (e.g. rows too long)
        group.step(steps)          # warm-up: first capture and replay
        _sync()
        t0 = time.perf_counter()
        group.step(steps)
        _sync()
        t = (time.perf_counter() - t0) / steps
        if log:
            log(f"tune group {cand}: {t * 1e3:.3f} ms/step")
        if best is None or t < best[0]:
            best = (t, cand)
    if best is None:
        raise ValueError("no candidate launch shape fits the boxes of this group")
    group.set_launch(**best[1], graph_steps=graph_steps)
    return dict(best[1], seconds_per_step=best[0])


def box_candidates(nz, two_step=True):
    """Single-step shapes, and (two_step: FP32 boxes at tau = 1) the two-steps-per-pass shapes,
    each with z chunks of 8..128 planes and the XCD remap on or off."""
    out = []
    for shape, zc, remap in itertools.product(SHAPES, (8, 16, 32, 64, 128), (0, 1)):
        if zc <= max(nz, 8):
            out.append(dict(shape, z_chunk=zc, xcd_remap=remap, steps_per_pass=1))
    if two_step:
        for shape, zc, remap in itertools.product(SHAPES2, (8, 16, 32, 64, 128), (0, 1)):
            if zc <= max(nz, 8):
                out.append(dict(shape, z_chunk=zc, xcd_remap=remap, steps_per_pass=2))
    return out


def tune_box(box, steps=16, candidates=None, log=None):
    """Same for one box (a paper_2105_08772_amd.Box)."""
    from . import LbmScError
    best = None
    for cand in candidates or box_candidates(box.dims[2]):
        try:
            box.set_launch(cand["rows"], cand["z_chunk"], cand["xcd_remap"], cand["prefetch"],
                           cand["waves"], cand["tile_x"], 64, cand.get("steps_per_pass", 1))
        except LbmScError:
            continue
        box.step(2)
        _sync()
        t0 = time.perf_counter()
        box.step(steps)
        _sync()
        t = (time.perf_counter() - t0) / steps
        if log:
            log(f"tune box {cand}: {t * 1e3:.3f} ms/step")
        if best is None or t < best[0]:
            best = (t, cand)
    if best is None:
        raise ValueError("no candidate launch shape fits this box")
    c = best[1]
    box.set_launch(c["rows"], c["z_chunk"], c["xcd_remap"], c["prefetch"], c["waves"],
                   c["tile_x"], 64, c.get("steps_per_pass", 1))
    return dict(c, seconds_per_step=best[0])
