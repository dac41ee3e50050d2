"""Continuous batching on the GPU: requests that arrive while others run are admitted into the
same multi-box launch, and every request's result (stop step, stop reason and final populations)
is bitwise the same as when it is served alone, also when admission is limited by memory."""
import sys

import numpy as np
import pytest

from paper_2105_08772_amd import serve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class ChunkClockGpu(serve.GpuBackend):
    """The real GPU backend with a deterministic clock: one unit of time per step chunk."""

    def __init__(self, clock, **kw):
        super().__init__(**kw)
        self.clock = clock

    def step(self, n):
        super().step(n)
        self.clock.t += 1.0


REQS = [
    dict(rid=0, L=24, radius=6.0, g_over_gc=1.3, bubble=False, seed=1, arrival=0.0),
    dict(rid=1, L=32, radius=8.0, g_over_gc=1.2, bubble=True, seed=2, arrival=0.0),  # dissolves
    dict(rid=2, L=20, radius=5.0, g_over_gc=1.5, bubble=False, seed=3, arrival=1.5),
    dict(rid=3, L=40, radius=12.0, g_over_gc=1.4, bubble=True, seed=4, arrival=3.2),
    dict(rid=4, L=36, radius=9.0, g_over_gc=1.25, bubble=False, seed=5, arrival=3.3),
]


def serve_all(reqs, budget=None, journal=None):
    clock = Clock()
    be = ChunkClockGpu(clock)
    if budget is None:
        budget = sum(be.bytes_needed(serve.Request(**r)) for r in reqs)
    srv = serve.Server(be, budget, chunk=256, observe_every=512, max_steps=40000, clock=clock,
                       sleep=clock.sleep, keep_final=True, journal=journal)
    for r in reqs:
        srv.submit(serve.Request(**r))
    recs = {r.rid: r for r in srv.run()}
    be.close()
    return recs, srv


JOURNAL = []


class ListJournal:
    def write(self, text):
        JOURNAL.append(text)

    def flush(self):
        pass


@pytest.fixture(scope="module")
def mixed():
    say("serving 5 requests together")
    return serve_all(REQS, journal=ListJournal())


def test_journal_records_every_request(mixed):
    import json
    recs, _ = mixed
    lines = [json.loads(t) for t in JOURNAL]
    assert sorted(l["rid"] for l in lines) == sorted(recs)
    for l in lines:
        r = recs[l["rid"]]
        assert l["status"] == r.status and l["steps"] == r.steps
        assert l["obs"]["dP"] == r.obs["dP"] and len(l["history"]) == r.steps // 512


def test_requests_overlap_on_the_device(mixed):
    recs, srv = mixed
    assert srv.max_active >= 3
    status = {k: r.status for k, r in recs.items()}
    assert all(v in ("converged", "evaporated") for v in status.values()), status
    assert sum(v == "converged" for v in status.values()) >= 3, status
    # the late requests were admitted while earlier ones were still running
    assert recs[2].admitted < max(recs[0].finished, recs[1].finished)
    for r in recs.values():
        say(f"request {r.rid}: L={r.L} {r.status} steps={r.steps} ({r.criterion}) "
            f"dP={r.obs['dP']:.6e} valid={r.valid} time-to-equilibrium={r.time_to_equilibrium:.1f}"
            f" chunks")


@pytest.mark.parametrize("rid", range(len(REQS)))
def test_each_request_alone_equals_in_the_mix(mixed, rid):
    recs, _ = mixed
    alone, _ = serve_all([dict(REQS[rid], arrival=0.0)])
    a, m = alone[rid], recs[rid]
    assert (a.status, a.criterion, a.steps) == (m.status, m.criterion, m.steps)
    assert np.array_equal(a.final, m.final)


def test_memory_limited_admission_gives_the_same_results(mixed):
    recs, _ = mixed
    clock = Clock()
    be = ChunkClockGpu(clock)
    sizes = sorted(be.bytes_needed(serve.Request(**r)) for r in REQS)
    be.close()
    limited, srv = serve_all(REQS, budget=sizes[-1] + sizes[-2])
    assert srv.max_active <= 2
    for rid, r in limited.items():
        assert (r.status, r.steps) == (recs[rid].status, recs[rid].steps)
        assert np.array_equal(r.final, recs[rid].final)


def test_backend_falls_back_to_xy_tiles_for_long_rows():
    """A group on full-row tiles cannot take a box whose rows are too long for the workgroup;
    the backend then switches the group to x-y tiles, stepping still equals the boxes alone, and
    the group returns to the full-row tiles once that box has left."""
    import paper_2105_08772_amd as lbm
    be = serve.GpuBackend()
    be.set_launch(rows=4, waves=8, tile_x=0, z_chunk=8, prefetch=0, persistent=0, workers=0,
                  graph_steps=0)
    small = be.create(serve.Request(rid=0, L=16, radius=4.0, g_over_gc=1.3, bubble=False, seed=1))
    cfg = lbm.config(700, 3, 2, psi=0, geom=lbm.LBM_SC_SLAB, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.3, slab_thickness=350.0, width=2.0, slab_axis=0,
                     stream=be.stream.cuda_stream)
    wide = lbm.Box(cfg)
    be.set_active([small])
    want = be.group.launch()
    assert want["tile_x"] == 0
    be.set_active([small, wide])
    assert be.group.launch()["tile_x"] == 64
    f_small, f_wide = small.get(), wide.get()
    be.step(4)
    got = [small.get(), wide.get()]
    for b, f in ((small, f_small), (wide, f_wide)):
        b.set(f)
        b.step(4)
    assert np.array_equal(got[0], small.get()) and np.array_equal(got[1], wide.get())
    be.set_active([small])
    assert be.group.launch() == want
    f_small = small.get()
    be.step(2)
    got = small.get()
    small.set(f_small)
    small.set_step(4)        # the state was 4 steps old: restores the dither's step count
    small.step(2)
    assert np.array_equal(got, small.get())
    be.group.set([])
    small.close()
    wide.close()
    be.close()
