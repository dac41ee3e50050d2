"""Scheduler of the continuous-batching server, exercised on the CPU with a scripted backend:
admission by memory in arrival order, retirement on the stop rule, unstable and cancelled
requests, step limit, rejection, and the bookkeeping of time to equilibrium."""
import math

import pytest

from paper_2105_08772_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBox:
    def __init__(self, req):
        self.req = req
        self.steps = 0


class ScriptedBackend:
    """dP relaxes as dP_inf (1 + exp(-steps / relax)); boxes named in `fail_at` turn non-finite
    at that step; each step call advances the clock by `dt` per chunk."""

    def __init__(self, clock, dt=1.0, relax=None, fail_at=None, never=(), evaporate=None):
        self.clock, self.dt = clock, dt
        self.evaporate = evaporate or {}
        self.relax = relax or {}
        self.fail_at = fail_at or {}
        self.never = set(never)
        self.active = []
        self.live = set()
        self.hook = None

    def bytes_needed(self, r):
        return r.L ** 3

    def create(self, r):
        b = FakeBox(r)
        self.live.add(r.rid)
        return b

    def set_active(self, boxes):
        self.active = list(boxes)

    def step(self, n):
        for b in self.active:
            b.steps += n
        self.clock.t += self.dt
        if self.hook:
            self.hook()

    def observe(self, b):
        rid = b.req.rid
        finite = not (rid in self.fail_at and b.steps >= self.fail_at[rid])
        if rid in self.never:
            dP = 1.0 + 0.5 * (b.steps // 2048 % 2)  # alternates between observations forever
        else:
            dP = 1.0 + math.exp(-b.steps / self.relax.get(rid, 1000.0))
        gone = rid in self.evaporate and b.steps >= self.evaporate[rid]
        return dict(finite=int(finite), dP=dP, has_du=1, du_max=1.0, mass=1.0, mass0=1.0,
                    n_center=0.4 if gone else 2.5, n_far=0.4, com=[b.req.L // 2] * 3)

    def destroy(self, b):
        self.live.discard(b.req.rid)

    def snapshot(self, b):
        return b.steps


def make(requests, budget, **kw):
    clock = Clock()
    be = ScriptedBackend(clock, **{k: kw.pop(k) for k in list(kw) if k in
                                   ("dt", "relax", "fail_at", "never", "evaporate")})
    srv = serve.Server(be, budget, chunk=512, observe_every=2048, clock=clock, sleep=clock.sleep,
                       **kw)
    for r in requests:
        srv.submit(r)
    return srv, be, clock


def req(rid, L, arrival):
    return serve.Request(rid=rid, L=L, radius=L / 4, g_over_gc=1.3, bubble=False, seed=rid,
                         arrival=arrival)


def test_admission_by_memory_in_arrival_order():
    reqs = [req(k, 10, 0.0) for k in range(5)]
    srv, be, _ = make(reqs, budget=2 * 1000)
    recs = srv.run()
    assert srv.max_active == 2
    assert all(r.status == "converged" for r in recs)
    admitted = sorted(recs, key=lambda r: r.admitted)
    assert [r.rid for r in admitted] == [0, 1, 2, 3, 4]
    assert srv.used == 0 and not be.live
    for r in recs:
        assert r.time_to_equilibrium == r.finished - r.arrival


def test_one_at_a_time_serving():
    """max_active = 1 (the single-box baseline): requests run strictly one after another in
    arrival order even when memory would admit more, and each waits for the previous one."""
    reqs = [req(k, 10, 0.1 * k) for k in range(4)]
    srv, be, _ = make(reqs, budget=10 ** 6, max_active=1)
    recs = sorted(srv.run(), key=lambda r: r.rid)
    assert srv.max_active == 1
    assert all(r.status == "converged" for r in recs)
    for a, b in zip(recs, recs[1:]):
        assert b.admitted >= a.finished
    assert recs[-1].time_to_equilibrium > recs[0].time_to_equilibrium


def test_unstable_request_is_retired_and_others_continue():
    reqs = [req(k, 10, 0.0) for k in range(3)]
    srv, be, _ = make(reqs, budget=10 ** 6, fail_at={1: 4096})
    recs = {r.rid: r for r in srv.run()}
    assert recs[1].status == "unstable" and recs[1].steps == 4096
    assert recs[0].status == "converged" and recs[2].status == "converged"
    assert not be.live and srv.used == 0


def test_evaporated_request_is_retired_and_flagged():
    reqs = [req(k, 10, 0.0) for k in range(3)]
    srv, be, _ = make(reqs, budget=10 ** 6, evaporate={2: 2048})
    recs = {r.rid: r for r in srv.run()}
    assert recs[2].status == "evaporated" and recs[2].steps == 2048
    assert recs[0].status == "converged" and recs[0].valid is True
    assert recs[2].valid is None


def test_cancel_queued_and_running_requests():
    reqs = [req(k, 10, 0.0) for k in range(4)]
    srv, be, clock = make(reqs, budget=2 * 1000)
    srv.cancel(3)                               # still queued when the loop starts

    def hook():
        if clock.t >= 2.0:
            srv.cancel(0)                       # running
    be.hook = hook
    recs = {r.rid: r for r in srv.run()}
    assert recs[3].status == "cancelled" and recs[3].admitted is None
    assert recs[0].status == "cancelled" and recs[0].admitted is not None
    assert recs[1].status == "converged" and recs[2].status == "converged"
    assert not be.live


def test_step_limit_and_rejection():
    reqs = [req(0, 10, 0.0), req(1, 100, 0.0), req(2, 10, 0.5)]
    srv, be, _ = make(reqs, budget=5000, never={0}, max_steps=8192, relax={2: 200.0})
    recs = {r.rid: r for r in srv.run()}
    assert recs[0].status == "step_limit" and recs[0].steps == 8192
    assert recs[1].status == "rejected"
    assert recs[2].status == "converged"


def test_late_arrivals_wait_and_join_running_boxes():
    reqs = [req(0, 10, 0.0), req(1, 10, 2.5), req(2, 10, 40.0)]
    srv, be, clock = make(reqs, budget=10 ** 6, relax={0: 4000.0, 1: 500.0, 2: 500.0})
    recs = {r.rid: r for r in srv.run()}
    assert recs[1].admitted >= 2.5 and recs[1].admitted < recs[0].finished   # overlapped
    assert recs[2].admitted >= 40.0                                          # idle wait
    s = srv.summary()
    assert s["converged"] == 3 and s["p50_time_to_equilibrium_s"] > 0


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serve.percentile(v, 50) == 50
    assert serve.percentile(v, 99) == 99
    assert serve.percentile([3.0], 99) == 3.0
    assert serve.percentile([1, 2, 3, 4], 50) == 2


def test_journal_has_one_json_line_per_request():
    import io
    import json
    buf = io.StringIO()
    reqs = [req(0, 10, 0.0), req(1, 10, 0.0), req(2, 10**3, 0.0), req(3, 10, 0.0)]
    srv, be, clock = make(reqs, budget=5000, relax={0: 300.0, 1: 300.0}, fail_at={3: 4096},
                          journal=buf)
    srv.cancel(1)
    srv.run()
    lines = [json.loads(l) for l in buf.getvalue().splitlines()]
    assert sorted(l["rid"] for l in lines) == [0, 1, 2, 3]
    by = {l["rid"]: l for l in lines}
    assert by[0]["status"] == "converged" and by[0]["criterion"] == "dP"
    assert by[0]["request"]["L"] == 10 and by[0]["tolerances"]["dp_tol"] == 1e-5
    assert [h[0] for h in by[0]["history"]] == list(range(2048, by[0]["steps"] + 1, 2048))
    assert by[0]["obs"]["dP"] == by[0]["history"][-1][1]
    assert by[0]["time_to_equilibrium_s"] > 0
    assert by[1]["status"] == "cancelled" and by[2]["status"] == "rejected"
    assert by[3]["status"] == "unstable" and by[3]["history"][-1][0] == 4096


def test_backend_leaves_the_xy_tile_fallback_when_the_wide_box_leaves():
    """GpuBackend.set_active on a stand-in group: a box too wide for the full-row tiles switches
    the group to x-y tiles; once it has left, the chosen full-row shape comes back."""
    from paper_2105_08772_amd import LbmScError

    class FakeGroup:
        def __init__(self):
            self.shape = dict(tile_x=0, rows=4, waves=8, z_chunk=8, prefetch=0, persistent=0,
                              steps_per_pass=1)
            self.boxes = []

        def set(self, boxes):
            if self.shape["tile_x"] == 0 and "wide" in boxes:
                raise LbmScError(-1, "rows too long for full-row tiles")
            self.boxes = list(boxes)

        def set_launch(self, **kw):
            assert not self.boxes
            self.shape.update(kw)

        def launch(self):
            return dict(self.shape)

    be = object.__new__(serve.GpuBackend)
    be.single, be.group, be.fallen_back, be.error = False, FakeGroup(), None, LbmScError
    chosen = be.group.launch()
    be.set_active(["small"])
    assert be.group.launch() == chosen
    be.set_active(["small", "wide"])
    assert be.group.launch()["tile_x"] == 64 and be.group.boxes == ["small", "wide"]
    be.set_active(["small", "wide", "other"])
    assert be.group.launch()["tile_x"] == 64
    be.set_active(["small"])
    assert be.group.launch() == chosen and be.group.boxes == ["small"]


def test_backend_leaves_two_steps_per_launch_for_a_box_that_cannot_take_them():
    """A box the two-step group refuses (tau != 1) switches the group to single-step x-y
    tiles; once it has left, the two-step launch comes back; other refusals propagate."""
    from paper_2105_08772_amd import LbmScError

    class FakeGroup:
        def __init__(self):
            self.shape = dict(tile_x=32, rows=2, waves=8, z_chunk=16, prefetch=0, persistent=0,
                              steps_per_pass=2)
            self.boxes = []

        def set(self, boxes):
            if self.shape["steps_per_pass"] == 2 and "tau08" in boxes:
                raise LbmScError(-1, "two steps per pass need tau = 1")
            if "bad" in boxes:
                raise LbmScError(-1, "a box was not created on the group's stream")
            self.boxes = list(boxes)

        def set_launch(self, **kw):
            assert not self.boxes
            self.shape.update(kw)

        def launch(self):
            return dict(self.shape)

    be = object.__new__(serve.GpuBackend)
    be.single, be.group, be.fallen_back, be.error = False, FakeGroup(), None, LbmScError
    chosen = be.group.launch()
    be.set_active(["a", "tau08"])
    assert be.group.launch()["steps_per_pass"] == 1 and be.group.boxes == ["a", "tau08"]
    be.set_active(["a"])
    assert be.group.launch() == chosen and be.group.boxes == ["a"]
    with pytest.raises(LbmScError):
        be.set_active(["a", "bad"])
    be.set_active(["a"])                 # the chosen launch comes back after a failed set
    assert be.group.launch() == chosen and be.group.boxes == ["a"]


class BackendError(RuntimeError):
    pass


class FailingBackend(ScriptedBackend):
    """The scripted backend whose calls raise its error for chosen requests: bytes_needed, create
    or the first observation at admission, an observation at a given step, or a multi-box step
    once a given clock time is reached."""
    error = BackendError

    def __init__(self, clock, fail_bytes=(), fail_create=(), fail_first_obs=(), fail_obs_at=None,
                 fail_step_at=None, **kw):
        super().__init__(clock, **kw)
        self.fail_bytes, self.fail_create = set(fail_bytes), set(fail_create)
        self.fail_first_obs = set(fail_first_obs)
        self.fail_obs_at = fail_obs_at or {}
        self.fail_step_at = fail_step_at

    def bytes_needed(self, r):
        if r.rid in self.fail_bytes:
            raise BackendError(f"invalid configuration of request {r.rid}")
        return super().bytes_needed(r)

    def create(self, r):
        if r.rid in self.fail_create:
            raise BackendError("out of device memory")
        return super().create(r)

    def observe(self, b):
        rid = b.req.rid
        if rid in self.fail_first_obs and b.steps == 0:
            raise BackendError("observation failed")
        if rid in self.fail_obs_at and b.steps >= self.fail_obs_at[rid]:
            raise BackendError("observation failed")
        return super().observe(b)

    def step(self, n):
        if self.fail_step_at is not None and self.clock.t >= self.fail_step_at:
            raise BackendError("launch failed")
        super().step(n)


class ListJournal:
    def __init__(self):
        self.lines = []

    def write(self, text):
        self.lines.append(text)

    def flush(self):
        pass


def test_backend_errors_at_admission_fail_only_that_request():
    """A request whose memory estimate, creation or first observation raises the backend's
    error is recorded as failed (with the error text and a journal line) and holds no memory;
    a box created before the failing observation is destroyed; the others are served."""
    import json
    clock = Clock()
    be = FailingBackend(clock, fail_bytes={1}, fail_create={2}, fail_first_obs={3})
    journal = ListJournal()
    srv = serve.Server(be, 10 ** 6, chunk=512, observe_every=2048, clock=clock, sleep=clock.sleep,
                       journal=journal)
    for k in range(5):
        srv.submit(req(k, 10, 0.1 * k))
    recs = {r.rid: r for r in srv.run()}
    assert recs[0].status == "converged" and recs[4].status == "converged"
    for rid, text in ((1, "invalid configuration"), (2, "out of device memory"),
                      (3, "observation failed")):
        assert recs[rid].status == "failed" and text in recs[rid].criterion, rid
        assert recs[rid].bytes == 0 and recs[rid].finished is not None
    assert srv.used == 0 and not be.live
    lines = [json.loads(x) for x in journal.lines]
    assert sorted(x["rid"] for x in lines) == [0, 1, 2, 3, 4]
    assert {x["rid"]: x["status"] for x in lines}[2] == "failed"


def test_backend_error_while_observing_a_running_box():
    clock = Clock()
    # request 1 never converges by itself; its observation at step 4096 raises
    be = FailingBackend(clock, fail_obs_at={1: 4096}, never={1})
    srv = serve.Server(be, 10 ** 6, chunk=512, observe_every=2048, clock=clock, sleep=clock.sleep)
    for k in range(3):
        srv.submit(req(k, 10, 0.0))
    recs = {r.rid: r for r in srv.run()}
    assert recs[1].status == "failed" and recs[1].steps == 4096
    assert recs[0].status == recs[2].status == "converged"
    assert srv.used == 0 and not be.live


def test_backend_error_of_the_shared_step_fails_every_running_box_and_is_raised():
    clock = Clock()
    be = FailingBackend(clock, fail_step_at=2.0)
    journal = ListJournal()
    srv = serve.Server(be, 10 ** 6, chunk=512, observe_every=2048, clock=clock, sleep=clock.sleep,
                       journal=journal, keep_final=True)
    for k in range(3):
        srv.submit(req(k, 10, 0.0))
    with pytest.raises(BackendError):
        srv.run()
    assert all(srv.records[k].status == "failed" for k in range(3))
    assert all(srv.records[k].final is None for k in range(3))
    assert len(journal.lines) == 3 and srv.used == 0 and not be.live
