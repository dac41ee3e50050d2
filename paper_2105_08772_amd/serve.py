"""Continuous-batching server of droplet/bubble relaxation requests on one GPU.

Requests (box size, radius, coupling, droplet or bubble) arrive over time. The server admits them
in arrival order while their device memory fits in the HBM budget, keeps every admitted box
resident, and advances all of them together with one multi-box launch per step (a group). New
requests join the group between step chunks, so their work overlaps with the boxes already on the
GPU. Every box is observed (FP64) each time its own step count reaches a multiple of the
observation interval (the paper's 2^11, Sec. 4) and is retired as soon as its stop rule holds;
its memory is then free for the next request.

Stop rule (Sec. 4 convergence criteria read for a served workload):
  evaporated - the droplet or bubble has dissolved: the density contrast between the centre and
               the far probe fell below half of its initial value (a closed box cannot sustain
               every small droplet or bubble; such runs are excluded from the analysis, as the
               paper excludes runs whose centre of mass drifts);
  converged  - between consecutive observations of the box, |dP(t) - dP(t - dt)| <= dp_tol |dP(t)|
               (the paper's criterion i), or max_x |u(t) - u(t - dt)| <= du_tol (the velocity
               criterion read as a maximum; dt is even, so the staggered momentum mode that flips
               sign every step cancels); FP64 boxes must in addition keep their mass to mass_tol;
  unstable   - the observation saw a non-finite value or n <= 0;
  step_limit - the box reached max_steps without converging;
  cancelled  - the request was cancelled (queued or running);
  failed     - the backend raised its error while creating or observing the box (the error text
               is kept as the criterion); the other requests keep being served. An error of a
               multi-box step fails every box on the GPU (each gets its record and journal line)
               and is raised again.
Converged results also carry the paper's validity flag: every coordinate of the centre of mass
within com_tol (1e-3) of the box centre.
A box's evolution and stop decision depend only on its own state and step count, so its result is
the same whether it runs alone or in the mix (the multi-box launch is bitwise equal to stepping
the box alone).

The GPU work goes through a backend object (GpuBackend below); the scheduler itself is plain
Python so that admission, cancellation and failure handling can be exercised on the CPU.
"""
import dataclasses
import json
import time


@dataclasses.dataclass
class Request:
    rid: int
    L: int
    radius: float
    g_over_gc: float
    bubble: bool
    seed: int
    arrival: float = 0.0        # seconds after the server's start
    psi: int = 0
    n_in: float = 0.0           # initial densities inside/outside; both 0: flat coexistence
    n_out: float = 0.0


@dataclasses.dataclass
class Record:
    rid: int
    L: int
    status: str = "queued"      # queued, running, converged, evaporated, unstable, step_limit,
                                # cancelled, rejected, failed
    arrival: float = 0.0
    admitted: float = None
    finished: float = None
    steps: int = 0
    bytes: int = 0
    criterion: str = None
    obs: dict = None
    final: object = None        # final populations, when the server keeps them
    contrast0: float = None     # |n_center - n_far| at admission
    valid: bool = None          # converged and centre of mass within com_tol of the centre
    history: list = dataclasses.field(default_factory=list)  # (steps, dP) at every observation

    @property
    def time_to_equilibrium(self):
        return None if self.finished is None else self.finished - self.arrival


class GpuBackend:
    """Boxes and one group on a dedicated stream of the current GPU. With single=True the active
    boxes are stepped one by one through the plain single-box path (lbm_sc_step) instead of one
    multi-box launch: the baseline the batched server is compared with."""

    def __init__(self, prec=None, stream=None, tau=1.0, width=2.0, noise_amp=1e-6, single=False,
                 packed_rows=None):
        import torch

        from . import (LBM_SC_BUBBLE, LBM_SC_DROPLET, LBM_SC_FP32_SHIFTED, Box, Group, LbmScError,
                       LBM_SC_OBS_WORKSPACE_BYTES_PER_NODE, config, lbm_sc_device_bytes)
        self._torch = torch
        self._ws = LBM_SC_OBS_WORKSPACE_BYTES_PER_NODE
        self.stream = stream or torch.cuda.Stream()
        self.prec = LBM_SC_FP32_SHIFTED if prec is None else prec
        self._Box, self._Group, self._config = Box, Group, config
        self.error = LbmScError     # the error the scheduler treats as a failed request
        self._bubble, self._droplet = LBM_SC_BUBBLE, LBM_SC_DROPLET
        self._bytes = lbm_sc_device_bytes
        self.tau, self.width, self.noise_amp = tau, width, noise_amp
        self.group = Group(self.stream.cuda_stream)
        self.launch = None
        self.single = single
        # the group's launch and the boxes' row layout, unless the caller sets them: FP32-shifted
        # boxes at tau = 1 take two steps per launch (x-y tiles, fastest on rows padded to whole
        # lines), other boxes full-row single-step tiles (fastest on rows packed at pitch nx); the
        # single-box path keeps its own x-y tiles on padded rows
        two = self.prec == LBM_SC_FP32_SHIFTED and tau == 1.0
        self.packed_rows = (not single and not two) if packed_rows is None else bool(packed_rows)
        if not single:
            self.group.set_launch(**(self.TWO_STEP if two else self.FULL_ROW))
        self.active = []
        self.fallen_back = None    # the launch shape replaced by FALLBACK, while it is replaced

    def config(self, r):
        return self._config(r.L, psi=r.psi, geom=self._bubble if r.bubble else self._droplet,
                            prec=self.prec, tau=self.tau, g_over_gc=r.g_over_gc,
                            radius=r.radius, width=self.width, noise_amp=self.noise_amp,
                            seed=r.seed, n_in=r.n_in, n_out=r.n_out,
                            stream=self.stream.cuda_stream, packed_rows=int(self.packed_rows))

    def bytes_needed(self, r):
        # the box's own memory plus a device observation workspace of its size: the boxes share
        # one workspace as large as the largest of them, so this sum over admitted boxes bounds
        # what they use
        return int(self._bytes(self.config(r))) + self._ws * r.L ** 3

    def free_bytes(self):
        free, _total = self._torch.cuda.mem_get_info()
        return int(free)

    def create(self, r):
        return self._Box(self.config(r))

    # measured on the served workload (32 Poisson requests, L ~ U{32..192}) with FP32-shifted
    # populations: p50 / p99 time to equilibrium 1.58 / 7.99 s two steps per launch in 32 x 16
    # tiles with z chunks of 16 planes on padded rows, against 1.71 / 9.75 s in single-step
    # full-row tiles (4 nodes per thread, z chunks of 8) on packed rows
    TWO_STEP = dict(rows=2, waves=8, tile_x=32, z_chunk=16, prefetch=0, persistent=0, workers=0,
                    items_per_cu=0, xcd_remap=1, steps_per_pass=2, graph_steps=64)
    FULL_ROW = dict(rows=4, waves=8, tile_x=0, z_chunk=8, prefetch=0, persistent=0, workers=0,
                    items_per_cu=0, xcd_remap=1, steps_per_pass=1, graph_steps=64)
    # single-step x-y tiles: every box fits them (full-row tiles need rows short enough for the
    # workgroup, two steps per launch FP32 boxes at tau = 1)
    FALLBACK = dict(rows=2, waves=4, tile_x=64, prefetch=0, persistent=0, steps_per_pass=1)

    def set_active(self, boxes):
        if self.single:
            self.active = list(boxes)
            return
        if self.fallen_back is not None:
            # back to the chosen shape: the box that needed x-y tiles may have left
            self.group.set([])
            self.group.set_launch(**self.fallen_back)
            self.fallen_back = None
        try:
            self.group.set(boxes)
        except self.error:
            launch = self.group.launch()
            if launch["tile_x"] != 0 and launch.get("steps_per_pass", 1) != 2:
                raise
            # a box's rows are too long for the full-row tiles, or a box cannot take two steps
            # per launch (tau != 1): switch the group to single-step x-y tiles
            self.group.set([])
            self.group.set_launch(**self.FALLBACK)
            self.fallen_back = launch   # restored by the next call, also if this set fails
            self.group.set(boxes)

    def set_launch(self, **kw):
        """Set the group's launch: the given fields over the current ones, one step per launch
        unless steps_per_pass is given."""
        self.fallen_back = None
        self.group.set_launch(**dict({"steps_per_pass": 1}, **kw))

    def step(self, n):
        if self.single:
            for b in self.active:
                b.step(n)
        else:
            self.group.step(n)

    def observe(self, box):
        obs, _ = box.observables(profile=False, raise_unstable=False)
        return obs

    def snapshot(self, box):
        return box.get()

    def destroy(self, box):
        box.close()

    def close(self):
        self.group.close()


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]


class Server:
    def __init__(self, backend, budget_bytes, chunk=512, observe_every=2048, max_steps=200000,
                 dp_tol=1e-5, du_tol=1e-9, mass_tol=None, clock=None, sleep=None, log=None,
                 keep_final=False, com_tol=1e-3, max_active=None, journal=None):
        if observe_every % chunk:
            raise ValueError("observe_every must be a multiple of chunk")
        if observe_every % 2:
            raise ValueError("observe_every must be even")
        self.b = backend
        self.budget = int(budget_bytes)
        self.chunk = chunk
        self.every = observe_every
        self.max_steps = max_steps
        self.dp_tol, self.du_tol, self.mass_tol = dp_tol, du_tol, mass_tol
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.log = log
        self.keep_final = keep_final
        self.com_tol = com_tol
        self.max_active_allowed = max_active   # None: limited by memory only
        # journal: a writable text file; one JSON line per finished request (request, status,
        # steps, times, tolerances, final observables, dP history)
        self.journal = journal
        self.queue = []            # requests not yet admitted, arrival order
        self.active = {}           # rid -> (request, box, record, last_obs)
        self.records = {}
        self.used = 0
        self.t0 = None
        self.node_steps = 0
        self.max_active = 0
        self._cancel = set()
        self._requests = {}

    # -- requests -------------------------------------------------------------------------------
    def submit(self, req):
        self.queue.append(req)
        self.queue.sort(key=lambda r: (r.arrival, r.rid))
        self.records[req.rid] = Record(rid=req.rid, L=req.L, arrival=req.arrival)
        self._requests[req.rid] = req

    def cancel(self, rid):
        self._cancel.add(rid)

    # -- loop -----------------------------------------------------------------------------------
    def _now(self):
        return self.clock() - self.t0

    def _retire(self, rid, status, criterion=None):
        req, box, rec, last = self.active.pop(rid)
        rec.status = status
        rec.criterion = criterion
        rec.finished = self._now()
        rec.obs = last
        if status == "converged" and last is not None and "com" in last:
            c = [L // 2 for L in (req.L, req.L, req.L)]
            rec.valid = all(abs(x - y) <= self.com_tol for x, y in zip(last["com"], c))
        if self.keep_final and status != "failed":
            rec.final = self.b.snapshot(box)
        self.b.destroy(box)
        self.used -= rec.bytes
        if self.log:
            self.log(f"retire {rid} L={req.L} {status} ({criterion}) steps={rec.steps} "
                     f"t={rec.finished:.3f}s")
        self._write_journal(rec)

    def _write_journal(self, rec):
        if self.journal is None:
            return
        req = self._requests.get(rec.rid)
        obs = None
        if rec.obs is not None:
            obs = {k: (list(v) if isinstance(v, (list, tuple)) else v) for k, v in rec.obs.items()
                   if isinstance(v, (int, float, list, tuple))}
        line = {"rid": rec.rid, "request": dataclasses.asdict(req) if req else None,
                "status": rec.status, "criterion": rec.criterion, "steps": rec.steps,
                "arrival_s": rec.arrival, "admitted_s": rec.admitted, "finished_s": rec.finished,
                "time_to_equilibrium_s": rec.time_to_equilibrium, "valid": rec.valid,
                "tolerances": {"dp_tol": self.dp_tol, "du_tol": self.du_tol,
                               "mass_tol": self.mass_tol, "observe_every": self.every,
                               "max_steps": self.max_steps},
                "history": rec.history, "obs": obs}
        self.journal.write(json.dumps(line) + "\n")
        self.journal.flush()

    def _fail(self, rec, err, now):
        rec.status, rec.finished, rec.criterion = "failed", now, str(err)
        if self.log:
            self.log(f"request {rec.rid} failed: {err}")
        self._write_journal(rec)

    def _admit(self):
        changed = False
        now = self._now()
        error = getattr(self.b, "error", Exception)
        while self.queue and self.queue[0].arrival <= now:
            req = self.queue[0]
            rec = self.records[req.rid]
            if req.rid in self._cancel:
                self.queue.pop(0)
                rec.status, rec.finished = "cancelled", now
                self._write_journal(rec)
                continue
            try:
                need = self.b.bytes_needed(req)
            except error as e:
                self.queue.pop(0)
                self._fail(rec, e, now)
                continue
            if need > self.budget:
                self.queue.pop(0)
                rec.status, rec.finished, rec.criterion = "rejected", now, "larger than budget"
                self._write_journal(rec)
                continue
            if self.used + need > self.budget:
                break                  # first in, first admitted: wait for memory
            if self.max_active_allowed is not None and len(self.active) >= self.max_active_allowed:
                break
            self.queue.pop(0)
            box = None
            try:
                box = self.b.create(req)
                first = self.b.observe(box)
            except error as e:
                if box is not None:
                    self.b.destroy(box)
                rec.admitted = now
                self._fail(rec, e, now)
                continue
            rec.bytes = need
            self.used += need
            rec.admitted = now
            rec.status = "running"
            rec.contrast0 = abs(first["n_center"] - first["n_far"])
            self.active[req.rid] = (req, box, rec, first)
            changed = True
            if self.log:
                self.log(f"admit {req.rid} L={req.L} at {now:.3f}s (arrived {req.arrival:.3f}s), "
                         f"{len(self.active)} active, {self.used / 2**30:.2f} GiB")
        return changed

    def _check(self, rid, obs):
        req, box, rec, last = self.active[rid]
        self.active[rid] = (req, box, rec, obs)
        rec.history.append((rec.steps, obs.get("dP")))
        if not obs["finite"]:
            return "unstable", "non-finite or n <= 0"
        if abs(obs["n_center"] - obs["n_far"]) < 0.5 * rec.contrast0:
            return "evaporated", "contrast below half"
        dP, dP0 = obs["dP"], last["dP"]
        mass_ok = self.mass_tol is None or abs(obs["mass"] - obs["mass0"]) <= self.mass_tol * obs["mass0"]
        if mass_ok and dP != 0 and abs(dP - dP0) <= self.dp_tol * abs(dP):
            return "converged", "dP"
        if mass_ok and obs["has_du"] and obs["du_max"] <= self.du_tol:
            return "converged", "du_max"
        if rec.steps >= self.max_steps:
            return "step_limit", None
        return None, None

    def run(self):
        """Serve every submitted request to completion; returns the records."""
        self.t0 = self.clock()
        members = None
        while self.queue or self.active:
            for rid in [r for r in self.active if r in self._cancel]:
                self._retire(rid, "cancelled")
            changed = self._admit()
            if not self.active:
                if self.queue:
                    wait = self.queue[0].arrival - self._now()
                    if wait > 0:
                        self.sleep(wait)
                continue
            keys = sorted(self.active)
            error = getattr(self.b, "error", Exception)
            try:
                if changed or keys != members:
                    self.b.set_active([self.active[k][1] for k in keys])
                    members = keys
                self.max_active = max(self.max_active, len(keys))
                self.b.step(self.chunk)
            except error as e:
                # the shared launch failed: no box on the GPU has a trustworthy state
                for k in keys:
                    self._retire(k, "failed", str(e))
                raise
            for k in keys:
                rec = self.active[k][2]
                rec.steps += self.chunk
                self.node_steps += self.active[k][0].L ** 3 * self.chunk
            for k in keys:
                rec = self.active[k][2]
                if rec.steps % self.every == 0:
                    try:
                        obs = self.b.observe(self.active[k][1])
                    except error as e:
                        self._retire(k, "failed", str(e))
                        continue
                    status, crit = self._check(k, obs)
                    if status:
                        self._retire(k, status, crit)
        self.wall = self._now()
        return [self.records[k] for k in sorted(self.records)]

    def summary(self):
        done = [r for r in self.records.values() if r.status == "converged"]
        tte = [r.time_to_equilibrium for r in done]
        out = {"requests": len(self.records), "converged": len(done),
               "statuses": {s: sum(1 for r in self.records.values() if r.status == s)
                            for s in sorted({r.status for r in self.records.values()})},
               "wall_s": round(self.wall, 3), "max_concurrent": self.max_active,
               "aggregate_MLUPS": round(self.node_steps / self.wall / 1e6, 1) if self.wall else None}
        if tte:
            out["p50_time_to_equilibrium_s"] = round(percentile(tte, 50), 3)
            out["p99_time_to_equilibrium_s"] = round(percentile(tte, 99), 3)
            out["mean_steps_to_converge"] = round(sum(r.steps for r in done) / len(done), 1)
        return out
