#!/usr/bin/env python3
"""Benchmark of the fused D3Q19 Shan-Chen lattice Boltzmann step on one MI355X.

Workload (default): one droplet in a 256^3 periodic box, FP32-shifted populations, psi =
exp(-1/n), G = 1.3 G_c, radius 60, tanh width 2, seeded uniform noise 1e-6 (seed 3), tau = 1.
A step is one fused time step of the whole box; every 2048 steps (the paper's convergence
interval 2^11) the run-control loop takes the FP64 observables, as it would to test convergence.
The state is created on the device before timing and stays resident in HBM.

Prints ONE JSON line with MLUPS (million lattice-node updates per second), the roofline of the
step kernel (algorithmic bytes 2 * 19 * 4 B per node update against 8 TB/s), and the oracle
timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("MLUPS + % of HBM roofline (1 GPU); batched droplets/hour and p50/p99 "
          "time-to-equilibrium")
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_droplet256_fp32.json")
GROUP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_group64_fp32.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_2105_08772_amd", "csrc", n)
              for n in ("step_kernels.hpp", "kernels.hpp", "d3q19.hpp")]
# the multi-box launches also depend on the host's work list and item order
GROUP_SRC = KERNEL_SRC + [os.path.join(ROOT, "paper_2105_08772_amd", "csrc", "lbm_sc.hip")]
GROUP_NODES = 102318059      # the batched mix (seed 2105)


def kernel_hash(paths=None):
    """Hash of the sources of the step kernels (their template code, layout and constants), or
    of the given files."""
    h = hashlib.sha256()
    for p in paths or KERNEL_SRC:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def group_hash():
    """Hash of the step kernels and of the host code that builds a group's work list."""
    return kernel_hash(GROUP_SRC)


def measured_traffic(nodes, prec, launch):
    """HBM bytes per step launch from committed rocprofv3 counter summaries, if they were taken
    on the current kernel source, precision and launch shape (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    shape = {k: v for k, v in launch.items() if k != "graph_steps"}   # replay changes no kernel
    if (t.get("kernel_sha256_16") != kernel_hash() or t.get("nodes") != nodes
            or t.get("prec") != prec or t.get("launch") != shape):
        return None
    return t.get("bytes_per_launch")


def counter_per_dispatch(run_dir, counter, kernel_prefix, last=None):
    """Median and count of one rocprofv3 counter (`--pmc COUNTER --output-format csv`) over the
    dispatches of kernels whose name starts with kernel_prefix (rows of one dispatch summed);
    `last`: only the last that many dispatches."""
    import csv
    import glob
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    per = {}
    for fn in files:
        with open(fn, newline="") as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter or not row["Kernel_Name"].startswith(kernel_prefix):
                    continue
                key = (fn, int(row["Dispatch_Id"]))
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    vals = [v for _, v in sorted(per.items())]
    if last:
        vals = vals[-last:]
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel_prefix} under {run_dir}")
    mid = sorted(vals)
    n = len(mid)
    med = mid[n // 2] if n % 2 else 0.5 * (mid[n // 2 - 1] + mid[n // 2])
    return float(med), n


def traffic_summary(prof_dir, bench_log, out_path):
    """HBM bytes per launch of the single-box step from four counter runs under prof_dir
    (pmc_FETCH_SIZE_step, pmc_WRITE_SIZE_step: the benchmark's step; pmc_FETCH_SIZE_copy,
    pmc_WRITE_SIZE_copy: the library's dword streaming copy of 1 GiB each way). Each counter is
    scaled by what it reads for the copy, whose bytes are known; the record carries the hash of
    the step kernels' sources and the launch shape, so the benchmark uses it only for that
    kernel. bench_log: the step run's output, whose last line is its JSON result."""
    with open(bench_log) as fh:
        res = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    copy_bytes = 1 << 30
    cf, ncf = counter_per_dispatch(os.path.join(prof_dir, "pmc_FETCH_SIZE_copy"), "FETCH_SIZE",
                                   "void lbm::(anonymous namespace)::k_stream_copy<")
    cw, ncw = counter_per_dispatch(os.path.join(prof_dir, "pmc_WRITE_SIZE_copy"), "WRITE_SIZE",
                                   "void lbm::(anonymous namespace)::k_stream_copy<")
    spp = res["config"]["launch"].get("steps_per_pass", 1)
    kernel = "void lbm::(anonymous namespace)::" + ("k_step2<" if spp == 2 else "k_step<")
    sf, nsf = counter_per_dispatch(os.path.join(prof_dir, "pmc_FETCH_SIZE_step"), "FETCH_SIZE",
                                   kernel)
    sw, nsw = counter_per_dispatch(os.path.join(prof_dir, "pmc_WRITE_SIZE_step"), "WRITE_SIZE",
                                   kernel)
    fscale, wscale = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    fb, wb = sf * 1024 * fscale, sw * 1024 * wscale
    launch = {k: v for k, v in res["config"]["launch"].items()
              if k not in ("graph_steps", "block", "tuned")}
    rec = {"kernel": "single-box fused step, 256^3 FP32-shifted droplet, default launch shape",
           "nodes": res["config"]["nodes"], "prec": "fp32", "launch": launch,
           "steps_per_launch": spp,
           "kernel_sha256_16": kernel_hash(),
           "FETCH_SIZE_KiB_per_dispatch": round(sf, 1), "WRITE_SIZE_KiB_per_dispatch": round(sw, 1),
           "copy_FETCH_SIZE_KiB_per_1GiB": round(cf, 1), "copy_WRITE_SIZE_KiB_per_1GiB": round(cw, 1),
           "fetch_scale": round(fscale, 5), "write_scale": round(wscale, 5),
           "fetch_bytes_per_launch": int(fb), "write_bytes_per_launch": int(wb),
           "bytes_per_launch": int(fb + wb),
           "algorithmic_bytes_per_launch": res["roofline"]["bytes_per_launch"],
           "dispatches": {"step_fetch": nsf, "step_write": nsw, "copy_fetch": ncf,
                          "copy_write": ncw}}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    alg = rec["algorithmic_bytes_per_launch"] / 2
    print(json.dumps(rec, indent=1))
    print(f"reads {fb / alg:.4f} x, writes {wb / alg:.4f} x the algorithmic bytes "
          f"({spp} step(s) per launch)")


def group_traffic(prof_dir, bench_log=None, timed_steps=256 + 128, out_path=None):
    """The same scaling for the multi-box step's counter runs (pmc_FETCH_SIZE_group,
    pmc_WRITE_SIZE_group), over the dispatches of the timed mix: its `timed_steps` steps (the
    256 steps of the counted run and the 128-step kernel timing), one dispatch per step, or per
    two steps when the tuned launch (from the counted run's bench line in bench_log) takes two
    steps per pass. Printed; with bench_log and out_path also written as the record the batched
    leg reads (keyed by the tuned launch and the group sources' hash)."""
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    spp, launch = 1, None
    if bench_log:
        with open(bench_log) as fh:
            res = json.loads([ln for ln in fh if ln.startswith("{")][-1])
        launch = res["batched"]["launch"]
        spp = launch.get("steps_per_pass", 1)
    kernel = "void lbm::(anonymous namespace)::" + ("k_step2_group<" if spp == 2 else "k_step_group<")
    out = {"kernel": kernel, "steps_per_launch": spp}
    for counter, scale in (("FETCH_SIZE", t["fetch_scale"]), ("WRITE_SIZE", t["write_scale"])):
        v, n = counter_per_dispatch(os.path.join(prof_dir, f"pmc_{counter}_group"), counter,
                                    kernel, timed_steps // spp)
        out[counter] = {"KiB_per_dispatch": round(v, 1), "bytes_per_launch": int(v * 1024 * scale),
                        "bytes_per_step": int(v * 1024 * scale / spp), "dispatches": n}
    print(json.dumps(out, indent=1))
    if out_path and launch is not None:
        rec = {"kernel": "multi-box step, batched 64-box mix (seed 2105), tuned launch",
               "nodes": GROUP_NODES, "launch": launch, "steps_per_launch": spp,
               "group_sha256_16": group_hash(),
               "fetch_scale": t["fetch_scale"], "write_scale": t["write_scale"],
               "FETCH_SIZE_KiB_per_dispatch": out["FETCH_SIZE"]["KiB_per_dispatch"],
               "WRITE_SIZE_KiB_per_dispatch": out["WRITE_SIZE"]["KiB_per_dispatch"],
               "fetch_bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"],
               "write_bytes_per_launch": out["WRITE_SIZE"]["bytes_per_launch"],
               "bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"]
               + out["WRITE_SIZE"]["bytes_per_launch"],
               "algorithmic_bytes_per_launch": 2 * 19 * 4 * GROUP_NODES * spp,
               "dispatches": n}
        with open(out_path, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")


def measured_group_traffic(nodes, launch):
    """HBM bytes per multi-box launch from the committed group counter record, if it was taken
    on the current group sources, the same mix and the same launch (else None)."""
    try:
        with open(GROUP_TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if (t.get("group_sha256_16") != group_hash() or t.get("nodes") != nodes
            or t.get("launch") != launch):
        return None
    return t.get("bytes_per_launch")


def stream_copy_gbps(torch, lbm, stream, nbytes=2 << 30, reps=20):
    """Achievable HBM bandwidth: the library's streaming copy of a 2 GiB buffer with 4-, 8- and
    16-byte lanes, counted as read + write bytes, and torch's device-to-device copy for
    comparison; "best" is the fastest of them."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    out = {}
    runs = {f"lbm_sc_stream_copy_{w}B": w for w in (4, 8, 16)}
    runs["torch_copy"] = None
    for name, lane in runs.items():
        def run():
            if lane is None:
                with torch.cuda.stream(stream):
                    b.copy_(a)
            else:
                lbm.lbm_sc_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream,
                                       lane_bytes=lane)
        for _ in range(3):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / 1e3 / reps
        out[name] = round(2 * nbytes / s / 1e9, 1)
    out["best"] = max(out.values())
    del a, b
    torch.cuda.empty_cache()
    return out


HELD_OUT_SEED = 2106


def run_batched(args, torch, lbm, stream, steps, log):
    """The batched workload: 64 cubic boxes (L ~ U{48..160}, R ~ U[0.15, 0.35] L, G/G_c ~
    U[1.05, 1.8], droplet or bubble, exp psi, FP32-shifted, tanh width 2, noise 1e-6), seeded
    2105, advanced together by one multi-box launch per step (or per two steps) with a launch
    shape and row layout autotuned on a held-out mix of the same distribution (seed 2106), and
    FP64 observations of every box every 2048 steps. Compared with the plain single-box FP64 path on a subset of the same boxes
    (throughput and dP after the same number of steps)."""
    from tests import inputs
    from paper_2105_08772_amd import tune
    spec = inputs.batched_boxes()

    def cfg(b, prec, st, packed=0):
        return lbm.config(b["L"], psi=lbm.LBM_SC_PSI_EXP,
                          geom=lbm.LBM_SC_BUBBLE if b["bubble"] else lbm.LBM_SC_DROPLET,
                          prec=prec, tau=1.0, g_over_gc=b["g_over_gc"], radius=b["radius"],
                          width=2.0, noise_amp=1e-6, seed=b["seed"], stream=st,
                          packed_rows=packed)

    # the launch shape is tuned on a held-out mix, so that the timed boxes are unseen by the tuner:
    # the single-step shapes on boxes whose rows are packed (pitch nx, no lanes idle over row
    # padding under full-row tiles), the two-steps-per-pass shapes (x-y tiles) on the same boxes
    # with rows padded to whole lines; the timed boxes take the row layout of the winner. The
    # single-box FP64 comparison keeps the default padded rows.
    held_spec = inputs.batched_boxes(seed=HELD_OUT_SEED)
    tuned = []
    for packed, spp in ((1, 1), (0, 2)):
        held = [lbm.Box(cfg(b, lbm.LBM_SC_FP32_SHIFTED, stream.cuda_stream, packed))
                for b in held_spec]
        hgroup = lbm.Group(stream.cuda_stream)
        hgroup.set(held)
        log(f"# batched: tuning {'single-step' if spp == 1 else 'two-step'} shapes on the held-out "
            f"mix (seed {HELD_OUT_SEED}, {hgroup.info()['nodes'] / 1e6:.1f} M nodes, packed rows "
            f"{packed})")
        cands = [c for c in tune.group_candidates() if c["steps_per_pass"] == spp]
        tuned.append(dict(tune.tune_group(hgroup, steps=8, candidates=cands,
                                          log=lambda m: log("# " + m)), packed_rows=packed))
        hgroup.close()
        for b in held:
            b.close()
        del held
        torch.cuda.empty_cache()
    best = min(tuned, key=lambda t: t["seconds_per_step"])
    log(f"# batched: tuned {best}")
    packed = best["packed_rows"]
    boxes = [lbm.Box(cfg(b, lbm.LBM_SC_FP32_SHIFTED, stream.cuda_stream, packed)) for b in spec]
    group = lbm.Group(stream.cuda_stream)
    group.set(boxes)
    ginfo = group.info()
    launch = {k: v for k, v in best.items() if k not in ("seconds_per_step", "packed_rows")}
    group.set_launch(**launch, graph_steps=64)
    log(f"# batched: {len(boxes)} boxes, {ginfo['nodes'] / 1e6:.1f} M nodes")
    # timed: `steps` steps of all boxes, FP64 observation of every box every 2048 steps
    for b in boxes:
        b.observables(profile=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(2048 - done % 2048, steps - done)
        group.step(n)
        done += n
        if done % 2048 == 0:
            for b in boxes:
                b.observables(profile=False, raise_unstable=False)
            if done % 8192 == 0:
                log(f"# batched: {done} of {steps} steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel time of one group step (graph replays, no observations)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    group.step(128)
    e1.record(stream)
    torch.cuda.synchronize()
    t_step = e0.elapsed_time(e1) / 1e3 / 128
    obs32 = [b.observables(profile=False, raise_unstable=False)[0] for b in boxes]
    steps_done = boxes[0].observables(profile=False, raise_unstable=False)[0]["step"]
    unstable = sum(1 for o in obs32 if not o["finite"])
    # plain single-box FP64 path on a subset, same number of steps from the same initial state
    subset = list(range(0, len(spec), 8))
    fp64 = []
    fp64_time = 0.0
    fp64_nodes = 0
    for k in subset:
        with lbm.Box(cfg(spec[k], lbm.LBM_SC_FP64, stream.cuda_stream)) as b64:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            b64.step(steps_done)
            torch.cuda.synchronize()
            fp64_time += time.perf_counter() - t1
            fp64_nodes += spec[k]["L"] ** 3
            o64 = b64.observables(profile=False, raise_unstable=False)[0]
            info64 = b64.info()
            # dissolved (R21): the centre/far contrast fell below half the initial one
            o64["dissolved"] = (abs(o64["n_center"] - o64["n_far"])
                                < 0.5 * abs(info64["n_in"] - info64["n_out"]))
            fp64.append(o64)
    dP_err = [abs(obs32[k]["dP"] - o["dP"]) / abs(o["dP"]) for k, o in zip(subset, fp64)
              if o["finite"] and obs32[k]["finite"] and o["dP"] != 0 and not o["dissolved"]]
    per_box = [dict(L=spec[k]["L"], bubble=spec[k]["bubble"], g_over_gc=round(spec[k]["g_over_gc"], 4),
                    dP_fp32=obs32[k]["dP"], dP_fp64=o["dP"], dissolved=o["dissolved"])
               for k, o in zip(subset, fp64)]
    group.close()
    for b in boxes:
        b.close()
    torch.cuda.empty_cache()
    total_nodes = ginfo["nodes"]
    mlups = total_nodes * steps / wall / 1e6
    mlups64 = fp64_nodes * steps_done / fp64_time / 1e6
    solve_steps = 20000
    return {
        "workload": "64 boxes L~U{48..160}, R~U[0.15,0.35]L, G/G_c~U[1.05,1.8], droplet/bubble, "
                    "exp psi, FP32-shifted, seed 2105, one multi-box launch per step or per two "
                    "steps (tuned), FP64 observations every 2048 steps",
        "boxes": len(boxes), "nodes": total_nodes, "steps": steps, "seconds": round(wall, 3),
        "MLUPS": round(mlups, 1),
        "droplets_per_hour": round(len(boxes) * 3600.0 / (wall * solve_steps / steps), 1),
        "kernel_ms_per_step": round(t_step * 1e3, 4),
        "kernel_GBps": round(ginfo["bytes_per_step"] / t_step / 1e9, 1),
        "kernel_frac_of_8TBps": round(ginfo["bytes_per_step"] / t_step / 1e9 / HBM_PEAK_GBPS, 4),
        # HBM bytes per launch (one or two steps) from the committed counter record of this mix
        # and launch, null when the record does not match
        "steps_per_launch": launch.get("steps_per_pass", 1),
        "traffic_bytes_per_launch": measured_group_traffic(total_nodes, dict(launch, packed_rows=packed)),
        "launch": dict(launch, packed_rows=packed),
        "tuned_ms_per_step": {("two_step" if t["steps_per_pass"] == 2 else "single_step"):
                              round(t["seconds_per_step"] * 1e3, 4) for t in tuned},
        "launch_tuned_on": f"held-out mix of the same distribution, seed {HELD_OUT_SEED}",
        "unstable_boxes": unstable,
        "fp64_single_path": {"boxes": len(subset), "MLUPS": round(mlups64, 1),
                             "droplets_per_hour": round(3600.0 / (total_nodes * solve_steps /
                                                                  (mlups64 * 1e6)) * len(boxes), 1),
                             "dP_rel_err_fp32_vs_fp64_max": max(dP_err) if dP_err else None,
                             "dP_rel_err_fp32_vs_fp64_median": float(sorted(dP_err)[len(dP_err) // 2])
                             if dP_err else None,
                             "steps_compared": steps_done,
                             "boxes_compared": len(dP_err),
                             "per_box": per_box},
        "speedup_vs_fp64_single": round(mlups / mlups64, 2),
    }


def run_served(args, torch, lbm, log, capacity_mlups=None):
    """The served workload: seeded Poisson arrivals of droplet/bubble requests (L ~ U{32..192},
    radius ~ U[max(6, 0.15 L), min(60, 0.35 L)], G/G_c ~ U[1.05, 1.8], exp psi, FP32-shifted),
    continuously batched into one multi-box launch per two steps, admitted by free HBM (less an 8 GiB
    reserve), each run until its stop rule holds (dP change < 1e-5 or max |du| < 1e-9 between
    observations 2048 steps apart; at most 100000 steps). Reports p50/p99 time to equilibrium
    and aggregate MLUPS. The same requests with the same arrivals and stop rule are then served
    by the plain single-box FP64 path, first come first served, one box at a time (measured, not
    modelled), and each request's converged dP is compared between the two. The offered load is
    the arrival rate times the mean work of a request (nodes x steps it ran), stated against the
    batched workload's throughput when that ran in the same invocation."""
    from tests import inputs
    from paper_2105_08772_amd import serve
    rate = args.served_rate
    spec = inputs.served_requests(seed=8772, count=args.served_count, rate=rate)

    def serve_all(backend, journal=None, **kw):
        budget = backend.free_bytes() - (8 << 30)
        srv = serve.Server(backend, budget, chunk=512, observe_every=2048, max_steps=100000,
                           dp_tol=1e-5, du_tol=1e-9, log=log, journal=journal, **kw)
        for r in spec:
            srv.submit(serve.Request(**r))
        recs = srv.run()
        backend.close()
        torch.cuda.empty_cache()
        return srv, recs, budget

    # the backend's default for FP32-shifted boxes at tau = 1: two steps per launch in 32 x 16
    # tiles on rows padded to whole lines, z chunks of 16 planes (a few boxes at a time: short
    # chunks keep every CU busy)
    be = serve.GpuBackend()
    assert be.group.launch()["steps_per_pass"] == 2 and not be.packed_rows
    journal = open(args.served_journal, "w") if args.served_journal else None
    srv, recs, budget = serve_all(be, journal=journal)
    if journal:
        journal.close()
    summ = srv.summary()
    log("served: FP64 single-box path, one request at a time")
    # the FP64 boxes must also keep their mass to 1e-12 (the served configuration's mass gate)
    srv64, recs64, _ = serve_all(serve.GpuBackend(prec=lbm.LBM_SC_FP64, single=True), max_active=1,
                                 mass_tol=1e-12)
    summ64 = srv64.summary()
    errs = []
    for a, b in zip(recs, recs64):
        if a.status == "converged" and b.status == "converged":
            errs.append(abs(a.obs["dP"] - b.obs["dP"]) / abs(b.obs["dP"]))
    work = [r.L ** 3 * r.steps for r in recs]
    offered = rate * sum(work) / len(work) / 1e6 if work else 0.0
    out = dict(summ)
    out.update({
        "offered_load_MLUPS": round(offered, 1),
        "offered_over_batched_capacity": round(offered / capacity_mlups, 3) if capacity_mlups else None,
        "workload": f"{len(spec)} requests, Poisson arrivals rate {rate}/s (seed 8772), L~U{{32..192}}, "
                    "R~U[max(6,0.15L),min(60,0.35L)], G/G_c~U[1.05,1.8], droplet/bubble, exp psi, "
                    "FP32-shifted, stop: dP change <1e-5 or max|du|<1e-9 per 2048 steps",
        "budget_GiB": round(budget / 2**30, 1),
        "droplets_per_hour": round(summ["converged"] * 3600.0 / summ["wall_s"], 1),
        "fp64_single_path": {
            "served_one_at_a_time": {k: summ64.get(k) for k in
                                     ("converged", "statuses", "wall_s", "aggregate_MLUPS",
                                      "p50_time_to_equilibrium_s", "p99_time_to_equilibrium_s",
                                      "mean_steps_to_converge")},
            "dP_rel_err_fp32_vs_fp64_max": max(errs) if errs else None,
            "dP_rel_err_fp32_vs_fp64_median": sorted(errs)[len(errs) // 2] if errs else None,
            "requests_compared": len(errs),
        },
        "per_request": [dict(rid=r.rid, L=r.L, status=r.status, criterion=r.criterion,
                             steps=r.steps, tte_s=None if r.finished is None else
                             round(r.time_to_equilibrium, 3),
                             fp64_status=r64.status, fp64_steps=r64.steps,
                             fp64_tte_s=None if r64.finished is None else
                             round(r64.time_to_equilibrium, 3))
                        for r, r64 in zip(recs, recs64)],
    })
    return out


def run_tolman(args, torch, lbm, log):
    """A scaled version of the paper's droplet/bubble sweep (Sec. 4) for both pseudopotentials:
    couplings G/G_c - 1 in {0.159, 0.215, 0.293}, odd box sizes L in {41, ..., 251}, R = L/4,
    droplets and bubbles, the paper's tanh profile (width 1), all boxes served together until
    the paper's criterion (relative dP change < 1e-5 over 2048 steps), once with FP32-shifted
    and once with FP64 populations. The Tolman fit per coupling gives sigma_0 and delta; sigma_0
    is compared with the flat value from a converged FP64 slab (the paper reports that the two
    agree), every FP32 result (dP, sigma_s, R_s, and the fitted sigma_0 and delta) is stated
    against its FP64 counterpart, and the two pseudopotentials are compared through the
    mean-field prefactor sigma_0 / (G/G_c - 1)^(3/2)."""
    out = {"workload": "psi in {exp, 1-exp} x G/G_c-1 in {0.159,0.215,0.293} x L in "
                       "{41,47,55,61,67,77,87,103,123,157,201,251} x {droplet,bubble}, R=L/4, tanh width "
                       "1, served together until |dP change|/dP < 1e-5 per 2048 steps; "
                       "FP32-shifted and FP64 sweeps"}
    names = [n for n in ("exp", "oneminus") if args.tolman_psi in ("both", n)]
    for name in names:
        psi = lbm.LBM_SC_PSI_EXP if name == "exp" else lbm.LBM_SC_PSI_ONEMINUS
        out[name] = tolman_sweep(torch, lbm, log, psi)
    if len(names) < 2:
        return out
    pref = {}
    for name in ("exp", "oneminus"):
        pref[name] = {g: c["flat_sigma0"] / (float(g) - 1) ** 1.5
                      for g, c in out[name]["couplings"].items()}
    out["flat_sigma0_prefactor"] = pref
    out["flat_sigma0_prefactor_ratio_exp_over_oneminus"] = {
        g: pref["exp"][g] / pref["oneminus"][g] for g in pref["exp"] if g in pref["oneminus"]}
    return out


def tolman_sweep(torch, lbm, log, psi):
    from paper_2105_08772_amd import analysis, serve
    ratios = (1.159, 1.215, 1.293)
    sizes = (41, 47, 55, 61, 67, 77, 87, 103, 123, 157, 201, 251)
    spec = {}
    rid = 0
    for g in ratios:
        for L in sizes:
            for bubble in (False, True):
                spec[rid] = dict(g_over_gc=g, L=L, bubble=bubble)
                rid += 1

    def sweep(prec):
        be = serve.GpuBackend(prec=prec, width=1.0, packed_rows=True)
        be.set_launch(rows=4, waves=8, tile_x=0, z_chunk=8, prefetch=0, persistent=0, workers=0,
                      graph_steps=64)
        srv = serve.Server(be, be.free_bytes() - (8 << 30), chunk=512, observe_every=2048,
                           max_steps=100000, dp_tol=1e-5, du_tol=0.0, log=log)
        for k, v in spec.items():
            srv.submit(serve.Request(rid=k, L=v["L"], radius=v["L"] / 4.0,
                                     g_over_gc=v["g_over_gc"], bubble=v["bubble"],
                                     seed=1000 + k, arrival=0.0, psi=psi))
        recs = srv.run()
        be.close()
        torch.cuda.empty_cache()
        conv = {r.rid: r for r in recs if r.status == "converged"}
        fits = analysis.analyse([dict(spec[k], obs=r.obs) for k, r in conv.items()])
        return srv, conv, fits

    res = {}
    for name, prec in (("fp32", lbm.LBM_SC_FP32_SHIFTED), ("fp64", lbm.LBM_SC_FP64)):
        log(f"tolman sweep psi={psi} {name}")
        res[name] = sweep(prec)
    # flat sigma_0: FP64 slab 4 x 4 x 64, liquid thickness 32, width 1, 40000 steps
    stream = torch.cuda.Stream()
    flat = {}
    for g in ratios:
        cfg = lbm.config(4, 4, 64, psi=psi, geom=lbm.LBM_SC_SLAB, prec=lbm.LBM_SC_FP64,
                         g_over_gc=g, slab_thickness=32.0, width=1.0, slab_axis=2,
                         stream=stream.cuda_stream)
        with lbm.Box(cfg) as b:
            b.step(40000)
            o, _ = b.observables()
        flat[g] = dict(sigma0=o["sigma0_flat"], pn_spread_rel=o["pn_spread"] / o["P_out"])
    srv32, conv32, fits32 = res["fp32"]
    srv64, conv64, fits64 = res["fp64"]
    out = {"wall_s": {"fp32": round(srv32.wall, 2), "fp64": round(srv64.wall, 2)},
           "statuses": {"fp32": srv32.summary()["statuses"], "fp64": srv64.summary()["statuses"]},
           "couplings": {}}
    for g in ratios:
        f = fits32.get(round(g, 10))
        f64 = fits64.get(round(g, 10))
        entry = {"flat_sigma0": flat[g]["sigma0"], "flat_pn_spread_rel": flat[g]["pn_spread_rel"]}
        # a coupling with fewer than two distinct curvatures has no fit (NaN): reported as null
        fin = lambda v: v if not (isinstance(v, float) and math.isnan(v)) else None  # noqa: E731
        if f:
            entry.update({k: fin(f[k]) for k in ("sigma0", "delta", "rms", "npoints", "delta_hat0",
                                                 "no_minimum")})
            entry["sigma0_fit_over_flat"] = fin(f["sigma0"] / flat[g]["sigma0"])
            entry["points"] = [dict(kappa=round(p["kappa"], 6), sigma_s=round(p["sigma_s"], 8),
                                    R_s=round(p["R_s"], 4), R_e=round(p["R_e"], 4),
                                    bubble=p["bubble"]) for p in f["points"]]
        if f and f64:
            entry["fp64"] = {k: fin(f64[k]) for k in ("sigma0", "delta", "delta_hat0", "npoints")}
            entry["sigma0_rel_err_fp32_vs_fp64"] = fin(abs(f["sigma0"] - f64["sigma0"]) / f64["sigma0"])
            entry["delta_err_fp32_vs_fp64"] = fin(abs(f["delta"] - f64["delta"]))
        # per run, where both precisions converged
        errs = {"dP": [], "sigma_s": [], "R_s": []}
        for k in sorted(set(conv32) & set(conv64)):
            if spec[k]["g_over_gc"] != g:
                continue
            a, b = conv32[k].obs, conv64[k].obs
            if not (a["R_s"] > 0 and b["R_s"] > 0):
                continue
            errs["dP"].append(abs(a["dP"] - b["dP"]) / abs(b["dP"]))
            sa, sb = 0.5 * a["dP"] * a["R_s"], 0.5 * b["dP"] * b["R_s"]
            errs["sigma_s"].append(abs(sa - sb) / abs(sb))
            errs["R_s"].append(abs(a["R_s"] - b["R_s"]) / b["R_s"])
        entry["per_run_rel_err_fp32_vs_fp64"] = {
            k: {"max": max(v), "median": sorted(v)[len(v) // 2], "runs": len(v)}
            for k, v in errs.items() if v}
        out["couplings"][str(g)] = entry
    gs = [g for g in ratios if fits32.get(round(g, 10))
          and not math.isnan(fits32[round(g, 10)]["sigma0"])]
    if len(gs) >= 2:
        x = [g - 1 for g in gs]
        out["sigma0_exponent"] = analysis.scaling_exponent(
            x, [fits32[round(g, 10)]["sigma0"] for g in gs])["exponent"]
        out["flat_sigma0_exponent"] = analysis.scaling_exponent(x, [flat[g]["sigma0"] for g in gs])["exponent"]
        if all(fits32[round(g, 10)]["delta"] > 0 for g in gs):
            out["delta_exponent"] = analysis.scaling_exponent(
                x, [fits32[round(g, 10)]["delta"] for g in gs])["exponent"]
    return out


def run_oneminus(args, torch, lbm, stream, steps):
    """The same 256^3 droplet with the second pseudopotential of Sec. 4, psi = 1 - exp(-n)
    (G/G_c = 1.3, its own flat coexistence densities), in the main run's precision and launch:
    `steps` steps with an FP64 observation every 2048 (wall clock) and the step kernel's average
    duration over back-to-back steps (HIP events on the library's stream)."""
    prec = {"fp32": lbm.LBM_SC_FP32_SHIFTED, "fp32m64": lbm.LBM_SC_FP32_SHIFTED_MATH64,
            "fp64": lbm.LBM_SC_FP64}[args.prec]
    L = args.size
    cfg = lbm.config(L, L, L, psi=lbm.LBM_SC_PSI_ONEMINUS, geom=lbm.LBM_SC_DROPLET, prec=prec,
                     tau=1.0, g_over_gc=1.3, radius=args.radius, width=2.0, noise_amp=1e-6,
                     seed=3, stream=stream.cuda_stream)
    with lbm.Box(cfg) as box:
        info = box.info()
        box.step(128)
        box.observables(profile=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            n = min(2048 - done % 2048, steps - done)
            box.step(n)
            done += n
            if done % 2048 == 0:
                box.observables(profile=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        box.step(1024)
        e1.record(stream)
        torch.cuda.synchronize()
        t_step = e0.elapsed_time(e1) / 1e3 / 1024
        obs, _ = box.observables(profile=False)
    return {"workload": f"droplet {L}^3 periodic, {PREC_NAMES[args.prec]} populations, "
                        f"psi=1-exp(-n), G/G_c=1.3, R={args.radius:g}, tanh width 2, noise 1e-6 "
                        f"seed 3, tau=1, FP64 observables every 2048 steps",
            "n_in": info["n_in"], "n_out": info["n_out"], "steps": steps,
            "MLUPS": round(info["nodes"] * steps / wall / 1e6, 1),
            "kernel_ms": round(t_step * 1e3, 5),
            "kernel_GBps": round(info["bytes_per_step"] / t_step / 1e9, 1),
            "kernel_frac_of_8TBps": round(info["bytes_per_step"] / t_step / 1e9 / HBM_PEAK_GBPS, 4),
            "checks": {"finite": obs["finite"],
                       "mass_drift_rel": abs(obs["mass"] - obs["mass0"]) / obs["mass0"],
                       "dP": obs["dP"]}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(args, nodes_gpu):
    """The FP64 oracle on the host cores: its own initial state of the same droplet, then
    `cpu_steps` plain steps of the whole box on all threads; plus one step of a 128^3 box of the
    same droplet (radius scaled) on one thread for the single-core rate."""
    import oracle
    from oracle import core, eos
    oracle.build(force=False)
    kind = 0 if args.psi == "exp" else 1
    G = eos.G_of(1.3, kind)
    ng, nl, _ = eos.coexistence_rule(G, kind)
    L = args.size
    n0 = core.init_density(L, L, L, core.DROPLET, args.radius, 2.0, nl, ng, 1e-6, 3)
    f = core.init_populations(n0, G, kind)
    del n0
    threads = core.threads()
    t0 = time.perf_counter()
    f = core.run(f, G, 1.0, kind, args.cpu_steps)
    dt = time.perf_counter() - t0
    del f
    nodes = L ** 3
    # single core, smaller box
    Ls = 128
    n0 = core.init_density(Ls, Ls, Ls, core.DROPLET, args.radius * Ls / L, 2.0, nl, ng, 1e-6, 3)
    f = core.init_populations(n0, G, kind)
    core.set_threads(1)
    t1 = time.perf_counter()
    core.run(f, G, 1.0, kind, 1)
    dt1 = time.perf_counter() - t1
    core.set_threads(threads)
    return {"value": round(nodes * args.cpu_steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{args.cpu_steps} steps of the whole {L}^3 droplet (FP64 oracle, "
                      f"{dt:.1f} s on {threads} threads)",
            "cpu_model": cpu_model(),
            "one_core_MLUPS": round(Ls ** 3 / dt1 / 1e6, 3),
            "one_core_sample": f"1 step of a {Ls}^3 droplet on 1 thread ({dt1:.1f} s)"}


def plain_method_full_run(torch, lbm):
    """The plain-method configuration run in full on both sides: a 32^3 FP64 droplet (exp psi,
    G/G_c = 1.3, R = 8, tanh width 2, noise 1e-6 seed 1), 2000 steps, by the oracle on all host
    threads and by the library on the GPU (from the same initial state), with the largest
    difference of the final populations."""
    import numpy as np
    from oracle import core
    cfg = lbm.config(32, psi=lbm.LBM_SC_PSI_EXP, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP64,
                     g_over_gc=1.3, radius=8.0, width=2.0, noise_amp=1e-6, seed=1)
    with lbm.Box(cfg) as b:
        G = b.info()["G"]
        f0 = b.get()
        b.step(64)                       # capture the step chunk outside the timing
        b.set(f0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(2000)
        b.sync()
        gpu_s = time.perf_counter() - t0
        f_gpu = b.get()
    t0 = time.perf_counter()
    f_cpu = core.run(f0, G, 1.0, core.PSI_EXP, 2000)
    cpu_s = time.perf_counter() - t0
    return {"oracle_s": round(cpu_s, 3), "gpu_fp64_s": round(gpu_s, 4),
            "oracle_threads": core.threads(),
            "max_rel_diff": float(np.abs(f_gpu - f_cpu).max() / np.abs(f_cpu).max())}


PREC_NAMES = {"fp32": "FP32-shifted", "fp32m64": "FP32-shifted (FP64 arithmetic)",
              "fp64": "FP64"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50000,
                    help="timed steps of the 256^3 droplet (default: the configuration's 50000)")
    ap.add_argument("--warmup", type=int, default=128)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--radius", type=float, default=60.0)
    ap.add_argument("--psi", choices=["exp", "oneminus"], default="exp")
    ap.add_argument("--prec", choices=["fp32", "fp32m64", "fp64"], default="fp32",
                    help="fp32: FP32-shifted storage and arithmetic; fp32m64: FP32-shifted storage,"
                         " FP64 arithmetic; fp64: FP64 storage and arithmetic")
    ap.add_argument("--observe-every", type=int, default=2048)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--remap", type=int, default=-1)
    ap.add_argument("--prefetch", type=int, default=-1)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--tile-x", type=int, default=-1, help="64, 32, or 0 for full-row tiles")
    ap.add_argument("--steps-per-pass", type=int, default=0,
                    help="1 or 2 time steps per kernel pass (0: the library's default)")
    ap.add_argument("--tune", action="store_true", help="sweep launch shapes, keep the fastest")
    ap.add_argument("--cpu-steps", type=int, default=25)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--mode", choices=["step", "copy"], default="step",
                    help="copy: only the streaming-copy reference (for counter calibration)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--copy-reps", type=int, default=5)
    ap.add_argument("--copy-lane", type=int, default=4, choices=[4, 8, 16],
                    help="bytes each lane of the copy kernel moves per access (--mode copy)")
    ap.add_argument("--served-count", type=int, default=32,
                    help="requests of the served workload to run after the main timing (0 = skip;"
                         " default: 32)")
    ap.add_argument("--served-rate", type=float, default=1.0,
                    help="request arrival rate (1/s); the default offers about 0.8 of the batched "
                         "throughput")
    ap.add_argument("--served-journal", default=None,
                    help="write one JSON line per served request (FP32 batched run) to this file")
    ap.add_argument("--served-capacity", type=float, default=None,
                    help="batched throughput (MLUPS) to state the offered load against when the "
                         "batched workload is not run in the same invocation")
    ap.add_argument("--tolman", action="store_true",
                    help="run the scaled droplet/bubble sweep and the Tolman analysis")
    ap.add_argument("--tolman-psi", choices=["both", "exp", "oneminus"], default="both",
                    help="pseudopotentials of the Tolman sweep")
    ap.add_argument("--oneminus-steps", type=int, default=4096,
                    help="steps of the same 256^3 droplet with psi = 1 - exp(-n) timed after the "
                         "main run (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=20000,
                    help="steps of the batched 64-box workload measured after the main timing "
                         "(0 = skip; default: the configuration's 20000)")
    ap.add_argument("--traffic-from", default=None,
                    help="CPU only: turn the rocprofv3 counter runs under this directory into the "
                         "traffic record the benchmark reads (see traffic_summary)")
    ap.add_argument("--traffic-bench-log", default=None,
                    help="with --traffic-from: output of the counted step run")
    ap.add_argument("--traffic-group-log", default=None,
                    help="with --traffic-from and no --traffic-bench-log: output of the counted "
                         "batched run (its tuned launch names the group kernel)")
    args = ap.parse_args()
    if args.traffic_from:
        if args.traffic_bench_log:
            traffic_summary(args.traffic_from, args.traffic_bench_log, TRAFFIC_FILE)
        else:
            group_traffic(args.traffic_from, args.traffic_group_log,
                          out_path=GROUP_TRAFFIC_FILE if args.traffic_group_log else None)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (there is no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2105_08772_amd as lbm

    torch.cuda.set_device(0)
    # a dedicated stream (default priority): the library enqueues on it and the timing events
    # are recorded on it
    stream = torch.cuda.Stream()
    if args.mode == "copy":
        nbytes = args.copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(args.copy_reps):
            lbm.lbm_sc_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream,
                                   lane_bytes=args.copy_lane)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": nbytes,
                          "bytes_written_per_launch": nbytes, "launches": args.copy_reps}))
        return
    L = args.size
    psi = lbm.LBM_SC_PSI_EXP if args.psi == "exp" else lbm.LBM_SC_PSI_ONEMINUS
    prec = {"fp32": lbm.LBM_SC_FP32_SHIFTED, "fp32m64": lbm.LBM_SC_FP32_SHIFTED_MATH64,
            "fp64": lbm.LBM_SC_FP64}[args.prec]
    cfg = lbm.config(L, L, L, psi=psi, geom=lbm.LBM_SC_DROPLET, prec=prec, tau=1.0,
                     g_over_gc=1.3, radius=args.radius, width=2.0, noise_amp=1e-6, seed=3,
                     stream=stream.cuda_stream)
    box = lbm.Box(cfg)
    info = box.info()
    nodes = info["nodes"]
    print(f"# created {L}^3 box, {info['device_bytes'] / 2**30:.2f} GiB on the device",
          file=sys.stderr, flush=True)
    bytes_per_step = info["bytes_per_step"]

    def time_steps(k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        box.step(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / k

    tuned = None
    if args.tune:
        best = None
        from paper_2105_08772_amd import tune
        for c in tune.box_candidates(L):
            try:
                box.set_launch(c["rows"], c["z_chunk"], c["xcd_remap"], c["prefetch"], c["waves"],
                               c["tile_x"], 64, c.get("steps_per_pass", 1))
            except lbm.LbmScError:
                continue
            box.step(8)
            t = time_steps(64)
            print(f"# tune {c} {nodes / t / 1e6:.0f} MLUPS {bytes_per_step / t / 1e9:.0f} GB/s",
                  file=sys.stderr, flush=True)
            if best is None or t < best[0]:
                best = (t, c)
        tuned = best[1]
        box.set_launch(tuned["rows"], tuned["z_chunk"], tuned["xcd_remap"], tuned["prefetch"],
                       tuned["waves"], tuned["tile_x"], 64, tuned.get("steps_per_pass", 1))
    if (args.rows or args.zchunk or args.remap >= 0 or args.prefetch >= 0 or args.waves
            or args.tile_x >= 0 or args.steps_per_pass):
        lc = box.launch()
        box.set_launch(args.rows or lc["rows"], args.zchunk or lc["z_chunk"],
                       args.remap if args.remap >= 0 else lc["xcd_remap"],
                       args.prefetch if args.prefetch >= 0 else lc["prefetch"],
                       args.waves or lc["waves"], args.tile_x if args.tile_x >= 0 else lc["tile_x"],
                       64, args.steps_per_pass or lc["steps_per_pass"])
    info = box.info()
    launch = box.launch()

    # warmup
    box.step(args.warmup)
    box.observables(profile=False)
    torch.cuda.synchronize()

    # timed region: K steps with an FP64 observation every observe_every steps
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    last = None
    while done < K:
        n = min(args.observe_every - done % args.observe_every, K - done)
        box.step(n)
        done += n
        if done % args.observe_every == 0:
            last, _ = box.observables(profile=False)
            if done % (8 * args.observe_every) == 0:
                print(f"# {done} of {K} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    mlups = nodes * K / wall / 1e6
    print(f"# timed {K} steps: {mlups:.0f} MLUPS", file=sys.stderr, flush=True)

    # the dominant kernel alone: average launch duration over back-to-back steps (a launch
    # advances the box by steps_per_pass steps)
    spp = launch["steps_per_pass"]
    k_steps = min(K, 2048)
    step_s = time_steps(k_steps)
    achieved = bytes_per_step / step_s / 1e9
    obs, _ = box.observables(profile=False)
    box.close()

    copy_bw = None if args.no_copy else stream_copy_gbps(torch, lbm, stream)
    traffic = measured_traffic(nodes, args.prec, launch)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == lbm.LBM_SC_FP32_SHIFTED else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"droplet {L}^3 periodic, {PREC_NAMES[args.prec]} populations,"
                        f" psi={args.psi}, G/G_c=1.3, R={args.radius:g}, tanh width 2,"
                        f" noise 1e-6 seed 3, tau=1, FP64 observables every {args.observe_every}"
                        f" steps",
            "nodes": nodes,
            "launch": dict(launch, block=[info["block_x"], info["block_y"]],
                           tuned=tuned is not None),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel_ms": round(step_s * spp * 1e3, 5),
            "steps_per_launch": spp,
            "bytes_per_launch": bytes_per_step * spp,
            "stream_copy_GBps": copy_bw,
            "frac_of_best_copy": round(achieved / copy_bw["best"], 4) if copy_bw else None,
        },
        "checks": {"finite": obs["finite"],
                   "mass_drift_rel": abs(obs["mass"] - obs["mass0"]) / obs["mass0"],
                   "dP": obs["dP"], "R_s": obs["R_s"]},
    }
    if args.oneminus_steps > 0 and args.psi == "exp":
        print("# 256^3 droplet with psi = 1 - exp(-n)", file=sys.stderr, flush=True)
        out["psi_oneminus"] = run_oneminus(args, torch, lbm, stream, args.oneminus_steps)
    if args.batched_steps > 0:
        out["batched"] = run_batched(args, torch, lbm, stream, args.batched_steps,
                                     lambda m: print(m, file=sys.stderr, flush=True))
    if args.tolman:
        out["tolman"] = run_tolman(args, torch, lbm,
                                   lambda m: print("# " + m, file=sys.stderr, flush=True))
    if args.served_count > 0:
        cap = out["batched"]["MLUPS"] if "batched" in out else args.served_capacity
        out["served"] = run_served(args, torch, lbm,
                                   lambda m: print("# " + m, file=sys.stderr, flush=True), cap)
    if not args.no_cpu:
        print("# timing the oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, nodes)
        out["cpu_baseline"]["plain_method_32cubed"] = plain_method_full_run(torch, lbm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
