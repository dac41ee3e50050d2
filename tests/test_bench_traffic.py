"""The counter summary of bench.py (CPU only): rocprofv3 counter tables in, HBM bytes per launch
out. Synthetic tables with known values check the per-dispatch sum over rows, the median, the
kernel filter and the scaling by the copy calibration; the committed traffic record must be the
one bench.py accepts for the current step-kernel sources."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
STEP = "void lbm::(anonymous namespace)::k_step<float, float, 0, true, 2, false, 8, 64>(...)"
COPY = "void lbm::(anonymous namespace)::k_stream_copy<float>(float const*, float*, unsigned long)"


def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_run(d, counter, rows):
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for disp, name, val in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": val})


def test_counter_median_sums_rows_of_a_dispatch_and_filters_kernels(tmp_path):
    b = bench()
    d = str(tmp_path / "run")
    # dispatch 2 reported in two rows (e.g. per XCD): 30 + 10; another kernel is ignored
    write_run(d, "FETCH_SIZE", [(1, STEP, 10.0), (2, STEP, 30.0), (2, STEP, 10.0), (3, COPY, 1e9),
                                (4, STEP, 20.0), (5, STEP, 100.0)])
    med, n = b.counter_per_dispatch(d, "FETCH_SIZE", "void lbm::(anonymous namespace)::k_step<")
    assert (med, n) == (30.0, 4)          # median of 10, 40, 20, 100
    med, n = b.counter_per_dispatch(d, "FETCH_SIZE", "void lbm::(anonymous namespace)::k_step<",
                                    last=2)
    assert (med, n) == (60.0, 2)          # 20 and 100
    with pytest.raises(SystemExit):
        b.counter_per_dispatch(d, "WRITE_SIZE", "void lbm::(anonymous namespace)::k_step<")


def test_traffic_summary_scales_by_the_copy(tmp_path):
    b = bench()
    p = str(tmp_path)
    gib_kib = (1 << 30) / 1024
    # the copy's FETCH_SIZE reads half its bytes, WRITE_SIZE all of them
    write_run(os.path.join(p, "pmc_FETCH_SIZE_copy"), "FETCH_SIZE", [(1, COPY, gib_kib / 2)] * 1)
    write_run(os.path.join(p, "pmc_WRITE_SIZE_copy"), "WRITE_SIZE", [(1, COPY, gib_kib)])
    write_run(os.path.join(p, "pmc_FETCH_SIZE_step"), "FETCH_SIZE", [(7, STEP, 600.0)])
    write_run(os.path.join(p, "pmc_WRITE_SIZE_step"), "WRITE_SIZE", [(7, STEP, 1000.0)])
    log = os.path.join(p, "bench.log")
    res = {"config": {"nodes": 8, "launch": {"rows": 2, "z_chunk": 64, "xcd_remap": 1,
                                             "prefetch": 0, "waves": 8, "tile_x": 64,
                                             "graph_steps": 64, "block": [64, 16],
                                             "tuned": False}},
           "roofline": {"bytes_per_launch": 2 * 1000 * 1024}}
    with open(log, "w") as fh:
        fh.write("# some stderr line\n" + json.dumps(res) + "\nrocprofv3 finalization\n")
    out = os.path.join(p, "traffic.json")
    b.traffic_summary(p, log, out)
    t = json.load(open(out))
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["fetch_bytes_per_launch"] == 1200 * 1024
    assert t["write_bytes_per_launch"] == 1000 * 1024
    assert t["bytes_per_launch"] == 2200 * 1024
    assert t["launch"] == {"rows": 2, "z_chunk": 64, "xcd_remap": 1, "prefetch": 0, "waves": 8,
                           "tile_x": 64}
    assert t["kernel_sha256_16"] == b.kernel_hash()


def test_committed_traffic_record_matches_the_current_step_kernels():
    b = bench()
    with open(b.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert t["kernel_sha256_16"] == b.kernel_hash(), \
        "step kernel sources changed since the counters were taken: profile again"
    launch = dict(t["launch"], graph_steps=64)
    assert b.measured_traffic(t["nodes"], t["prec"], launch) == t["bytes_per_launch"]
    # per launch: reads at least one pass over the state (a launch of two steps reads and writes
    # it once), at most that times the planes a z chunk pulls over the planes it steps (one more
    # on each side for one step, three for two) and 20 % of halo re-reads in x and y; writes one
    # pass
    spp = t.get("steps_per_launch", 1)
    alg = t["algorithmic_bytes_per_launch"] / 2 / spp
    zc = t["launch"]["z_chunk"]
    chunk = (zc + 2 * (2 * spp - 1)) / zc
    assert 1.0 <= t["fetch_bytes_per_launch"] / alg < 1.2 * chunk
    assert 0.99 < t["write_bytes_per_launch"] / alg < 1.01


GROUP1 = "void lbm::(anonymous namespace)::k_step_group<float, float, 4, false, 8, 0>(...)"
GROUP2 = "void lbm::(anonymous namespace)::k_step2_group<32, 16, 8, false, 4>(...)"


def test_group_traffic_follows_the_tuned_kernel(tmp_path, capsys):
    """The batched counter summary takes the dispatches of the tuned group kernel over the timed
    mix only (the tuner's dispatches of every kernel come first), one per step or per two steps,
    and reports bytes per launch and per step."""
    b = bench()
    p = str(tmp_path)
    rec = json.load(open(b.TRAFFIC_FILE))
    # tuner: both kernels; timed mix: 384 steps = 192 two-step launches of 1000 KiB read
    tuner = [(k, GROUP1 if k % 2 else GROUP2, 5000.0) for k in range(1, 50)]
    timed = [(100 + k, GROUP2, 1000.0) for k in range(192)]
    write_run(os.path.join(p, "pmc_FETCH_SIZE_group"), "FETCH_SIZE", tuner + timed)
    write_run(os.path.join(p, "pmc_WRITE_SIZE_group"), "WRITE_SIZE",
              tuner + [(d, n, 800.0) for d, n, _ in timed])
    log = os.path.join(p, "group.log")
    with open(log, "w") as fh:
        fh.write(json.dumps({"batched": {"launch": {"steps_per_pass": 2, "tile_x": 32}}}) + "\n")
    rec_path = os.path.join(p, "group_record.json")
    b.group_traffic(p, log, out_path=rec_path)
    out = json.loads(capsys.readouterr().out)
    assert out["steps_per_launch"] == 2 and out["kernel"].endswith("k_step2_group<")
    g = json.load(open(rec_path))
    assert g["launch"] == {"steps_per_pass": 2, "tile_x": 32} and g["steps_per_launch"] == 2
    assert g["group_sha256_16"] == b.group_hash() and g["nodes"] == b.GROUP_NODES
    assert g["bytes_per_launch"] == g["fetch_bytes_per_launch"] + g["write_bytes_per_launch"]
    assert g["algorithmic_bytes_per_launch"] == 152 * b.GROUP_NODES * 2
    assert out["FETCH_SIZE"]["dispatches"] == 192 and out["FETCH_SIZE"]["KiB_per_dispatch"] == 1000.0
    assert out["FETCH_SIZE"]["bytes_per_launch"] == int(1000 * 1024 * rec["fetch_scale"])
    assert out["FETCH_SIZE"]["bytes_per_step"] == int(1000 * 1024 * rec["fetch_scale"] / 2)
    assert out["WRITE_SIZE"]["bytes_per_step"] == int(800 * 1024 * rec["write_scale"] / 2)
    # a single-step launch: the last 384 dispatches of the single-step kernel
    with open(log, "w") as fh:
        fh.write(json.dumps({"batched": {"launch": {"steps_per_pass": 1}}}) + "\n")
    b.group_traffic(p, log)
    out = json.loads(capsys.readouterr().out)
    assert out["steps_per_launch"] == 1 and out["FETCH_SIZE"]["dispatches"] == 25
    assert out["FETCH_SIZE"]["KiB_per_dispatch"] == 5000.0


def test_committed_group_traffic_record_matches_the_current_sources():
    """The batched leg reports the committed counter record only for the group sources and the
    launch it was taken on; the record is consistent with itself."""
    b = bench()
    with open(b.GROUP_TRAFFIC_FILE) as fh:
        g = json.load(fh)
    assert g["group_sha256_16"] == b.group_hash(), \
        "step kernels or group host code changed since the counters were taken: profile again"
    assert b.measured_group_traffic(g["nodes"], g["launch"]) == g["bytes_per_launch"]
    assert b.measured_group_traffic(g["nodes"], dict(g["launch"], z_chunk=7)) is None
    assert g["bytes_per_launch"] == g["fetch_bytes_per_launch"] + g["write_bytes_per_launch"]
    spp = g["steps_per_launch"]
    one_pass = g["algorithmic_bytes_per_launch"] / 2 / spp
    # a launch reads at least one pass over the state and writes about one (plus padding lanes)
    assert g["fetch_bytes_per_launch"] >= one_pass
    assert 0.99 < g["write_bytes_per_launch"] / one_pass < 1.15
