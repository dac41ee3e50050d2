"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same seeded inputs.

Bars (written into each test):
  - FP64 storage: max |f_gpu - f_oracle| / max |f_oracle| <= 1e-11 after one step from an
    identical state, and the same along the 2000-step 32^3 droplet;
  - FP32-shifted storage: one step from the identical (FP32-representable) state within a bound
    derived from single-precision rounding of the collision (a few ulp of the largest shifted
    population), and after 2000 steps densities, dP and mass within three times the measured
    differences from FP64 (FP32_DROPLET_BOUNDS);
  - FP32-shifted storage with FP64 arithmetic: one step within half an ulp of the oracle per
    stored population (the rest population within the sum of the others' rounding errors);
  - launch shapes: bitwise identical results (the per-node arithmetic does not depend on them).
"""
import sys

import numpy as np
import pytest

import paper_2105_08772_amd as lbm
from oracle import core, eos, observe
from tests import inputs

pytestmark = pytest.mark.gpu

XI, W, _ = core.tables()
TOL64 = 1e-11
# converged 64^3 FP32 droplet, 32768 steps: measured 2.4e-8 with the dithered rest-population
# rounding (plain round-to-nearest drifts about 1e-10 per step at the same densities, ~3e-6);
# the bound is three times the measured value
DRIFT_BOUND = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def two_steps_at(f, G, x, y, z, psi=0, tau=1.0):
    """The oracle's two steps at node (x, y, z) of the state f: two whole steps on the node's
    periodic neighbourhood of radius 4 (the whole axis where the box is shorter than 9), on which
    the node's result depends and nothing else (a pin in the oracle tests)."""
    idx, centre = [], []
    for c, n in zip((x, y, z), f.shape[:0:-1]):
        if n >= 9:
            idx.append((np.arange(-4, 5) + c) % n)
            centre.append(4)
        else:
            idx.append(np.arange(n))
            centre.append(c)
    ix, iy, iz = idx
    sub = np.ascontiguousarray(f[:, iz][:, :, iy][:, :, :, ix])
    return core.run(sub, G, tau, psi, 2)[:, centre[2], centre[1], centre[0]]


def fp32_representable(f, rho_ref):
    """The FP64 state that an FP32-shifted box holds after set_populations(f)."""
    g = (f - W.reshape(19, 1, 1, 1) * rho_ref).astype(np.float32).astype(np.float64)
    return g + W.reshape(19, 1, 1, 1) * rho_ref


def make_box(dims, prec=lbm.LBM_SC_FP64, psi=lbm.LBM_SC_PSI_EXP, ratio=1.3, tau=1.0,
             rho_ref=0.0, packed=0):
    nx, ny, nz = dims
    cfg = lbm.config(nx, ny, nz, psi=psi, geom=lbm.LBM_SC_FROM_HOST, prec=prec, tau=tau,
                     g_over_gc=ratio, rho_ref=rho_ref if rho_ref else 1.0, packed_rows=packed)
    return lbm.Box(cfg)


SHAPES = [(4, 4, 4), (32, 32, 32), (37, 29, 11), (130, 7, 6), (5, 70, 9), (1, 1, 8), (2, 3, 5),
          (3, 3, 3)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("psi,ratio,tau", [(0, 1.3, 1.0), (1, 1.2, 0.8), (0, 1.6, 1.3)])
def test_one_step_fp64(dims, psi, ratio, tau):
    say(f"one step FP64 dims={dims} psi={psi} G/Gc={ratio} tau={tau}")
    f = inputs.random_populations(dims, 100 + sum(dims), W * 1.5, amp=0.3)
    G = ratio * lbm.lbm_sc_gc(psi)
    with make_box(dims, psi=psi, ratio=ratio, tau=tau) as b:
        b.set(f)
        b.step(1)
        g = b.get()
    ref = core.step(f, G, tau, psi)
    assert rel_err(g, ref) <= TOL64


@pytest.mark.parametrize("dims", [(4, 4, 4), (37, 29, 11), (130, 7, 6), (64, 40, 20)])
@pytest.mark.parametrize("tau", [1.0, 0.7])
@pytest.mark.parametrize("prefetch", [0, 1])
def test_one_step_fp32_shifted(dims, tau, prefetch):
    say(f"one step FP32 dims={dims} tau={tau}")
    rho_ref = 1.5
    f = fp32_representable(inputs.random_populations(dims, 7 + sum(dims), W * 1.5, amp=0.3), rho_ref)
    G = 1.3 * lbm.lbm_sc_gc(0)
    with make_box(dims, prec=lbm.LBM_SC_FP32_SHIFTED, tau=tau, rho_ref=rho_ref) as b:
        b.set(f)
        # the single-step kernel in its default tile (prefetch is compiled for 4-wave workgroups)
        b.set_launch(2, dims[2], 1, prefetch, 4 if prefetch else 8, 64)
        b.step(1)
        g = b.get()
    ref = core.step(f, G, tau, 0)
    # single-precision collision: each shifted population carries a few roundings of quantities
    # no larger than the largest |f| (measured at most 4.0e-8 of max |f| over these cases; the
    # bound is three times that, about 2 ulp of the largest population)
    err = rel_err(g, ref)
    say(f"  max |f_gpu - f_oracle| / max |f_oracle| = {err:.3e}")
    assert err <= 1.2e-7
    # mass per node is closed exactly up to the last rounding
    n_g = g.sum(axis=0)
    n_r = ref.sum(axis=0)
    assert abs(n_g.sum() - n_r.sum()) / n_r.sum() < 1e-7


@pytest.mark.parametrize("dims", [(4, 4, 4), (37, 29, 11), (130, 7, 6), (64, 40, 20)])
@pytest.mark.parametrize("psi,ratio,tau", [(0, 1.3, 1.0), (1, 1.2, 0.8)])
def test_one_step_fp32_storage_fp64_arithmetic(dims, psi, ratio, tau):
    """FP32-shifted storage with FP64 arithmetic, one step from an identical state: each stored
    population i > 0 is the oracle's value rounded once to single precision (within half an ulp
    of it, plus 1e-12 max|f| for the different FP64 rounding orders); the rest population, closed
    from the 18 rounded values and rounded with a dither of at most half an ulp, within the sum
    of their errors plus 1.5 ulp."""
    say(f"one step FP32 storage / FP64 arithmetic dims={dims} psi={psi} tau={tau}")
    rho_ref = 1.5
    f = fp32_representable(inputs.random_populations(dims, 11 + sum(dims), W * 1.5, amp=0.3), rho_ref)
    G = ratio * lbm.lbm_sc_gc(psi)
    with make_box(dims, prec=lbm.LBM_SC_FP32_SHIFTED_MATH64, psi=psi, ratio=ratio, tau=tau,
                  rho_ref=rho_ref) as b:
        b.set(f)
        b.step(1)
        g = b.get()
    ref = core.step(f, G, tau, psi)
    shift = W.reshape(19, 1, 1, 1) * rho_ref
    gs, rs = g - shift, ref - shift
    slack = 1e-12 * np.abs(ref).max()
    half_ulp = 0.5 * np.spacing(np.abs(rs).astype(np.float32)).astype(np.float64)
    err = np.abs(gs - rs)
    assert np.all(err[1:] <= half_ulp[1:] + slack)
    # population i at node x was collided at x - xi_i: move the errors back to the colliding node
    src_err = np.stack([np.roll(err[i], shift=(-XI[i, 2], -XI[i, 1], -XI[i, 0]), axis=(0, 1, 2))
                        for i in range(1, 19)])
    # the rest population is rounded after a dither of at most half an ulp: at most 1.5 ulp
    assert np.all(err[0] <= src_err.sum(axis=0) + 3 * half_ulp[0] + 19 * slack)
    say(f"  max error / half ulp (i > 0): {float((err[1:] / (half_ulp[1:] + slack)).max()):.3f}")


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED,
                                  lbm.LBM_SC_FP32_SHIFTED_MATH64])
def test_launch_shapes_are_bitwise_identical(prec):
    say(f"launch shapes prec={prec}")
    dims = (70, 45, 33)
    rho_ref = 1.5
    f = fp32_representable(inputs.random_populations(dims, 3, W * 1.5, amp=0.3), rho_ref)
    outs = []
    shapes = ((1, 1, 0, 0, 4, 64), (2, 7, 1, 1, 4, 64), (4, 33, 1, 0, 4, 64),
              (4, 5, 0, 1, 4, 64), (1, 64, 1, 1, 4, 64), (2, 3, 0, 0, 4, 64),
              (2, 9, 1, 0, 8, 64), (1, 33, 0, 0, 8, 64), (1, 2, 1, 1, 4, 32), (2, 5, 0, 1, 4, 32),
              (2, 11, 1, 0, 4, 32), (1, 4, 1, 0, 8, 32), (2, 33, 0, 0, 8, 32),
              (4, 7, 1, 0, 8, 0), (4, 33, 0, 0, 8, 0), (2, 6, 1, 0, 8, 0), (4, 5, 0, 0, 4, 0))
    if prec == lbm.LBM_SC_FP32_SHIFTED:
        shapes += ((8, 5, 1, 0, 8, 0), (8, 33, 0, 0, 8, 0))
    for rows, zc, remap, pf, waves, tx in shapes:
        with make_box(dims, prec=prec, rho_ref=rho_ref) as b:
            b.set(f)
            b.set_launch(rows, zc, remap, pf, waves, tx)
            assert b.launch() == dict(rows=rows, z_chunk=min(zc, 33), xcd_remap=remap, prefetch=pf,
                                      waves=waves, tile_x=tx, graph_steps=64, steps_per_pass=1)
            b.step(3)
            outs.append(b.get())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    with make_box(dims, prec=prec, rho_ref=rho_ref) as b:
        bad_shapes = [(3, 4, 1, 0, 4, 64), (2, 0, 1, 0, 4, 64), (2, 4, 2, 0, 4, 64),
                      (2, 4, 1, 0, 6, 64), (4, 4, 1, 0, 8, 64), (2, 4, 1, 1, 8, 64),
                      (4, 4, 1, 0, 4, 32), (2, 4, 1, 0, 4, 16), (2, 4, 1, 0, 4, 0),
                      (8, 4, 1, 0, 4, 0), (1, 4, 1, 0, 8, 0), (4, 4, 1, 1, 8, 0)]
        if prec != lbm.LBM_SC_FP32_SHIFTED:
            bad_shapes.append((8, 4, 1, 0, 8, 0))   # 8 nodes per thread: FP32 arithmetic only
        for bad in bad_shapes:
            with pytest.raises(lbm.LbmScError):
                b.set_launch(*bad)
    # full-row tiles need rows that fit: px = 704 leaves no room for 4 nodes per thread
    with make_box((700, 3, 2), prec=prec, rho_ref=rho_ref) as b:
        with pytest.raises(lbm.LbmScError):
            b.set_launch(4, 2, 1, 0, 8, 0)


def test_graph_replay_equals_plain_launches():
    """lbm_sc_step replays captured chunks of graph_steps launches: bitwise the same as plain
    launches for step counts below, at and above the chunk, after an odd number of steps (the
    chunk was captured from the other buffer), after a change of launch shape and after
    set_populations; odd or too long chunks are rejected."""
    say("graph replay vs plain launches")
    dims = (37, 29, 11)
    rho_ref = 1.5
    f = fp32_representable(inputs.random_populations(dims, 21, W * 1.5, amp=0.3), rho_ref)
    runs = {}
    for K in (0, 2, 6):
        with make_box(dims, prec=lbm.LBM_SC_FP32_SHIFTED, rho_ref=rho_ref) as b:
            b.set(f)
            b.set_launch(2, dims[2], 1, 0, 8, 64, K)   # single steps (two-step graphs: their own test)
            out = []
            for n in (1, 6, 7, 13, 2):
                b.step(n)
                out.append(b.get())
            b.set_launch(1, 5, 0, 1, 4, 64, K)     # new shape: the chunk is captured again
            b.step(9)
            out.append(b.get())
            b.set(f)                                # same buffers, new state
            b.step(8)
            out.append(b.get())
            for bad in (3, -2, 4098):
                with pytest.raises(lbm.LbmScError):
                    b.set_launch(2, 4, 1, 0, 8, 64, bad)
        runs[K] = out
    for K in (2, 6):
        for a, c in zip(runs[K], runs[0]):
            assert np.array_equal(a, c)


def test_steps_recorded_into_a_caller_graph():
    """lbm_sc_step inside a caller's stream capture records plain launches into the caller's
    graph; replaying it (several times, with eager work and synchronisation between the
    replays) matches a box stepped eagerly from the same state after every replay. An odd step
    count is refused inside the capture (its replays would repeat one step), and so is a group
    step; the host step counter, advanced once at the capture, is set right with set_step."""
    import torch
    say("steps inside a caller's graph capture")
    s = torch.cuda.Stream()
    dims = (24, 20, 16)
    rho_ref = 1.5
    f = fp32_representable(inputs.random_populations(dims, 31, W * 1.5, amp=0.3), rho_ref)
    cfg = lbm.config(*dims, psi=0, geom=lbm.LBM_SC_FROM_HOST, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.3, rho_ref=rho_ref, stream=s.cuda_stream)
    with lbm.Box(cfg) as b, lbm.Box(cfg) as ref:
        b.set(f)
        ref.set(f)
        torch.cuda.synchronize()
        grp = lbm.Group(s.cuda_stream)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            with pytest.raises(lbm.LbmScError) as odd:
                b.step(3)
            with pytest.raises(lbm.LbmScError) as in_group:
                grp.step(2)
            refused = []   # calls that wait for the stream or go through host memory
            for call in (b.sync, b.get, lambda: b.set(f), lambda: b.set_step(1),
                         lambda: b.observables(profile=False), lambda: grp.set([b]),
                         lambda: grp.set_launch(rows=2)):
                with pytest.raises(lbm.LbmScError) as e:
                    call()
                refused.append(e.value.code)
            b.step(4)
        assert odd.value.code == lbm.LBM_SC_EINVAL and in_group.value.code == lbm.LBM_SC_EINVAL
        assert refused == [lbm.LBM_SC_EINVAL] * 7
        grp.close()
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            ref.step(4)
            assert np.array_equal(b.get(), ref.get())
        assert b.observables(profile=False)[0]["step"] == 4
        b.set_step(12)
        b.step(2)
        ref.step(2)
        assert np.array_equal(b.get(), ref.get())
        assert b.observables(profile=False)[0]["step"] == ref.observables(profile=False)[0]["step"] == 14
        # a count of at least the box's own graph chunk (64 steps), which outside a capture it
        # replays from its internal graph, is recorded as plain launches too
        g2 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g2, stream=s):
            b.step(66)
        for _ in range(2):
            g2.replay()
            torch.cuda.synchronize()
            ref.step(66)
            assert np.array_equal(b.get(), ref.get())


@pytest.mark.parametrize("dims", SHAPES + [(100, 37, 9), (129, 5, 4), (101, 45, 7)])
@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED])
def test_full_row_tiles_one_step(dims, prec):
    """Full-row tiles (tile_x 0) against the oracle (FP64, 1e-11) and bitwise against the default
    x-y tiles (FP32) after one and three steps, on tiny, ragged and multi-tile boxes, with rows
    padded to whole lines and with packed rows (pitch nx; the default x-y tiles run on those too)."""
    say(f"full-row tiles dims={dims} prec={prec}")
    rho_ref = 1.5
    f = fp32_representable(inputs.random_populations(dims, 5 + sum(dims), W * 1.5, amp=0.3), rho_ref)
    G = 1.3 * lbm.lbm_sc_gc(0)
    outs = []
    launches = (None, (4, 3, 1, 0, 8, 0), (2, 3, 1, 0, 8, 0), (4, 2, 0, 0, 4, 0))
    if prec == lbm.LBM_SC_FP32_SHIFTED:
        launches += ((8, 2, 0, 0, 8, 0),)
    for packed in (0, 1):
        for launch in launches:
            with make_box(dims, prec=prec, rho_ref=rho_ref, packed=packed) as b:
                b.set(f)
                if launch:
                    b.set_launch(*launch)
                b.step(1)
                g1 = b.get()
                b.step(2)
                outs.append((g1, b.get()))
    if prec == lbm.LBM_SC_FP64:
        ref = core.step(f, G, 1.0, 0)
        assert rel_err(outs[1][0], ref) <= TOL64
        assert rel_err(outs[len(launches) + 1][0], ref) <= TOL64
    for g1, g3 in outs[1:]:
        assert np.array_equal(g1, outs[0][0]) and np.array_equal(g3, outs[0][1])


def droplet_cfg(prec=lbm.LBM_SC_FP64, n=32, R=8.0, seed=1, noise=1e-6, geom=lbm.LBM_SC_DROPLET,
                psi=lbm.LBM_SC_PSI_EXP, ratio=1.3):
    return lbm.config(n, n, n, psi=psi, geom=geom, prec=prec, tau=1.0, g_over_gc=ratio,
                      radius=R, width=2.0, noise_amp=noise, seed=seed)


@pytest.mark.parametrize("geom", [lbm.LBM_SC_DROPLET, lbm.LBM_SC_BUBBLE])
def test_initial_state_matches_oracle(geom):
    say(f"initial state geom={geom}")
    cfg = droplet_cfg(geom=geom, n=21, R=5.0, seed=12345)
    with lbm.Box(cfg) as b:
        info = b.info()
        f = b.get()
    G = info["G"]
    n0 = core.init_density(21, 21, 21, core.DROPLET, 5.0, 2.0, info["n_in"], info["n_out"], 1e-6,
                           12345)
    ref = core.init_populations(n0, G, core.PSI_EXP)
    assert rel_err(f, ref) <= 1e-13
    ng, nl, _ = eos.coexistence_rule(G, core.PSI_EXP)
    if geom == lbm.LBM_SC_DROPLET:
        assert abs(info["n_in"] - nl) < 1e-12 and abs(info["n_out"] - ng) < 1e-12
    else:
        assert abs(info["n_in"] - ng) < 1e-12 and abs(info["n_out"] - nl) < 1e-12


@pytest.fixture(scope="module")
def droplet32_run():
    """The 32^3 FP64 droplet (exp psi, G = 1.3 G_c, tau = 1, R = 8, width 2, noise 1e-6, seed 1)
    stepped 2000 times on the GPU and by the oracle, compared every 250 steps."""
    say("32^3 FP64 droplet: GPU vs oracle over 2000 steps")
    cfg = droplet_cfg()
    errs = []
    with lbm.Box(cfg) as b:
        info = b.info()
        G = info["G"]
        f = b.get()
        ref = f.copy()
        for k in range(8):
            b.step(250)
            ref = core.run(ref, G, 1.0, core.PSI_EXP, 250)
            g = b.get()
            errs.append(rel_err(g, ref))
        obs, prof = b.observables()
    return dict(errs=errs, g=g, ref=ref, obs=obs, prof=prof, info=info)


def test_droplet32_trajectory_parity(droplet32_run):
    errs = droplet32_run["errs"]
    say("relative errors every 250 steps:", errs)
    assert max(errs) <= TOL64


def test_droplet32_one_step_from_late_state(droplet32_run):
    """Per-step parity at step 2000 from the oracle's own state."""
    ref = droplet32_run["ref"]
    G = droplet32_run["info"]["G"]
    with make_box((32, 32, 32)) as b:
        b.set(ref)
        b.step(1)
        g = b.get()
    assert rel_err(g, core.step(ref, G, 1.0, core.PSI_EXP)) <= TOL64


def test_droplet32_observables(droplet32_run):
    obs = droplet32_run["obs"]
    G = droplet32_run["info"]["G"]
    o = observe.observables(droplet32_run["ref"], G, core.PSI_EXP)
    assert obs["step"] == 2000
    assert obs["finite"] == 1
    assert abs(obs["mass"] - o["mass"]) <= 1e-12 * o["mass"]
    assert abs(obs["mass"] - obs["mass0"]) <= 1e-12 * obs["mass0"]
    for k in ("n_center", "n_far", "P_in", "P_out"):
        assert abs(obs[k] - o[k]) <= 1e-11 * abs(o[k]), k
    assert abs(obs["dP"] - o["dP"]) <= 1e-9 * abs(o["dP"])
    for k in ("C", "R_s", "sigma_s", "R_e"):
        assert abs(obs[k] - o[k]) <= 1e-9 * abs(o[k]), k
    for c in range(3):
        assert abs(obs["com"][c] - o["com"][c]) <= 1e-10
        assert abs(obs["mom"][c] - o["mom"][c]) <= 1e-10
    assert np.abs(droplet32_run["prof"] - o["prof"]).max() <= 1e-11 * np.abs(o["prof"]).max()
    # a droplet: liquid inside and higher pressure inside (Laplace); its surface of tension lies
    # inside the equimolar surface and sigma_s is below the flat value (positive Tolman length
    # for droplets, Sec. 4); sigma_0 = 0.0495 is the flat lattice value at G/G_c = 1.3
    assert obs["n_center"] > 2.0 and obs["n_far"] < 0.6 and obs["dP"] > 0
    assert obs["C"] > 0 and 0 < obs["R_s"] < obs["R_e"] and 0 < obs["sigma_s"] < 0.0495


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED])
def test_packed_rows_equal_padded_rows(prec):
    """Initial state, 20 steps (default x-y tiles and full-row tiles), observables and profiles of
    a droplet and a slab with packed rows (pitch nx) are bitwise those of the padded box: the
    layout changes addresses only, the observation reductions run in canonical node order."""
    for dims, geom in (((45, 37, 21), lbm.LBM_SC_DROPLET), ((33, 20, 50), lbm.LBM_SC_SLAB)):
        say(f"packed rows prec={prec} dims={dims}")
        res = []
        for packed in (0, 1):
            cfg = lbm.config(*dims, psi=0, geom=geom, prec=prec, g_over_gc=1.4, radius=7.0,
                             slab_thickness=16.0, width=2.0, noise_amp=1e-6, seed=4,
                             packed_rows=packed)
            with lbm.Box(cfg) as b:
                f0 = b.get()
                b.step(10)
                o1, p1 = b.observables()
                b.set_launch(4, 5, 1, 0, 8, 0)
                b.step(10)
                o2, p2 = b.observables()
                res.append((f0, b.get(), o1, p1, o2, p2))
        a, c = res
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
        for oa, oc in ((a[2], c[2]), (a[4], c[4])):
            for k, v in oa.items():
                w = oc[k]
                if isinstance(v, float) and np.isnan(v):
                    assert np.isnan(w), k
                else:
                    assert np.array_equal(np.asarray(v), np.asarray(w)), k
        assert np.array_equal(a[3], c[3]) and np.array_equal(a[5], c[5])


def test_du_against_previous_call():
    say("du between observation calls")
    cfg = droplet_cfg(n=16, R=4.0)
    with lbm.Box(cfg) as b:
        f0 = b.get()
        o0, _ = b.observables()
        assert o0["has_du"] == 1 and o0["du_max"] == 0.0   # nothing moved since creation
        b.step(10)
        o1, _ = b.observables()
        f1 = b.get()
    G = 1.3 * lbm.lbm_sc_gc(0)
    _, u0 = core.velocity(f0, G, 0)
    _, u1 = core.velocity(f1, G, 0)
    d = np.abs(u1 - u0)
    assert abs(o1["du_max"] - d.max()) <= 1e-12 + 1e-9 * d.max()
    assert abs(o1["du_l1"] - d.sum() / 16**3) <= 1e-12 + 1e-9 * d.sum() / 16**3


def test_slab_observables_match_oracle():
    say("slab 8x6x48 FP64 observables")
    cfg = lbm.config(8, 6, 48, geom=lbm.LBM_SC_SLAB, prec=lbm.LBM_SC_FP64, g_over_gc=1.3,
                     slab_thickness=24.0, width=2.0, slab_axis=2)
    with lbm.Box(cfg) as b:
        b.step(300)
        obs, prof = b.observables()
        f = b.get()
        G = b.info()["G"]
    o = observe.observables(f, G, core.PSI_EXP, geom=core.SLAB, slab_axis=2)
    assert np.abs(prof - o["prof"]).max() <= 1e-12 * np.abs(o["prof"]).max()
    assert abs(obs["sigma0_flat"] - o["sigma0_flat"]) <= 1e-10 * abs(o["sigma0_flat"])
    assert abs(obs["pn_spread"] - o["pn_spread"]) <= 1e-12


def test_slab_along_x_equals_slab_along_z():
    """Rotating the box rotates the answer: the x-normal slab reports the z-normal profile."""
    say("slab orientation")
    outs = []
    for axis, dims in ((2, (6, 5, 40)), (0, (40, 5, 6))):
        cfg = lbm.config(*dims, geom=lbm.LBM_SC_SLAB, g_over_gc=1.2, slab_thickness=20.0,
                         width=2.0, slab_axis=axis)
        with lbm.Box(cfg) as b:
            b.step(200)
            obs, prof = b.observables()
        outs.append((obs, prof))
    (oz, pz), (ox, px) = outs
    assert np.abs(pz[0] - px[0]).max() < 1e-13
    assert abs(oz["sigma0_flat"] - ox["sigma0_flat"]) < 1e-12
    assert np.abs(pz[3] - px[1]).max() < 1e-13   # P_N: P^zz of the z slab = P^xx of the x slab


# FP32 against FP64 on the 32^3 droplet after 2000 steps, three times the measured values:
# largest density difference / n_l, relative dP difference, relative mass drift of the FP32 run
# (measured: FP32 arithmetic 8.0e-7, 9.6e-7, 8.2e-10; FP64 arithmetic 5.2e-7, 4.4e-7, 9.2e-9)
FP32_DROPLET_BOUNDS = {lbm.LBM_SC_FP32_SHIFTED: (2.5e-6, 3e-6, 3e-9),
                       lbm.LBM_SC_FP32_SHIFTED_MATH64: (1.6e-6, 1.4e-6, 3e-8)}


def test_fp32_vs_fp64_droplet_after_2000_steps():
    """FP32-shifted populations (single- or double-precision arithmetic) against FP64 on the 32^3
    droplet: densities, dP and the mass drift after 2000 steps within FP32_DROPLET_BOUNDS."""
    say("32^3 droplet FP32-shifted vs FP64, 2000 steps")
    res = {}
    for prec in (lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP32_SHIFTED_MATH64):
        with lbm.Box(droplet_cfg(prec=prec)) as b:
            b.step(2000)
            obs, prof = b.observables()
            n = b.get().sum(axis=0)
            res[prec] = (obs, prof, n, b.info())
    o64, _, n64, info = res[lbm.LBM_SC_FP64]
    nl = info["n_in"]
    for prec in (lbm.LBM_SC_FP32_SHIFTED, lbm.LBM_SC_FP32_SHIFTED_MATH64):
        o32, _, n32, _ = res[prec]
        drift = abs(o32["mass"] - o32["mass0"]) / o32["mass0"]
        say(f"prec {prec}: max |n32-n64| / n_l = {np.abs(n32 - n64).max() / nl:.3e}, "
            f"|dP32-dP64|/dP64 = {abs(o32['dP'] - o64['dP']) / o64['dP']:.3e}, "
            f"relative mass drift {drift:.3e}")
        b_n, b_dp, b_drift = FP32_DROPLET_BOUNDS[prec]
        assert np.abs(n32 - n64).max() <= b_n * nl
        assert abs(o32["dP"] - o64["dP"]) <= b_dp * o64["dP"]
        assert drift <= b_drift


def test_fp32_mass_drift_of_a_converged_droplet():
    """Once a droplet has converged its state repeats, and plain round-to-nearest of the rest
    population (which closes each node's mass) is biased the same way at every bulk node, so
    the FP32 mass drifts linearly; a dither pattern fixed in time still leaves a linear drift
    (measured 2.4e-8 here). The dither moved to an unrelated position every step leaves a random
    walk of the rounding errors: a 64^3 droplet (R = 16) converged for 8192 steps, then 32768
    more steps (measured 2.1e-9)."""
    say("FP32 mass drift of a converged 64^3 droplet")
    cfg = lbm.config(64, psi=0, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.3, radius=16.0, width=2.0, noise_amp=1e-6, seed=5)
    with lbm.Box(cfg) as b:
        b.step(8192)
        o1 = b.observables(profile=False)[0]
        b.step(32768)
        o2 = b.observables(profile=False)[0]
    drift = abs(o2["mass"] - o1["mass"]) / o1["mass"]
    say(f"converged 64^3 FP32: relative mass change over 32768 steps {drift:.3e}, "
        f"dP change {abs(o2['dP'] - o1['dP']) / o1['dP']:.2e}")
    assert abs(o2["dP"] - o1["dP"]) <= 1e-3 * o1["dP"]     # converged
    assert drift <= DRIFT_BOUND


def test_unstable_state_is_reported():
    say("non-finite state detection")
    dims = (8, 8, 8)
    f = inputs.random_populations(dims, 5, W * 1.0, amp=0.1)
    f[3, 2, 2, 2] = np.nan
    with make_box(dims) as b:
        b.set(f)
        obs, _ = b.observables(raise_unstable=False)
        assert obs["finite"] == 0
        with pytest.raises(lbm.LbmScError) as e:
            b.observables()
        assert e.value.code == lbm.LBM_SC_EUNSTABLE


def test_stream_copy_helper():
    import torch
    # 1 M floats plus a tail that is not a whole number of 1024-element blocks
    a = torch.arange((1 << 20) + 4 * 333, dtype=torch.float32, device="cuda")
    for lane in (4, 8, 16):
        b = torch.zeros_like(a)
        lbm.lbm_sc_stream_copy(a.data_ptr(), b.data_ptr(), a.numel() * 4, lane_bytes=lane)
        torch.cuda.synchronize()
        assert torch.equal(a, b), lane
    with pytest.raises(lbm.LbmScError):
        lbm.lbm_sc_stream_copy(a.data_ptr(), b.data_ptr(), 12)
    with pytest.raises(lbm.LbmScError):
        lbm.lbm_sc_stream_copy(a.data_ptr(), b.data_ptr(), 1 << 20, lane_bytes=2)
    # ranges that are not device memory, or run past their allocation, are refused before the
    # copy kernel could touch them
    host = torch.empty(1 << 22, dtype=torch.uint8, pin_memory=True)
    hp = (host.data_ptr() + 255) // 256 * 256
    with pytest.raises(lbm.LbmScError) as e:
        lbm.lbm_sc_stream_copy(hp, b.data_ptr(), 1 << 20)
    assert "device memory" in lbm.lbm_sc_last_error()
    big = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    small = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    n = 512 << 20
    with pytest.raises(lbm.LbmScError) as e:
        lbm.lbm_sc_stream_copy(big.data_ptr(), small.data_ptr(), n)
    assert e.value.code == lbm.LBM_SC_EINVAL
    p, q = big.data_ptr(), small.data_ptr()
    if not (p < q + n and q < p + n):
        assert "allocation" in lbm.lbm_sc_last_error()


def test_zero_steps_is_a_no_op():
    dims = (6, 5, 4)
    f = inputs.random_populations(dims, 8, W * 1.0, amp=0.1)
    with make_box(dims) as b:
        b.set(f)
        b.step(0)
        assert np.array_equal(b.get(), f)


def test_full_size_bench_workload_sampled():
    """The 256^3 FP32-shifted droplet (exp psi, G/G_c = 1.3, R = 60, width 2, noise 1e-6,
    seed 3) in the launch shape the benchmark times: one step checked on sampled nodes against
    the oracle's single-node collision, plus mass conservation over 20 steps."""
    say("256^3 FP32 bench workload, sampled one-step parity")
    cfg = lbm.config(256, 256, 256, psi=0, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.3, radius=60.0, width=2.0, noise_amp=1e-6, seed=3)
    rng = np.random.default_rng(2024)
    with lbm.Box(cfg) as b:
        G = b.info()["G"]
        f0 = b.get()
        b.step(1)
        f1 = b.get()
        o0 = b.observables(profile=False)[0]
        b.step(19)
        o1 = b.observables(profile=False)[0]
    # sampled nodes: random ones plus nodes across the interface and on the box faces
    pts = [tuple(rng.integers(0, 256, 3)) for _ in range(120)]
    pts += [(128 + 60 + d, 128, 128) for d in range(-3, 4)] + [(0, 0, 0), (255, 255, 255),
                                                                (255, 0, 128)]
    scale = np.abs(f0).max()
    worst = 0.0
    for (x, y, z) in pts:
        fs = core.collide_at(f0, G, 1.0, 0, x, y, z)
        for i in range(19):
            d = ((x + XI[i, 0]) % 256, (y + XI[i, 1]) % 256, (z + XI[i, 2]) % 256)
            worst = max(worst, abs(f1[i, d[2], d[1], d[0]] - fs[i]) / scale)
    say("worst sampled error / max|f| =", worst)
    # measured 7.2e-8 of max |f| on MI355X; the bound is three times that
    assert worst <= 2.2e-7
    assert abs(o1["mass"] - o0["mass"]) <= 1e-7 * o0["mass"]


def test_full_size_bench_workload_two_steps_sampled():
    """The same 256^3 droplet advanced by one launch of the kernel the benchmark times (two time
    steps per pass in the default shape). After two steps a node's populations depend only on
    the state within 4 nodes of it, so the oracle's two whole steps on the periodic 9^3
    neighbourhood of a sampled node give that node's exact result; every population of each
    sampled node is checked against it."""
    say("256^3 FP32 bench workload, sampled two-step parity")
    cfg = lbm.config(256, 256, 256, psi=0, geom=lbm.LBM_SC_DROPLET, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.3, radius=60.0, width=2.0, noise_amp=1e-6, seed=3)
    rng = np.random.default_rng(2026)
    with lbm.Box(cfg) as b:
        assert b.launch()["steps_per_pass"] == 2
        G = b.info()["G"]
        f0 = b.get()
        b.step(2)
        f2 = b.get()
    pts = [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(40)]
    pts += [(128 + 60 + d, 128, 128) for d in range(-3, 4)] + [(0, 0, 0), (255, 255, 255),
                                                                (255, 0, 128), (31, 32, 63)]
    scale = np.abs(f0).max()
    worst = 0.0
    for (x, y, z) in pts:
        worst = max(worst, np.abs(f2[:, z, y, x] - two_steps_at(f0, G, x, y, z)).max() / scale)
    say("worst sampled error / max|f| =", worst)
    # measured 7.4e-8 of max |f| on MI355X (two FP32 steps, the first stored and reloaded from
    # LDS as it would be from memory); the bound is three times that
    assert worst <= 2.2e-7


# FP32 at 480^3: three times the measured 6.5e-8 (one step) and 6.7e-8 (two-step launch)
@pytest.mark.parametrize("L,prec,tol", [(400, lbm.LBM_SC_FP64, TOL64),
                                         (480, lbm.LBM_SC_FP32_SHIFTED, 2.2e-7)])
def test_box_beyond_32bit_offsets_sampled(L, prec, tol):
    """Boxes whose population buffers span well over 4 GiB (9.7 GB at 400^3 FP64, 8.4 GB at
    480^3 FP32): one step of a noisy droplet checked on sampled nodes - many of them in the top
    planes, at the largest offsets - against the oracle's single-node collision; for FP32 also
    the next two steps, one launch of the two-steps-per-pass kernel, against the oracle's two
    steps from the same state; then mass conservation over 8 steps."""
    say(f"{L}^3 prec {prec}: sampled one-step parity beyond 32-bit offsets")
    cfg = lbm.config(L, L, L, psi=0, geom=lbm.LBM_SC_DROPLET, prec=prec, g_over_gc=1.3,
                     radius=0.3 * L, width=2.0, noise_amp=1e-6, seed=11)
    rng = np.random.default_rng(L)
    two = prec == lbm.LBM_SC_FP32_SHIFTED
    with lbm.Box(cfg) as b:
        G = b.info()["G"]
        f0 = b.get()
        b.step(1)
        f1 = b.get()
        o0 = b.observables(profile=False)[0]
        if two:
            assert b.launch()["steps_per_pass"] == 2
            b.step(2)
            f3 = b.get()
            b.step(6)
        else:
            b.step(8)
        o1 = b.observables(profile=False)[0]
    pts = [tuple(int(v) for v in rng.integers(0, L, 3)) for _ in range(40)]
    pts += [(int(rng.integers(0, L)), int(rng.integers(0, L)), L - 1 - int(rng.integers(0, 4)))
            for _ in range(40)]
    pts += [(L - 1, L - 1, L - 1), (0, L - 1, L - 1), (L - 1, 0, 0), (L // 2 + int(0.3 * L), L // 2, L // 2)]
    scale = np.abs(f0).max()
    worst = 0.0
    for (x, y, z) in pts:
        fs = core.collide_at(f0, G, 1.0, 0, x, y, z)
        for i in range(19):
            d = ((x + XI[i, 0]) % L, (y + XI[i, 1]) % L, (z + XI[i, 2]) % L)
            worst = max(worst, abs(f1[i, d[2], d[1], d[0]] - fs[i]) / scale)
    del f0
    say("worst sampled error / max|f| =", worst)
    assert worst <= tol
    if two:
        worst2 = max(np.abs(f3[:, z, y, x] - two_steps_at(f1, G, x, y, z)).max() / scale
                     for (x, y, z) in pts)
        del f3
        say("two-step launch: worst sampled error / max|f| =", worst2)
        assert worst2 <= tol
    del f1
    assert o1["finite"]
    mtol = 1e-12 if prec == lbm.LBM_SC_FP64 else 1e-7
    assert abs(o1["mass"] - o0["mass"]) <= mtol * o0["mass"]


def test_largest_z_plane_sampled():
    """The largest z-plane one buffer resource can address: 7296 x 7358 nodes in FP32 (the 19
    population planes of a z-plane, pitch padding included, take 4294717440 bytes, just under
    4 GiB; a plane one row larger is rejected before anything is allocated). One step of a noisy flat box checked on sampled nodes - the far corner
    of the plane included - against the oracle's single-node collision, then the next two steps
    (one launch of the two-steps-per-pass kernel on a box two planes high) against the oracle's
    two steps from the same state."""
    say("largest z-plane (7296 x 7358 x 2, FP32): sampled one-step parity")
    nx, ny, nz = 7296, 7358, 2
    cfg = lbm.config(nx, ny, nz, psi=0, geom=lbm.LBM_SC_SLAB, prec=lbm.LBM_SC_FP32_SHIFTED,
                     g_over_gc=1.3, slab_thickness=3000.0, width=2.0, slab_axis=0,
                     noise_amp=1e-6, seed=17)
    rng = np.random.default_rng(7296)
    with lbm.Box(cfg) as b:
        assert b.launch()["steps_per_pass"] == 2
        G = b.info()["G"]
        f0 = b.get()
        b.step(1)
        f1 = b.get()
        b.step(2)
        f3 = b.get()
    pts = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz)))
           for _ in range(30)]
    pts += [(nx - 1, ny - 1, nz - 1), (0, ny - 1, 0), (nx - 1, 0, 1), (nx // 2 + 1500, 17, 1)]
    scale = np.abs(f0).max()
    worst = 0.0
    for (x, y, z) in pts:
        fs = core.collide_at(f0, G, 1.0, 0, x, y, z)
        for i in range(19):
            d = ((x + XI[i, 0]) % nx, (y + XI[i, 1]) % ny, (z + XI[i, 2]) % nz)
            worst = max(worst, abs(f1[i, d[2], d[1], d[0]] - fs[i]) / scale)
    del f0
    say("worst sampled error / max|f| =", worst)
    # FP32 bounds: three times the measured 6.5e-8 (one step) and 7.2e-8 (two-step launch)
    assert worst <= 2.2e-7
    worst2 = max(np.abs(f3[:, z, y, x] - two_steps_at(f1, G, x, y, z)).max() / scale
                 for (x, y, z) in pts)
    del f1, f3
    say("two-step launch: worst sampled error / max|f| =", worst2)
    assert worst2 <= 2.2e-7
    with pytest.raises(lbm.LbmScError):
        lbm.lbm_sc_create(lbm.config(nx, ny + 1, nz, psi=0, geom=lbm.LBM_SC_SLAB,
                                     prec=lbm.LBM_SC_FP32_SHIFTED, g_over_gc=1.3,
                                     slab_thickness=3000.0, width=2.0, slab_axis=0))


def test_full_size_batched_workload_sampled():
    """The 64-box batched workload (seed 2105, L ~ U{48..160}, FP32-shifted) in one group with
    the full-row tiles the benchmark's tuner picks (4 nodes per thread, z chunks of 8, hipGraph
    chunks of 64 steps): one group step checked on sampled nodes of every 8th box against the
    oracle's single-node collision, then 64 graph-replayed steps conserving every box's mass."""
    import torch
    say("batched 64-box workload, sampled one-step parity")
    st = torch.cuda.Stream()
    spec = inputs.batched_boxes()
    boxes = [lbm.Box(lbm.config(b["L"], psi=0,
                                geom=lbm.LBM_SC_BUBBLE if b["bubble"] else lbm.LBM_SC_DROPLET,
                                prec=lbm.LBM_SC_FP32_SHIFTED, tau=1.0, g_over_gc=b["g_over_gc"],
                                radius=b["radius"], width=2.0, noise_amp=1e-6, seed=b["seed"],
                                stream=st.cuda_stream)) for b in spec]
    rng = np.random.default_rng(77)
    sub = list(range(0, len(boxes), 8))
    worst = 0.0
    with lbm.Group(st.cuda_stream) as g:
        g.set_launch(rows=4, waves=8, tile_x=0, z_chunk=8, prefetch=0, xcd_remap=1, persistent=0,
                     workers=0, graph_steps=64)
        g.set(boxes)
        f0 = {k: boxes[k].get() for k in sub}
        o0 = [b.observables(profile=False, raise_unstable=False)[0] for b in boxes]
        g.step(1)
        for k in sub:
            L = spec[k]["L"]
            f1 = boxes[k].get()
            G = boxes[k].info()["G"]
            scale = np.abs(f0[k]).max()
            pts = [tuple(int(v) for v in rng.integers(0, L, 3)) for _ in range(12)]
            pts += [(L - 1, L - 1, L - 1), (0, L - 1, L // 2), (L - 1, 0, 0)]
            for (x, y, z) in pts:
                fs = core.collide_at(f0[k], G, 1.0, 0, x, y, z)
                for i in range(19):
                    d = ((x + XI[i, 0]) % L, (y + XI[i, 1]) % L, (z + XI[i, 2]) % L)
                    worst = max(worst, abs(f1[i, d[2], d[1], d[0]] - fs[i]) / scale)
            del f0[k]
        g.step(64)
        o1 = [b.observables(profile=False, raise_unstable=False)[0] for b in boxes]
    for b in boxes:
        b.close()
    say("worst sampled error / max|f| =", worst)
    assert worst <= 1e-6
    for a, b in zip(o0, o1):
        assert b["finite"]
        assert abs(b["mass"] - a["mass"]) <= 1e-7 * a["mass"]


@pytest.mark.parametrize("prec", [lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED])
def test_checkpoint_resume_is_bitwise(prec):
    """A state saved with get_populations at step n and restored into a new box with
    set_populations + set_step(n) continues bitwise as the uninterrupted run (the step count
    also seeds the FP32 dither, so without set_step an FP32 state diverges at the rounding
    level); the observed step counter follows."""
    say(f"checkpoint/resume prec={prec}")
    cfg = droplet_cfg(prec=prec, n=20, R=5.0, seed=9)
    with lbm.Box(cfg) as a:
        a.step(37)
        saved = a.get()
        a.step(50)
        want = a.get()
        o_want = a.observables(profile=False)[0]
    with lbm.Box(cfg) as b:
        b.set(saved)
        b.set_step(37)
        b.step(50)
        assert np.array_equal(b.get(), want)
        o = b.observables(profile=False)[0]
        assert o["step"] == 87 and o["mass"] == o_want["mass"]
        with pytest.raises(lbm.LbmScError):
            b.set_step(-1)
    with lbm.Box(cfg) as c:
        c.set(saved)
        c.step(50)
        if prec == lbm.LBM_SC_FP64:
            assert np.array_equal(c.get(), want)     # no dither in double precision
        else:
            assert not np.array_equal(c.get(), want)
