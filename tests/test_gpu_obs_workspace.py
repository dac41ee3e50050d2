"""The observation workspace that the boxes of one device share (density, psi and momentum of
every node while observables, a population read-back or upload, or an initial state are
computed; each box keeps only its last observed velocity).

A box's observables and populations must not depend on which other boxes exist, how large they
are, in which order they are observed, or whether another thread observes at the same time:
every result is compared bitwise with the same box's calls made with no other box alive.
"""
import sys
import threading

import numpy as np
import pytest

import paper_2105_08772_amd as lbm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_cfg():
    return lbm.config(24, 20, 18, prec=lbm.LBM_SC_FP64, g_over_gc=1.3, radius=5.0, width=2.0,
                      noise_amp=1e-6, seed=5)


def large_cfg():
    return lbm.config(40, 33, 30, prec=lbm.LBM_SC_FP32_SHIFTED, g_over_gc=1.4, radius=9.0,
                      width=2.0, noise_amp=1e-6, seed=6)


def same(a, b):
    for k, v in a.items():
        w = b[k]
        if isinstance(v, (list, tuple, np.ndarray)):
            assert np.array_equal(np.asarray(v), np.asarray(w), equal_nan=True), k
        elif isinstance(v, float) and np.isnan(v):
            assert np.isnan(w), k
        else:
            assert v == w, k


def script(box, rounds):
    """Steps and observations of one box; the observations (with du against the previous one)
    and the final populations."""
    out = []
    for k in range(rounds):
        box.step(6 + 2 * k)
        o, prof = box.observables()
        out.append((o, prof))
    return out, box.get()


def alone(cfg, rounds):
    with lbm.Box(cfg) as b:
        return script(b, rounds)


def test_observations_do_not_depend_on_the_other_boxes():
    ref_s = alone(small_cfg(), 3)
    ref_l = alone(large_cfg(), 3)
    say("two boxes, observed in turn; the larger one leaves first")
    s = lbm.Box(small_cfg())
    big = lbm.Box(large_cfg())   # the workspace grows while the small box holds state
    obs_s, obs_l = [], []
    for k in range(3):
        s.step(6 + 2 * k)
        big.step(6 + 2 * k)
        obs_l.append(big.observables())
        obs_s.append(s.observables())
    fl = big.get()
    big.close()
    fs = s.get()                 # read back through the workspace the small box now shares alone
    for (o, p), (ro, rp) in zip(obs_s, ref_s[0]):
        same(o, ro)
        assert np.array_equal(p, rp)
    for (o, p), (ro, rp) in zip(obs_l, ref_l[0]):
        same(o, ro)
        assert np.array_equal(p, rp)
    assert np.array_equal(fs, ref_s[1]) and np.array_equal(fl, ref_l[1])
    # set (an upload through the workspace) and observe again after the large box has gone
    s.set(fs)
    o, _ = s.observables()
    # set observes the state once (its mass is the new reference), so the velocity change of an
    # unchanged state is exactly 0
    assert o["step"] == 0 and o["has_du"] and o["du_max"] == 0.0 and o["du_l1"] == 0.0
    assert np.array_equal(s.get(), fs)
    s.close()


def test_concurrent_threads_share_the_workspace():
    cfgs = [small_cfg(), large_cfg(), small_cfg()]
    refs = [alone(c, 4) for c in cfgs]
    say("three boxes, one thread each")
    boxes = [lbm.Box(c) for c in cfgs]
    res, errs = [None] * 3, []

    def run(i):
        try:
            res[i] = script(boxes[i], 4)
        except Exception as e:    # reported below: a thread's exception is not the test's
            errs.append(e)

    ts = [threading.Thread(target=run, args=(i,)) for i in range(3)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for b in boxes:
        b.close()
    assert not errs, errs
    for (obs, f), (robs, rf) in zip(res, refs):
        for (o, p), (ro, rp) in zip(obs, robs):
            same(o, ro)
            assert np.array_equal(p, rp)
        assert np.array_equal(f, rf)
