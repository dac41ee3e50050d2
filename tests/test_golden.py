"""The oracle against the numbers the paper prints and the generator's published outputs, read
from the cited fixtures in tests/golden/ (CPU only)."""
import json
import os

import numpy as np

from oracle import core, eos, reduced

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


PAPER = load("paper_printed_values.json")
XI, W_LAT, W_SC = core.tables()


def frac(v):
    return v[0] / v[1]


def test_printed_critical_couplings():
    cs2 = frac(PAPER["cs2"]["value"])
    for name, kind in (("exp", core.PSI_EXP), ("oneminus", core.PSI_ONEMINUS)):
        entry = PAPER["critical_coupling_times_cs2"][name]
        _, Gc = eos.critical_point(kind)
        assert round(Gc * cs2, entry["decimals"]) == entry["value"]


def test_printed_force_weights_3d_and_e2():
    entry = PAPER["force_weights_3d"]
    sq = (XI ** 2).sum(axis=1)
    assert np.all(W_SC[sq == 1] == frac(entry["W1"]))
    assert np.all(W_SC[sq == 2] == frac(entry["W2"]))
    # e_2 of Eq. (bulkp): sum_a W_a xi_ax^2
    assert abs(float((W_SC * XI[:, 0] ** 2).sum()) - PAPER["e2"]["value"]) < 1e-15


def test_printed_force_weights_2d():
    """The D2Q9 code used for the flat runs carries the printed 2D weights, and they are what the
    3D weights sum to over velocities with the same (x, z) projection."""
    entry = PAPER["force_weights_2d"]
    c = reduced.D2Q9.c
    W = reduced.D2Q9.W
    sq = (c ** 2).sum(axis=1)
    assert np.allclose(W[sq == 1], frac(entry["W1"]), rtol=0, atol=1e-16)
    assert np.allclose(W[sq == 2], frac(entry["W2"]), rtol=0, atol=1e-16)
    # projection of D3Q19 onto (x, z)
    proj = {}
    for i in range(1, 19):
        key = (int(XI[i, 0]), int(XI[i, 2]))
        if key != (0, 0):
            proj[key] = proj.get(key, 0.0) + W_SC[i]
    for (cx, cz), v in proj.items():
        want = frac(entry["W1"]) if cx * cx + cz * cz == 1 else frac(entry["W2"])
        assert abs(v - want) < 1e-15


def test_bulk_pressure_uses_printed_e2_and_cs2():
    cs2 = frac(PAPER["cs2"]["value"])
    e2 = PAPER["e2"]["value"]
    for kind in (core.PSI_EXP, core.PSI_ONEMINUS):
        G = eos.G_of(1.3, kind)
        for n in (0.3, 1.0, 2.7):
            psi = eos.psi(n, kind)[0]
            assert abs(eos.pressure(n, G, kind) - (cs2 * n + 0.5 * cs2 * G * e2 * psi * psi)) < 1e-15


def test_sweep_protocol_values():
    """The printed couplings lie above the critical point and the printed box sizes are odd (the
    centre node floor(L/2) is then the exact centre); the observation interval is 2^11."""
    assert all(g > 0 for g in PAPER["couplings_minus_one"]["values"])
    assert all(L % 2 == 1 for L in PAPER["box_sizes"]["values"])
    assert PAPER["convergence"]["observation_interval"] == 2 ** 11


def test_splitmix64_published_outputs_drive_the_noise():
    fix = load("splitmix64_outputs.json")
    for case in fix["cases"]:
        state = int(case["state"], 16)
        out = int(case["output"], 16)
        u = (out >> 11) * 2.0 ** -53
        # noise(seed, k, amp) = amp * (2u - 1) with u from SplitMix64(seed ^ k)
        assert core.noise(state, 0, 1.0) == 2.0 * u - 1.0
        assert core.noise(0, state, 0.5) == 0.5 * (2.0 * u - 1.0)
