"""The Tolman analysis on synthetic Laplace data whose sigma_0 and delta are known."""
import math

import numpy as np
import pytest

from paper_2105_08772_amd import analysis


def synthetic_runs(g, sigma0, delta, radii, k2=0.0, dhat=None):
    runs = []
    for R in radii:
        for bubble in (False, True):
            kappa = (-1.0 if bubble else 1.0) / R
            sigma_s = sigma0 * (1 - 2 * delta * kappa + k2 * kappa ** 2)
            dP = 2 * sigma_s / R
            dh = 0.0 if dhat is None else dhat
            Re = R + (-1.0 if bubble else 1.0) * dh
            runs.append(dict(g_over_gc=g, bubble=bubble, obs=dict(R_s=R, dP=dP, R_e=Re)))
    return runs


def test_recovers_sigma0_and_delta_from_droplets_and_bubbles():
    runs = synthetic_runs(1.3, 0.05, 0.8, [10, 12, 15, 20, 25, 30], dhat=0.6)
    out = analysis.analyse(runs)[1.3]
    assert out["sigma0"] == pytest.approx(0.05, rel=1e-12)
    assert out["delta"] == pytest.approx(0.8, rel=1e-10)
    assert out["delta_hat0"] == pytest.approx(0.6, rel=1e-10)
    # bubbles sit at negative curvature, with sigma_s above sigma_0 for delta > 0
    for p in out["points"]:
        assert (p["kappa"] < 0) == p["bubble"]
        assert (p["sigma_s"] > 0.05) == p["bubble"]


def test_second_order_term_cancels_between_droplets_and_bubbles():
    """With the same radii on both sides, a curvature-squared term shifts sigma_0 but not the
    linear slope: delta is recovered exactly."""
    runs = synthetic_runs(1.2, 0.03, 1.5, [12, 16, 24], k2=4.0)
    out = analysis.analyse(runs)[1.2]
    assert out["delta"] * out["sigma0"] == pytest.approx(1.5 * 0.03, rel=1e-10)


def test_mean_field_exponents():
    g1 = np.array([0.05, 0.1, 0.2, 0.3])
    s = analysis.scaling_exponent(g1, 0.3 * g1 ** 1.5)
    assert s["exponent"] == pytest.approx(1.5, abs=1e-12)
    assert s["prefactor"] == pytest.approx(0.3, rel=1e-12)
    d = analysis.scaling_exponent(g1, 0.2 / g1)
    assert d["exponent"] == pytest.approx(-1.0, abs=1e-12)


def test_laplace_point_rejects_runs_without_surface_of_tension():
    with pytest.raises(ValueError):
        analysis.laplace_point(dict(R_s=float("nan"), dP=0.0, R_e=3.0), False)
    k, s, Rs, Re = analysis.laplace_point(dict(R_s=10.0, dP=0.01, R_e=10.5), True)
    assert k == -0.1 and s == pytest.approx(0.05) and math.isclose(Re, 10.5)


def test_a_coupling_with_one_curvature_gets_nan_fits():
    runs = synthetic_runs(1.3, 0.05, 0.8, [10, 12]) + synthetic_runs(1.5, 0.07, 0.6, [20])[:1]
    out = analysis.analyse(runs)
    assert out[1.3]["sigma0"] == pytest.approx(0.05, rel=1e-12)
    assert len(out[1.5]["points"]) == 1
    assert all(math.isnan(out[1.5][k]) for k in ("sigma0", "delta", "delta_hat0"))
    with pytest.raises(ValueError):
        analysis.fit_line([1.0, 1.0], [2.0, 3.0])
