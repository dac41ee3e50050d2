"""Tolman-length analysis of converged droplets and bubbles (Sec. 3 and Sec. 4 of
arXiv:2105.08772), on the observables that the library reports for each box.

For each converged run: the surface of tension R_s and sigma_s = dP R_s / 2 (Eq. Laplace2nd at
the minimum of sigma[R]), the curvature 1/R_s taken positive for droplets and negative for
bubbles, and the equimolar radius R_e. For one coupling, the points (1/R_s, sigma_s) are fitted
by the first-order expansion sigma_s = sigma_0 (1 - 2 delta / R_s) (Eq. sigma_c without the
second-order term): the intercept is sigma_0 (the flat limit R_s^-1 -> 0) and the slope is
-2 delta sigma_0. The alternative definition delta_hat = +-(R_e - R_s) (plus for droplets, minus
for bubbles) is extrapolated linearly in 1/R_s to the flat limit. Across couplings the
mean-field scalings sigma_0 ~ (G/G_c - 1)^mu and delta ~ (G/G_c - 1)^lambda are fitted on a
log-log scale (the paper reports mu = 3/2 and lambda close to -1).
"""
import math

import numpy as np


def laplace_point(obs, bubble):
    """(signed curvature, sigma_s, R_s, R_e) of one converged run from its observables."""
    Rs = obs["R_s"]
    if not (Rs > 0):
        raise ValueError("run has no surface of tension (dP <= 0 or C <= 0)")
    sigma_s = 0.5 * obs["dP"] * Rs
    kappa = (-1.0 if bubble else 1.0) / Rs
    return kappa, sigma_s, Rs, obs["R_e"]


def fit_line(x, y, w=None):
    """Weighted least-squares line y = a + b x; returns (a, b, residual rms). A line needs at
    least two distinct abscissae (ValueError otherwise)."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    if len(np.unique(x)) < 2:
        raise ValueError("a line fit needs at least two distinct abscissae")
    w = np.ones_like(x) if w is None else np.asarray(w, dtype=float)
    A = np.stack([np.ones_like(x), x], axis=1) * np.sqrt(w)[:, None]
    coef, *_ = np.linalg.lstsq(A, y * np.sqrt(w), rcond=None)
    res = y - (coef[0] + coef[1] * x)
    return float(coef[0]), float(coef[1]), float(np.sqrt(np.mean(res ** 2)))


def tolman_fit(kappa, sigma_s):
    """sigma_0 and delta from sigma_s = sigma_0 (1 - 2 delta kappa) (kappa = signed 1/R_s)."""
    a, b, rms = fit_line(kappa, sigma_s)
    return dict(sigma0=a, delta=-b / (2.0 * a), rms=rms, npoints=len(kappa))


def delta_hat(Re, Rs, bubble):
    """Alternative Tolman length +-(R_e - R_s): plus for droplets, minus for bubbles."""
    return (-1.0 if bubble else 1.0) * (Re - Rs)


def delta_hat_flat(kappa, dhat):
    """Flat-interface limit of delta_hat: intercept of a straight line in the signed curvature."""
    a, b, rms = fit_line(kappa, dhat)
    return dict(delta_hat0=a, delta_hat_slope=b, delta_hat_rms=rms)


def scaling_exponent(g_minus_1, values):
    """Exponent and prefactor of values = A (G/G_c - 1)^e, by a line in log-log."""
    a, b, rms = fit_line(np.log(g_minus_1), np.log(values))
    return dict(exponent=b, prefactor=math.exp(a), rms_log=rms)


def analyse(runs):
    """runs: iterable of dicts with keys g_over_gc, bubble, obs (converged observables).
    Returns, per coupling, the points and both fits; runs whose sigma[R] has no minimum
    (dP <= 0 or C <= 0) are counted under "no_minimum" and left out. A coupling with fewer than
    two distinct curvatures keeps its points and gets NaN fits."""
    by_g = {}
    skipped = {}
    for r in runs:
        obs = r["obs"]
        if not (obs["R_s"] > 0):
            g = round(r["g_over_gc"], 10)
            skipped[g] = skipped.get(g, 0) + 1
            continue
        k, s, Rs, Re = laplace_point(obs, r["bubble"])
        by_g.setdefault(round(r["g_over_gc"], 10), []).append((k, s, Rs, Re, r["bubble"]))
    out = {}
    for g, pts in sorted(by_g.items()):
        kap = [p[0] for p in pts]
        sig = [p[1] for p in pts]
        dh = [delta_hat(p[3], p[2], p[4]) for p in pts]
        if len(set(kap)) >= 2:
            fits = dict(tolman_fit(kap, sig), **delta_hat_flat(kap, dh))
        else:
            nan = float("nan")
            fits = dict(sigma0=nan, delta=nan, rms=nan, npoints=len(kap), delta_hat0=nan,
                        delta_hat_slope=nan, delta_hat_rms=nan)
        out[g] = dict(points=[dict(kappa=p[0], sigma_s=p[1], R_s=p[2], R_e=p[3], bubble=p[4])
                              for p in pts],
                      no_minimum=skipped.get(g, 0), **fits)
    return out
