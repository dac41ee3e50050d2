"""Observables and surface-tension post-processing computed from a full FP64 population state.

TEST INFRASTRUCTURE ONLY (oracle): used by tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg, never by the product package.

Sources (arXiv:2105.08772):
  - n = sum f, physical velocity u = (sum xi f + F/2)/n (Sec. 2);
  - lattice pressure tensor, Eq. (sm:pt) (computed by the C oracle);
  - P_in at the box centre (floor(L/2), floor(L/2), floor(L/2)) and P_out at the far corner
    (Sec. 4); reading for even L: the far probe is (c + floor(L/2)) mod L on each axis, which is
    L - 1 for odd L as in the paper;
  - generalized surface tension sigma[R], Eq. (gen_sigma), evaluated along the x axis with
    P_T = P^yy (Sec. 3), and its minimum R_s;
  - equimolar radius R_e from M = 4 pi R_e^3 n_in/3 + (V - 4 pi R_e^3/3) n_out (Sec. 4);
  - flat sigma_0 = int_{L/2}^{L} (P_N - P_T) dx (Sec. 4);
  - velocity-change criterion du = L^-3 sum_x sum_a |u^a(t + dt) - u^a(t)| (Sec. 4).

Reading for the sigma[R] integral (P_J is a Heaviside jump, so it is integrated exactly):
  sigma[R] = int_0^inf (r/R)^2 [P_J(r;R) - P_T(r)] dr = dP R/3 + C/R^2,
  C = int_0^{R_out} r^2 (P_out - P_T(r)) dr (trapezoid on the lattice nodes r = 0..R_out,
  R_out = L - 1 - c). Its minimum is at R_s = (6 C/dP)^(1/3) with sigma_s = dP R_s/2.
"""
import numpy as np

from . import core

AXES = "xyz"


def centre(dims):
    return tuple(L // 2 for L in dims)


def far_probe(dims):
    return tuple((L // 2 + L // 2) % L for L in dims)


def min_image(v, c, L):
    d = v - c
    d = np.where(2 * d > L, d - L, d)
    d = np.where(2 * d < -L, d + L, d)
    return d


def sigma_C(r, PT, P_out):
    """C = int r^2 (P_out - P_T(r)) dr by the trapezoid rule on the given nodes."""
    y = r * r * (P_out - PT)
    return float(np.sum(0.5 * (y[1:] + y[:-1]) * np.diff(r)))


def sigma_of_R(R, dP, C):
    """Eq. (gen_sigma) with the jump part integrated exactly: dP R/3 + C/R^2."""
    R = np.asarray(R, dtype=float)
    return dP * R / 3.0 + C / (R * R)


def surface_of_tension(dP, C):
    """Closed-form minimiser of sigma[R]: R_s = (6C/dP)^(1/3), sigma_s = dP R_s / 2."""
    if not (dP > 0 and C > 0):
        return float("nan"), float("nan")
    Rs = (6.0 * C / dP) ** (1.0 / 3.0)
    return Rs, 0.5 * dP * Rs


def surface_of_tension_numeric(dP, C, R_lo, R_hi, npts=201, rounds=4):
    """Minimum of sigma[R] located numerically as the paper describes: sample sigma[R] on a grid,
    interpolate the minimum with the parabola through the lowest sample and its neighbours, and
    repeat on a finer grid around it."""
    lo, hi = R_lo, R_hi
    for _ in range(rounds):
        Rg = np.linspace(lo, hi, npts)
        s = sigma_of_R(Rg, dP, C)
        k = int(np.argmin(s))
        k = min(max(k, 1), npts - 2)
        x0, x1, x2 = Rg[k - 1], Rg[k], Rg[k + 1]
        y0, y1, y2 = s[k - 1], s[k], s[k + 1]
        den = (x0 - x1) * (x0 - x2) * (x1 - x2)
        a = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / den
        b = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / den
        xm = -b / (2 * a)
        h = Rg[1] - Rg[0]
        lo, hi = xm - 2 * h, xm + 2 * h
    return float(xm), float(sigma_of_R(xm, dP, C))


def equimolar_radius(M, V, n_in, n_out):
    """R_e from M = 4 pi R_e^3 n_in / 3 + (V - 4 pi R_e^3 / 3) n_out (IEEE division: infinite or
    NaN when n_in equals n_out, as in the library)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = np.float64(3.0) * (M - V * n_out) / (np.float64(4.0 * np.pi) * (n_in - n_out))
    return float(np.cbrt(v))


def observables(f, G, kind, geom=core.DROPLET, slab_axis=2, u_prev=None):
    """All observables of one state (pre-collision populations f, shape (19, nz, ny, nx)).

    Returns a dict with mass, mom (physical momentum sum), com, n_center, n_far, P_in, P_out,
    dP, C, R_s, sigma_s, R_e, sigma0_flat, pn_spread, du_l1, du_max, finite, the profile
    arrays prof (4, L) = [n, Pxx, Pyy, Pzz] and the velocity field u (for the next du)."""
    nz, ny, nx = f.shape[1:]
    dims = (nx, ny, nz)
    n, _ = core.density(f, kind)
    j, u = core.velocity(f, G, kind)
    P = core.pressure_tensor(f, G, kind)
    mass = float(n.sum())
    mom = [float((u[c] * n).sum()) for c in range(3)]
    c = centre(dims)
    far = far_probe(dims)
    com = []
    for a in range(3):
        L = dims[a]
        coord = np.arange(L)
        d = min_image(coord, c[a], L).astype(float)
        if L % 2 == 0:
            d[np.abs(2 * d) == L] = 0.0  # the node half a box away sits on both sides: weight 0
        shape = [1, 1, 1]
        shape[2 - a] = L
        com.append(c[a] + float((n * d.reshape(shape)).sum()) / mass)
    cx, cy, cz = c
    fx, fy, fz = far
    out = dict(mass=mass, mom=mom, com=com)
    out["n_center"] = float(n[cz, cy, cx])
    out["n_far"] = float(n[fz, fy, fx])
    out["P_in"] = float(P[0, cz, cy, cx])
    out["P_out"] = float(P[0, fz, fy, fx])
    out["dP"] = out["P_in"] - out["P_out"]
    if geom == core.SLAB:
        a = slab_axis
        sum_axes = tuple(k for k in range(3) if k != 2 - a)
        b = (a + 1) % 3
        prof = np.stack([n.mean(axis=sum_axes)] + [P[k].mean(axis=sum_axes) for k in range(3)])
        PN = prof[1 + a]
        PT = prof[1 + b]
        L = dims[a]
        out["sigma0_flat"] = float(np.sum(PN[L // 2:] - PT[L // 2:]))
        out["pn_spread"] = float(PN.max() - PN.min())
        out["C"] = float("nan")
        out["R_s"] = float("nan")
        out["sigma_s"] = float("nan")
        out["R_e"] = float("nan")
    else:
        prof = np.stack([n[cz, cy, :]] + [P[k, cz, cy, :] for k in range(3)])
        R_out = nx - 1 - cx
        r = np.arange(R_out + 1, dtype=float)
        PT = P[1, cz, cy, cx:cx + R_out + 1]
        C = sigma_C(r, PT, out["P_out"])
        Rs, ss = surface_of_tension(out["dP"], C)
        out["C"] = C
        out["R_s"] = Rs
        out["sigma_s"] = ss
        out["R_e"] = equimolar_radius(mass, nx * ny * nz, out["n_center"], out["n_far"])
        out["sigma0_flat"] = float("nan")
        out["pn_spread"] = float("nan")
    out["prof"] = prof
    if u_prev is not None:
        du = np.abs(u - u_prev)
        out["du_l1"] = float(du.sum()) / (nx * ny * nz)
        out["du_max"] = float(du.max())
    else:
        out["du_l1"] = float("nan")
        out["du_max"] = float("nan")
    out["finite"] = int(np.all(np.isfinite(f)) and np.all(n > 0))
    out["u"] = u
    return out
