"""Equation of state of the Shan-Chen fluid: bulk pressure, critical coupling, spinodals and the
leading-order flat-interface coexistence rule.

TEST INFRASTRUCTURE ONLY (oracle): used by tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg, never by the product package.

Sources (arXiv:2105.08772):
  - bulk pressure P(n) = n c_s^2 + (G c_s^2 e_2 / 2) psi(n)^2 with e_2 = 1, Eq. (bulkp);
  - critical coupling G_c from dP/dn = d^2P/dn^2 = 0 (text after Eq. bulkp); the paper prints
    G_c c_s^2 = -2.463 for psi = exp(-1/n) and -1.333 for psi = 1 - exp(-n) (Sec. 4);
  - "equilibrium values of n_g, n_l for a flat interface" (Sec. 4) are not given in closed form.
    Reading used here: on the lattice a flat steady interface at tau = 1 keeps the normal
    pressure P_N(z) = c_s^2 n + (G c_s^2/4) psi(z) (psi(z+1) + psi(z-1)) exactly constant
    (the mechanical-equilibrium property stated after Eq. sm:pt). Expanding psi(z+-1) to second
    order gives p0 - P(n) = (G c_s^2/4) psi psi''; multiplying by psi'/psi makes the right side
    a total derivative, so  int_{n_g}^{n_l} (p0 - P(n)) psi'(n)/psi(n) dn = 0  together with
    P(n_g) = P(n_l) = p0. The exact lattice values come from relaxing a flat interface
    (oracle.reduced.lattice_coexistence).
"""
import warnings

import numpy as np
from scipy import integrate, optimize

CS2 = 1.0 / 3.0
E2 = 1.0  # e_2 of Eq. (bulkp) for W(1) = 1/6, W(2) = 1/12

PSI_EXP = 0
PSI_ONEMINUS = 1


def psi(n, kind):
    """psi(n) and its first two derivatives d/dn, d^2/dn^2 (Sec. 4 pseudopotentials)."""
    if kind == PSI_EXP:
        p = np.exp(-1.0 / n)
        d1 = p / n**2
        d2 = p * (1.0 / n**4 - 2.0 / n**3)
        return p, d1, d2
    e = np.exp(-n)
    return 1.0 - e, e, -e


def dlogpsi(n, kind):
    """psi'(n)/psi(n), written so that it stays finite as n -> 0."""
    if kind == PSI_EXP:
        return 1.0 / (n * n)
    return 1.0 / np.expm1(n)


def pressure(n, G, kind):
    """Bulk pressure, Eq. (bulkp)."""
    p, _, _ = psi(n, kind)
    return n * CS2 + 0.5 * G * CS2 * E2 * p * p


def dpressure(n, G, kind):
    """dP/dn and d^2P/dn^2 of Eq. (bulkp)."""
    p, d1, d2 = psi(n, kind)
    return CS2 + G * CS2 * E2 * p * d1, G * CS2 * E2 * (d1 * d1 + p * d2)


def critical_point(kind):
    """(n_c, G_c): d^2P/dn^2 = 0 fixes n_c independently of G (it is the inflection of psi^2),
    then dP/dn = 0 at n_c fixes G_c. Solved numerically by bracketing."""
    def curv(n):  # d^2 (psi^2) / dn^2 / 2
        p, d1, d2 = psi(n, kind)
        return d1 * d1 + p * d2

    lo, hi = (0.2, 5.0)
    n_c = optimize.brentq(curv, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps)
    p, d1, _ = psi(n_c, kind)
    G_c = -CS2 / (CS2 * E2 * p * d1)
    return n_c, G_c


def Gc(kind):
    return critical_point(kind)[1]


def spinodals(G, kind):
    """Densities where dP/dn = 0 (gas-side maximum, liquid-side minimum) for G < G_c."""
    n_c, G_c = critical_point(kind)
    if not G < G_c:
        raise ValueError("no spinodal above the critical coupling")
    f = lambda n: dpressure(n, G, kind)[0]
    n_g = optimize.brentq(f, 1e-3, n_c, xtol=1e-15)
    n_l = optimize.brentq(f, n_c, 50.0, xtol=1e-15)
    return n_g, n_l


def _branch_roots(p0, G, kind):
    s_g, s_l = spinodals(G, kind)
    h = lambda n: pressure(n, G, kind) - p0
    n_g = optimize.brentq(h, min(1e-9, 0.5 * p0), s_g, xtol=1e-15)
    n_l = optimize.brentq(h, s_l, 200.0, xtol=1e-15)
    return n_g, n_l


def rule_residual(p0, G, kind):
    """int_{n_g}^{n_l} (p0 - P(n)) psi'(n)/psi(n) dn for the outer roots of P = p0."""
    n_g, n_l = _branch_roots(p0, G, kind)

    def integrand(n):
        return (p0 - pressure(n, G, kind)) * dlogpsi(n, kind)

    with warnings.catch_warnings():
        # at deep quench the integrand spans many decades; quad's round-off notice is benign here
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(integrand, n_g, n_l, epsabs=1e-15, epsrel=1e-13, limit=400)
    return val


def coexistence_rule(G, kind):
    """(n_g, n_l, p0) from the leading-order flat-interface rule in the module docstring."""
    s_g, s_l = spinodals(G, kind)
    p_hi = pressure(s_g, G, kind)
    p_lo = max(pressure(s_l, G, kind), 0.0)
    eps = 1e-9 * (p_hi - p_lo)
    # the residual is positive just below the gas-side spinodal pressure and negative near the
    # lower end of the coexistence range; scan down from the top for the first sign change
    grid = p_lo + (p_hi - p_lo) * (1.0 - np.geomspace(1e-9, 1.0, 60))
    grid[-1] = p_lo + eps
    hi, r_hi = p_hi - eps, rule_residual(p_hi - eps, G, kind)
    for p in grid[1:]:
        r = rule_residual(p, G, kind)
        if np.sign(r) != np.sign(r_hi):
            lo = p
            break
        hi, r_hi = p, r
    else:
        raise ValueError("no coexistence pressure found")
    p0 = optimize.brentq(lambda p: rule_residual(p, G, kind), lo, hi,
                         xtol=1e-15, rtol=4 * np.finfo(float).eps)
    n_g, n_l = _branch_roots(p0, G, kind)
    return n_g, n_l, p0


def G_of(g_over_gc, kind):
    return g_over_gc * Gc(kind)


__all__ = ["psi", "pressure", "dpressure", "critical_point", "Gc", "spinodals",
           "coexistence_rule", "rule_residual", "dlogpsi", "G_of", "CS2", "E2", "PSI_EXP", "PSI_ONEMINUS"]
