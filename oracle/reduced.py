"""Reduced-dimension Shan-Chen lattices (D1Q3 and D2Q9) written independently of the 3D C oracle.

TEST INFRASTRUCTURE ONLY (oracle): used by tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg, never by the product package.

Why they exist. A D3Q19 state that is uniform along y and mirror-symmetric in y at every node
evolves exactly as a D2Q9 state: summing the D3Q19 weights over velocities with the same (x, z)
projection gives 4/9, 1/9, 1/36, and summing the forcing weights W gives the 2D values
W(1) = 1/3, W(2) = 1/12 that the paper uses for its flat-interface runs (Sec. 4). Uniform along
two axes, the same reduction gives D1Q3 with weights 2/3, 1/6, 1/6 and a single forcing weight
W = 1/2. These codes therefore pin the 3D oracle on reduced states, and the 2D one reproduces the
paper's flat-interface sigma_0 measurement.

Each code applies the same published method as the 3D one (Sec. 2: Eq. lbm with BGK
Eq. sm:omega_i, the Guo term, the second-order equilibrium with the 1/2 on the quadratic term,
u_eq = (sum xi f + F/2)/n; Eq. SCForce; Eq. sm:pt), vectorised with numpy over the lattice.
Arrays: populations (Q, *space); space is (L,) in 1D and (ny, nx) in 2D, x fastest.
"""
import numpy as np

from . import eos

CS2 = 1.0 / 3.0


class Lattice:
    def __init__(self, c, w, W):
        self.c = np.asarray(c, dtype=np.int64)      # (Q, d)
        self.w = np.asarray(w, dtype=np.float64)    # lattice weights
        self.W = np.asarray(W, dtype=np.float64)    # forcing weights (0 for the rest vector)
        self.Q, self.d = self.c.shape

    # -- fields -----------------------------------------------------------------------------
    def _axes(self):
        return tuple(range(self.d))

    def _shift(self, a, vec):
        """Value at x + vec stored at x (periodic)."""
        # numpy axes of a field: (..., y, x) for d=2; (z,) for d=1. vec components follow
        # the same order as self.c: (x,) in 1D, (x, y) in 2D.
        shifts = tuple(-int(v) for v in vec[::-1])
        return np.roll(a, shifts, axis=tuple(range(a.ndim - self.d, a.ndim)))

    def density(self, f):
        return f.sum(axis=0)

    def force(self, psi, G):
        """Eq. (SCForce) with this lattice's W: F = -G c_s^2 psi(x) sum_a W_a psi(x+xi_a) xi_a."""
        s = np.zeros((self.d,) + psi.shape)
        for a in range(self.Q):
            if self.W[a] == 0.0:
                continue
            pn = self._shift(psi, self.c[a])
            for k in range(self.d):
                if self.c[a, k]:
                    s[k] += self.W[a] * pn * self.c[a, k]
        return -G * CS2 * psi * s

    def equilibrium(self, n, u):
        cu = np.tensordot(self.c.astype(float), u, axes=(1, 0))        # (Q, *space)
        uu = (u * u).sum(axis=0)
        wq = self.w.reshape((self.Q,) + (1,) * n.ndim)
        return wq * n * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2))

    def guo(self, tau, u, F):
        cf = np.tensordot(self.c.astype(float), F, axes=(1, 0))
        cu = np.tensordot(self.c.astype(float), u, axes=(1, 0))
        uf = (u * F).sum(axis=0)
        wq = self.w.reshape((self.Q,) + (1,) * u[0].ndim)
        # (xi^a/c_s^2 + (xi^a xi^b - c_s^2 delta^ab) u_b / c_s^4) F_a
        return (1.0 - 0.5 / tau) * wq * (cf / CS2 + (cu * cf - CS2 * uf) / (CS2 * CS2))

    def momentum(self, f):
        return np.tensordot(self.c.astype(float).T, f, axes=(1, 0))   # (d, *space)

    def velocity(self, f, G, kind):
        n = self.density(f)
        F = self.force(eos.psi(n, kind)[0], G)
        return (self.momentum(f) + 0.5 * F) / n

    def step(self, f, G, tau, kind):
        n = self.density(f)
        F = self.force(eos.psi(n, kind)[0], G)
        u = (self.momentum(f) + 0.5 * F) / n
        fs = f - (f - self.equilibrium(n, u)) / tau + self.guo(tau, u, F)
        out = np.empty_like(f)
        for i in range(self.Q):
            out[i] = self._shift(fs[i], -self.c[i])   # f_i(x + xi_i) = f*_i(x)
        return out

    def init_equilibrium(self, n, G, kind):
        """f = f_eq(n, -F/(2n)): zero physical velocity."""
        F = self.force(eos.psi(n, kind)[0], G)
        return self.equilibrium(n, -F / (2.0 * n))

    def pressure_tensor(self, f, G, kind):
        """Eq. (sm:pt) with this lattice's W: P^{mn} = n c_s^2 delta + (G c_s^2/2) psi sum_a W_a
        psi(x+xi_a) xi^m xi^n. Returns (d, d, *space)."""
        n = self.density(f)
        p = eos.psi(n, kind)[0]
        P = np.zeros((self.d, self.d) + n.shape)
        for a in range(self.Q):
            if self.W[a] == 0.0:
                continue
            pn = self._shift(p, self.c[a])
            for m in range(self.d):
                for k in range(self.d):
                    P[m, k] += self.W[a] * pn * self.c[a, m] * self.c[a, k]
        P *= 0.5 * G * CS2 * p
        for m in range(self.d):
            P[m, m] += n * CS2
        return P


D1Q3 = Lattice(c=[[0], [1], [-1]], w=[2 / 3, 1 / 6, 1 / 6], W=[0.0, 0.5, 0.5])

D2Q9 = Lattice(
    c=[[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [-1, -1], [1, -1], [-1, 1]],
    w=[4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
    W=[0.0] + [1 / 3] * 4 + [1 / 12] * 4,
)


def slab_profile(L, n_l, n_g, width, thickness=None):
    """Liquid slab centred at floor(L/2): n = (n_l+n_g)/2 - (n_l-n_g)/2 tanh((|d| - T/2)/width),
    d the minimum-image offset from the centre (the tanh profile of Sec. 4 with r = |d|)."""
    T = L / 2 if thickness is None else thickness
    c = L // 2
    d = np.arange(L) - c
    d = np.where(2 * d > L, d - L, d)
    d = np.where(2 * d < -L, d + L, d)
    return 0.5 * (n_l + n_g) - 0.5 * (n_l - n_g) * np.tanh((np.abs(d) - T / 2) / width)


def relax_flat(G, kind, L=64, n_l=None, n_g=None, width=1.0, tau=1.0, tol=1e-12,
               check_every=2000, max_steps=100000):
    """Relax a flat liquid slab on the D1Q3 lattice until the density field stops changing:
    max|n(t) - n(t - check_every)| < tol * n_l with check_every even (so the undamped staggered
    momentum mode, which flips sign every step, does not enter). Returns (f, steps).

    The slab is centred on a node with both interfaces on nodes. That symmetric state is a steady
    state but, at deep quench, a slowly unstable one: round-off seeds a drift of the interfaces
    towards an off-node position that grows by about e every 2e4 steps. The stopping rule halts
    at the symmetric steady state, long before the drift is visible."""
    if n_l is None:
        n_g, n_l, _ = eos.coexistence_rule(G, kind)
    n = slab_profile(L, n_l, n_g, width)
    f = D1Q3.init_equilibrium(n, G, kind)
    prev = D1Q3.density(f)
    steps = 0
    while steps < max_steps:
        for _ in range(check_every):
            f = D1Q3.step(f, G, tau, kind)
        steps += check_every
        cur = D1Q3.density(f)
        if np.max(np.abs(cur - prev)) < tol * n_l:
            break
        prev = cur
    return f, steps


def flat_observables(f1d, G, kind):
    """Embed a relaxed D1Q3 slab (normal along x) into a D2Q9 box with L_y = 4 (the paper's
    flat-interface geometry, Sec. 4) and measure it with the 2D lattice pressure tensor:
    P_N = P^xx, P_T = P^yy, p0 = mean P_N, sigma_0 = sum over the half box [L/2, L) of
    (P_N - P_T) (Sec. 4, flat-interface integral), n_l at the slab centre, n_g at x = 0."""
    L = f1d.shape[1]
    n = D1Q3.density(f1d)
    n2 = np.tile(n, (4, 1))
    # distribute each 1D population over the 2D velocities with the same x-projection,
    # proportionally to the 2D weights (keeps y-momentum zero)
    f2 = np.empty((9, 4, L))
    for i in range(9):
        cx = D2Q9.c[i, 0]
        j = {0: 0, 1: 1, -1: 2}[cx]
        group = [k for k in range(9) if D2Q9.c[k, 0] == cx]
        share = D2Q9.w[i] / sum(D2Q9.w[k] for k in group)
        f2[i] = share * np.tile(f1d[j], (4, 1))
    P = D2Q9.pressure_tensor(f2, G, kind)
    PN = P[0, 0, 0]
    PT = P[1, 1, 0]
    c = L // 2
    return dict(
        n=n, PN=PN, PT=PT, n_l=float(n[c]), n_g=float(n[0]), p0=float(PN.mean()),
        pn_spread=float(PN.max() - PN.min()),
        sigma0=float(np.sum(PN[L // 2:] - PT[L // 2:])),
        f2=f2, n2=n2,
    )


def lattice_coexistence(G, kind, L=64, **kw):
    """Flat-interface coexistence on the lattice (the reading of Sec. 4's "equilibrium values of
    n_g, n_l for a flat interface"): relax a D1Q3 slab from the leading-order rule densities and
    measure it. Returns the dict of flat_observables plus the number of steps taken."""
    f, steps = relax_flat(G, kind, L=L, **kw)
    out = flat_observables(f, G, kind)
    out["steps"] = steps
    out["f1d"] = f
    return out
