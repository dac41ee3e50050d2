"""Pins of the FP64 oracle against what the paper and the mathematics fix, independent of the oracle
itself (arXiv:2105.08772). CPU only.

Each test names what it pins and why a plausible mistake would fail it.
"""
import math

import numpy as np
import pytest

from oracle import core, eos, observe, reduced
from tests import inputs

XI, W_LAT, W_SC = core.tables()
CS2 = 1.0 / 3.0


def weights_scale(n0=1.0):
    return W_LAT * n0


# --------------------------------------------------------------------------------------------
# Velocity set and weights (Sec. 2, Eq. SCForce; Eq. bulkp for e_2 = 1)
# --------------------------------------------------------------------------------------------

def test_velocity_set_is_d3q19():
    vecs = {tuple(v) for v in XI.tolist()}
    assert len(vecs) == 19
    sq = (XI ** 2).sum(axis=1)
    assert sorted(sq.tolist()) == [0] + [1] * 6 + [2] * 12
    assert np.all(np.abs(XI) <= 1)
    assert tuple(XI[0]) == (0, 0, 0)
    for i in range(1, 19, 2):  # every moving velocity is followed by its opposite
        assert np.array_equal(XI[i + 1], -XI[i])


def test_lattice_weight_moments():
    """sum w = 1, sum w xi = 0, sum w xi xi = c_s^2 delta, 4th moment isotropic: pins the
    weights a textbook D3Q19 must have (the paper cites them)."""
    d = np.eye(3)
    assert abs(W_LAT.sum() - 1.0) < 1e-15
    assert np.abs(W_LAT @ XI).max() < 1e-16
    M2 = np.einsum("i,ia,ib->ab", W_LAT, XI, XI)
    assert np.abs(M2 - CS2 * d).max() < 1e-15
    M4 = np.einsum("i,ia,ib,ic,id->abcd", W_LAT, XI, XI, XI, XI)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.abs(M4 - iso).max() < 1e-15


def test_force_weights_printed_values_and_isotropy():
    """W(1) = 1/6, W(2) = 1/12 as printed after Eq. (SCForce); their second moment gives e_2 = 1
    (Eq. bulkp) and the fourth moment is isotropic ("4-th order lattice force isotropy")."""
    sq = (XI ** 2).sum(axis=1)
    assert np.all(W_SC[sq == 1] == 1.0 / 6.0)
    assert np.all(W_SC[sq == 2] == 1.0 / 12.0)
    d = np.eye(3)
    e2 = np.einsum("i,ia,ib->ab", W_SC, XI, XI)
    assert np.abs(e2 - d).max() < 1e-15
    M4 = np.einsum("i,ia,ib,ic,id->abcd", W_SC, XI, XI, XI, XI)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 3.0
    assert np.abs(M4 - iso).max() < 1e-15


# --------------------------------------------------------------------------------------------
# Equation of state (Eq. bulkp, Sec. 4)
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("kind,printed,n_c,closed", [
    (core.PSI_EXP, -2.463, 1.0, -math.e ** 2),
    (core.PSI_ONEMINUS, -1.333, math.log(2.0), -4.0),
])
def test_critical_coupling(kind, printed, n_c, closed):
    """G_c c_s^2 printed in Sec. 4 (3 decimals); closed forms from dP/dn = d2P/dn2 = 0."""
    nc, Gc = eos.critical_point(kind)
    assert abs(Gc * CS2 - printed) < 5e-4
    assert abs(nc - n_c) < 1e-12
    assert abs(Gc - closed) < 1e-11
    # at the critical point both derivatives vanish
    d1, d2 = eos.dpressure(nc, Gc, kind)
    assert abs(d1) < 1e-13 and abs(d2) < 1e-12


def test_psi_values():
    assert core.psi(1.0, core.PSI_EXP) == pytest.approx(math.exp(-1.0), rel=1e-16)
    assert core.psi(2.0, core.PSI_EXP) == pytest.approx(math.exp(-0.5), rel=1e-16)
    assert core.psi(math.log(2.0), core.PSI_ONEMINUS) == pytest.approx(0.5, rel=1e-15)


def test_spinodals_are_extrema_and_rule_is_an_isobar():
    for kind, r in ((core.PSI_EXP, 1.3), (core.PSI_ONEMINUS, 1.2)):
        G = eos.G_of(r, kind)
        sg, sl = eos.spinodals(G, kind)
        assert abs(eos.dpressure(sg, G, kind)[0]) < 1e-13
        assert abs(eos.dpressure(sl, G, kind)[0]) < 1e-13
        assert eos.dpressure(sg, G, kind)[1] < 0 < eos.dpressure(sl, G, kind)[1]
        ng, nl, p0 = eos.coexistence_rule(G, kind)
        assert ng < sg < sl < nl
        assert abs(eos.pressure(ng, G, kind) - p0) < 1e-14
        assert abs(eos.pressure(nl, G, kind) - p0) < 1e-14
        assert abs(eos.rule_residual(p0, G, kind)) < 1e-12


# --------------------------------------------------------------------------------------------
# The step: reductions to independent lower-dimensional codes
# --------------------------------------------------------------------------------------------

def _embed_reduced(g, keep_axes):
    """Embed a reduced state (D2Q9 on (z,x) or D1Q3 on z) into D3Q19, uniform along the other
    axes and mirror-symmetric in them, splitting each reduced population over the 3D velocities
    with the same projection in proportion to their weights."""
    if keep_axes == (0, 2):   # D2Q9: reduced velocity (cx, cz)
        lat = reduced.D2Q9
        nz, nx = g.shape[1:]
        shape3 = (nz, 3, nx)
        proj = {i: (XI[i, 0], XI[i, 2]) for i in range(19)}
        expand = lambda a: np.broadcast_to(a[:, None, :], shape3)
    else:                     # D1Q3 along z
        lat = reduced.D1Q3
        nz = g.shape[1]
        shape3 = (nz, 3, 3)
        proj = {i: (XI[i, 2],) for i in range(19)}
        expand = lambda a: np.broadcast_to(a[:, None, None], shape3)
    red_index = {tuple(c): i for i, c in enumerate(lat.c.tolist())}
    groups = {}
    for i in range(19):
        groups.setdefault(red_index[proj[i]], []).append(i)
    f = np.empty((19,) + shape3)
    for key, members in groups.items():
        tot = sum(W_LAT[m] for m in members)
        for m in members:
            f[m] = (W_LAT[m] / tot) * expand(g[key])
    return f, groups


def _project(f, groups, keep_axes):
    out = {}
    for key, members in groups.items():
        s = f[members].sum(axis=0)
        out[key] = s[:, 0, :] if keep_axes == (0, 2) else s[:, 0, 0]
    return np.stack([out[k] for k in sorted(out)])


@pytest.mark.parametrize("kind,ratio,tau", [(core.PSI_EXP, 1.3, 1.0), (core.PSI_EXP, 1.6, 0.8),
                                             (core.PSI_ONEMINUS, 1.2, 1.3)])
def test_step_reduces_to_d2q9(kind, ratio, tau):
    """A y-uniform, y-mirror-symmetric D3Q19 state must evolve exactly as the independent D2Q9
    code with the paper's 2D forcing weights W(1)=1/3, W(2)=1/12 (Sec. 4). Catches errors in any
    velocity with an x or z component, the equilibrium, the Guo term, the force and streaming."""
    G = eos.G_of(ratio, kind)
    rng = np.random.default_rng(7)
    nz, nx = 6, 5
    g = reduced.D2Q9.w[:, None, None] * (1.0 + 0.3 * rng.uniform(-1, 1, (9, nz, nx)))
    f, groups = _embed_reduced(g, (0, 2))
    f3 = f
    g2 = g
    for _ in range(3):
        f3 = core.step(np.ascontiguousarray(f3), G, tau, kind)
        g2 = reduced.D2Q9.step(g2, G, tau, kind)
        assert np.abs(_project(f3, groups, (0, 2)) - g2).max() < 2e-15
    # the pressure tensor of the embedded state is the 2D one
    P3 = core.pressure_tensor(np.ascontiguousarray(f), G, kind)
    P2 = reduced.D2Q9.pressure_tensor(g, G, kind)
    assert np.abs(P3[0][:, 0, :] - P2[0, 0]).max() < 1e-15   # xx
    assert np.abs(P3[2][:, 0, :] - P2[1, 1]).max() < 1e-15   # zz
    assert np.abs(P3[4][:, 0, :] - P2[0, 1]).max() < 1e-15   # xz


def test_step_reduces_to_d1q3():
    """An xy-uniform state evolves as the independent D1Q3 code (weights 2/3, 1/6, 1/6, W = 1/2)."""
    kind, G, tau = core.PSI_EXP, eos.G_of(1.4, core.PSI_EXP), 0.9
    rng = np.random.default_rng(11)
    L = 10
    g = reduced.D1Q3.w[:, None] * (1.0 + 0.4 * rng.uniform(-1, 1, (3, L)))
    f, groups = _embed_reduced(g, (2,))
    for _ in range(4):
        f = core.step(np.ascontiguousarray(f), G, tau, kind)
        g = reduced.D1Q3.step(g, G, tau, kind)
        assert np.abs(_project(f, groups, (2,)) - g).max() < 2e-15


# --------------------------------------------------------------------------------------------
# The step: symmetries, conservation, exact invariants
# --------------------------------------------------------------------------------------------

def _rotate(f, R):
    """Apply the lattice rotation/reflection R (3x3 integer) to a population field on a cubic
    periodic box: out[j](R x) = f[i](x) with xi_j = R xi_i."""
    L = f.shape[1]
    perm = np.empty(19, dtype=int)
    for i in range(19):
        v = R @ XI[i]
        perm[i] = [j for j in range(19) if np.array_equal(XI[j], v)][0]
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    X = np.stack([x, y, z]).reshape(3, -1)
    Y = (R @ X) % L
    out = np.empty_like(f)
    for i in range(19):
        out[perm[i]][Y[2], Y[1], Y[0]] = f[i].reshape(-1)
    return out


ROTATIONS = {
    "rot_z": np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]),
    "rot_x": np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]]),
    "rot_y": np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]]),
    "mirror_x": np.diag([-1, 1, 1]),
    "swap_xy": np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]]),
}


@pytest.mark.parametrize("name", sorted(ROTATIONS))
def test_step_is_equivariant_under_lattice_symmetries(name):
    """step(R f) = R step(f) for the cube's rotations and reflections: a wrong weight, a wrong
    velocity entry or an axis-specific slip in the force or the equilibrium breaks it."""
    R = ROTATIONS[name]
    kind, G, tau = core.PSI_EXP, eos.G_of(1.3, core.PSI_EXP), 0.85
    f = inputs.random_populations((5, 5, 5), 3, weights_scale(1.2), amp=0.3)
    a = core.step(_rotate(f, R), G, tau, kind)
    b = _rotate(core.step(f, G, tau, kind), R)
    assert np.abs(a - b).max() < 2e-15
    Pa = core.pressure_tensor(_rotate(f, R), G, kind)
    Pf = core.pressure_tensor(f, G, kind)
    # rotate the tensor field: P'(Rx) = R P(x) R^T
    full = np.empty((3, 3) + Pf.shape[1:])
    for k, (m, n) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        full[m, n] = Pf[k]
        full[n, m] = Pf[k]
    L = f.shape[1]
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    X = np.stack([x, y, z]).reshape(3, -1)
    Y = (R @ X) % L
    rot = np.einsum("am,mnk,bn->abk", R, full.reshape(3, 3, -1), R)
    for k, (m, n) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        exp_field = np.empty((L, L, L))
        exp_field[Y[2], Y[1], Y[0]] = rot[m, n]
        assert np.abs(Pa[k] - exp_field).max() < 2e-15


def test_step_is_translation_equivariant_on_a_ragged_box():
    kind, G, tau = core.PSI_ONEMINUS, eos.G_of(1.2, core.PSI_ONEMINUS), 1.0
    f = inputs.random_populations((7, 4, 5), 5, weights_scale(1.0), amp=0.3)
    s = (1, 3, 2)  # roll along z, y, x
    a = core.step(np.ascontiguousarray(np.roll(f, s, axis=(1, 2, 3))), G, tau, kind)
    b = np.roll(core.step(f, G, tau, kind), s, axis=(1, 2, 3))
    assert np.abs(a - b).max() < 1e-15


def test_uniform_state_is_a_fixed_point_and_pressure_is_bulk():
    """f = w n0 is unchanged by a step, and the lattice pressure tensor of Eq. (sm:pt) reduces to
    the bulk pressure of Eq. (bulkp) on it (this is where e_2 = 1 enters)."""
    for kind, n0 in ((core.PSI_EXP, 1.7), (core.PSI_ONEMINUS, 0.9)):
        G = eos.G_of(1.3, kind)
        f = np.ascontiguousarray(np.broadcast_to(W_LAT.reshape(19, 1, 1, 1) * n0, (19, 4, 3, 5)))
        g = core.step(f, G, 0.7, kind)
        assert np.abs(g - f).max() < 1e-15
        P = core.pressure_tensor(f, G, kind)
        p = eos.pressure(n0, G, kind)
        for k in range(3):
            assert np.abs(P[k] - p).max() < 1e-15
        for k in range(3, 6):
            assert np.abs(P[k]).max() < 1e-16


def test_conservation_and_zero_total_force():
    """Mass and physical momentum are conserved by a step; the Shan-Chen force sums to zero on a
    periodic box (pair antisymmetry of Eq. SCForce)."""
    kind, G, tau = core.PSI_EXP, eos.G_of(1.5, core.PSI_EXP), 0.75
    f = inputs.random_populations((6, 5, 7), 9, weights_scale(1.5), amp=0.4)
    n, ps = core.density(f, kind)
    F = core.force(ps, G)
    for c in range(3):
        assert abs(F[c].sum()) <= 1e-14 * np.abs(F[c]).sum()
    j0, u0 = core.velocity(f, G, kind)
    g = core.step(f, G, tau, kind)
    n1, _ = core.density(g, kind)
    j1, u1 = core.velocity(g, G, kind)
    assert abs(n1.sum() - n.sum()) <= 1e-14 * n.sum()
    for c in range(3):
        assert abs((u1[c] * n1).sum() - (u0[c] * n).sum()) <= 1e-13 * np.abs(j0[c]).sum()


def test_guo_collision_moments():
    """Moments of one collision at a node (before streaming), from the definitions in Sec. 2:
    sum f* = n; sum xi f* = j + F; sum xi xi f* = Pi - (Pi - Pi_eq)/tau + (1 - 1/(2 tau)) (uF + Fu)
    with Pi_eq = n c_s^2 delta + n u u and u = (j + F/2)/n. Catches a missing 1/2 in the
    equilibrium's quadratic term, a wrong Guo prefactor or a wrong sign of the force."""
    kind, G, tau = core.PSI_EXP, eos.G_of(1.4, core.PSI_EXP), 0.8
    f = inputs.random_populations((4, 4, 4), 13, weights_scale(1.3), amp=0.3)
    n, ps = core.density(f, kind)
    F = core.force(ps, G)
    for (x, y, z) in ((0, 0, 0), (1, 2, 3), (3, 1, 2)):
        fs = core.collide_at(f, G, tau, kind, x, y, z)
        fl = f[:, z, y, x]
        nn = fl.sum()
        j = XI.T @ fl
        Fk = F[:, z, y, x]
        u = (j + 0.5 * Fk) / nn
        assert abs(fs.sum() - nn) < 1e-14
        assert np.abs(XI.T @ fs - (j + Fk)).max() < 1e-14
        Pi = np.einsum("i,ia,ib->ab", fl, XI, XI)
        Pi_eq = nn * CS2 * np.eye(3) + nn * np.outer(u, u)
        want = Pi - (Pi - Pi_eq) / tau + (1 - 0.5 / tau) * (np.outer(u, Fk) + np.outer(Fk, u))
        assert np.abs(np.einsum("i,ia,ib->ab", fs, XI, XI) - want).max() < 1e-14


def test_one_step_on_4cubed_without_force_at_tau_one():
    """Brute-force check of one whole step on a 4^3 grid with G = 0 and tau = 1: the collision
    relaxes fully, so population i arriving at x is the equilibrium of the source node x - xi_i.
    Un-streaming every population (rolling it back by -xi_i) must give at each node a set that
    (a) carries the source node's density and momentum, (b) has the second moment
    n c_s^2 delta + j j / n, (c) has the third moment sum xi_a^3 f = j_a (xi_a^3 = xi_a on the
    lattice), and (d) is the same for two nodes with equal (n, j) but different populations.
    A population streamed the wrong way, a missing 1/2 or a wrong velocity definition fails it."""
    f = inputs.random_populations((4, 4, 4), 77, weights_scale(1.2), amp=0.3)
    # two nodes with different populations but the same density and momentum
    a, b = (1, 2, 3), (3, 0, 1)
    delta = np.zeros(19)
    delta[0], delta[7], delta[8] = 0.01, -0.005, -0.005   # (1,1,0) and (-1,-1,0): same n, same j
    f[:, b[2], b[1], b[0]] = f[:, a[2], a[1], a[0]] + delta
    g = core.step(f, 0.0, 1.0, core.PSI_EXP)
    back = np.stack([np.roll(g[i], shift=(-XI[i, 2], -XI[i, 1], -XI[i, 0]), axis=(0, 1, 2))
                     for i in range(19)])
    n = f.sum(axis=0)
    j = np.einsum("ic,izyx->czyx", XI, f)
    assert np.abs(back.sum(axis=0) - n).max() < 1e-15
    assert np.abs(np.einsum("ic,izyx->czyx", XI, back) - j).max() < 1e-15
    Pi = np.einsum("ia,ib,izyx->abzyx", XI, XI, back)
    want = n * CS2 * np.eye(3)[:, :, None, None, None] + np.einsum("azyx,bzyx->abzyx", j, j) / n
    assert np.abs(Pi - want).max() < 1e-14
    for c in range(3):
        assert np.abs(np.einsum("i,izyx->zyx", XI[:, c] ** 3, back) - j[c]).max() < 1e-15
    assert np.abs(f[:, b[2], b[1], b[0]] - f[:, a[2], a[1], a[0]]).max() > 1e-3
    assert np.abs(back[:, b[2], b[1], b[0]] - back[:, a[2], a[1], a[0]]).max() < 1e-15


def test_init_is_equilibrium_at_zero_velocity():
    """Initial populations: sum f = n, sum xi f = -F/2 (zero physical velocity), second moment
    n c_s^2 delta + n u u with u = -F/(2n): pins the equilibrium's three moments."""
    kind, G = core.PSI_EXP, eos.G_of(1.3, core.PSI_EXP)
    n0 = core.init_density(9, 8, 7, core.DROPLET, 2.5, 1.0, 2.5, 0.4, 1e-3, 42)
    f = core.init_populations(n0, G, kind)
    n, ps = core.density(f, kind)
    F = core.force(ps, G)
    assert np.abs(n - n0).max() < 1e-14
    j = np.einsum("ic,izyx->czyx", XI, f)
    assert np.abs(j + 0.5 * F).max() < 1e-15
    u = -F / (2 * n0)
    Pi = np.einsum("ia,ib,izyx->abzyx", XI, XI, f)
    want = n0 * CS2 * np.eye(3)[:, :, None, None, None] + n0 * np.einsum("azyx,bzyx->abzyx", u, u)
    assert np.abs(Pi - want).max() < 1e-14
    _, uu = core.velocity(f, G, kind)
    assert np.abs(uu).max() < 1e-15


@pytest.mark.parametrize("dims", [(4, 6, 8), (8, 4, 4)])
def test_staggered_momentum_identity(dims):
    """For even L_a: J_a = sum_x (-1)^{x_a} j_a obeys J_a(t+1) = -(J_a(t) + sum_x (-1)^{x_a} F_a(t))
    exactly (every population with xi_a != 0 moves one node along a, and the Guo collision adds
    F to the momentum). A wrong streaming direction or a wrong force sign breaks it."""
    kind, G, tau = core.PSI_EXP, eos.G_of(1.3, core.PSI_EXP), 0.9
    f = inputs.random_populations(dims, 17, weights_scale(1.1), amp=0.3)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sign = [(-1.0) ** x, (-1.0) ** y, (-1.0) ** z]
    for _ in range(3):
        n, ps = core.density(f, kind)
        F = core.force(ps, G)
        j = np.einsum("ic,izyx->czyx", XI, f)
        g = core.step(f, G, tau, kind)
        j1 = np.einsum("ic,izyx->czyx", XI, g)
        for a in range(3):
            J0 = (sign[a] * j[a]).sum()
            SF = (sign[a] * F[a]).sum()
            J1 = (sign[a] * j1[a]).sum()
            assert abs(J1 + J0 + SF) < 1e-13 * (np.abs(j[a]).sum() + np.abs(F[a]).sum())
        f = g


def test_collide_at_matches_full_step():
    """The single-node evaluation used for sampled checks equals the whole-box step."""
    kind, G, tau = core.PSI_ONEMINUS, eos.G_of(1.25, core.PSI_ONEMINUS), 1.0
    f = inputs.random_populations((5, 6, 4), 19, weights_scale(1.0), amp=0.3)
    g = core.step(f, G, tau, kind)
    nz, ny, nx = f.shape[1:]
    for (x, y, z) in ((0, 0, 0), (4, 5, 3), (2, 3, 1)):
        fs = core.collide_at(f, G, tau, kind, x, y, z)
        for i in range(19):
            d = ((x + XI[i, 0]) % nx, (y + XI[i, 1]) % ny, (z + XI[i, 2]) % nz)
            assert g[i, d[2], d[1], d[0]] == fs[i]


@pytest.mark.slow
def test_mass_drift_config_droplet_32():
    """The 32^3 FP64 droplet (exp psi, G = 1.3 G_c, tau = 1, R = 8, tanh width 2, noise 1e-6,
    seed 1) keeps its total mass to 1e-12 relative over 2000 steps; momentum stays at its
    round-off level."""
    kind = core.PSI_EXP
    G = eos.G_of(1.3, kind)
    ng, nl, _ = eos.coexistence_rule(G, kind)
    n0 = core.init_density(32, 32, 32, core.DROPLET, 8.0, 2.0, nl, ng, 1e-6, 1)
    f = core.init_populations(n0, G, kind)
    M0 = n0.sum()
    f = core.run(f, G, 1.0, kind, 2000)
    n, _ = core.density(f, kind)
    assert abs(n.sum() - M0) / M0 < 1e-12
    _, u = core.velocity(f, G, kind)
    for c in range(3):
        assert abs((u[c] * n).sum()) < 1e-10


# --------------------------------------------------------------------------------------------
# Flat interface: the paper's machine-precision mechanical equilibrium and coexistence
# --------------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def flat13():
    G = eos.G_of(1.3, core.PSI_EXP)
    return G, reduced.lattice_coexistence(G, core.PSI_EXP, L=64)


def test_flat_interface_normal_pressure_is_constant(flat13):
    """Sec. 2 after Eq. (sm:pt): for a flat interface the normal component P_N is constant
    through the interface on the lattice, to machine precision."""
    G, out = flat13
    assert out["pn_spread"] / out["p0"] < 1e-12
    assert out["n_l"] > 2 and out["n_g"] < 0.5
    # the 3D oracle keeps the same state steady and reports the same constant P_zz
    f1 = out["f1d"]
    f3, _ = _embed_reduced(f1, (2,))
    f3 = np.ascontiguousarray(f3)
    g3 = core.step(f3, G, 1.0, core.PSI_EXP)
    assert np.abs(g3 - f3).max() < 1e-11
    P = core.pressure_tensor(f3, G, core.PSI_EXP)
    PN = P[2][:, 1, 1]
    assert (PN.max() - PN.min()) / out["p0"] < 1e-12
    assert abs(PN.mean() - out["p0"]) < 1e-13
    # sigma_0 from the 3D tensor (P_N = P^zz, P_T = P^xx) equals the 2D measurement
    L = len(PN)
    s3 = np.sum(PN[L // 2:] - P[0][L // 2:, 1, 1])
    assert abs(s3 - out["sigma0"]) < 1e-13


@pytest.mark.parametrize("kind,ratio,tol", [
    (core.PSI_EXP, 1.1, 2e-5), (core.PSI_EXP, 1.2, 5e-4), (core.PSI_EXP, 1.3, 2e-3),
    (core.PSI_ONEMINUS, 1.1, 2e-5), (core.PSI_ONEMINUS, 1.2, 5e-4)])
def test_flat_coexistence_vs_integral_rule(kind, ratio, tol):
    """The relaxed lattice slab's bulk densities against the leading-order integral rule
    int (p0 - P) psi'/psi dn = 0 (derived from the flat mechanical equilibrium). The two agree up
    to lattice corrections that grow with the quench; the tolerance covers the spread that the
    interface's position relative to the nodes causes (about 7e-4 at G/G_c = 1.3)."""
    G = eos.G_of(ratio, kind)
    ng, nl, p0 = eos.coexistence_rule(G, kind)
    out = reduced.lattice_coexistence(G, kind, L=64)
    assert abs(out["n_l"] / nl - 1) < tol
    assert abs(out["n_g"] / ng - 1) < 3 * tol
    assert abs(out["p0"] / p0 - 1) < 3 * tol


@pytest.mark.slow
def test_sigma0_mean_field_scaling_and_universality():
    """Sec. 4: sigma_0 scales as (G/G_c - 1)^{3/2} and both pseudopotentials share the prefactor."""
    s = {}
    for kind in (core.PSI_EXP, core.PSI_ONEMINUS):
        for r in (1.1, 1.2):
            s[kind, r] = reduced.lattice_coexistence(eos.G_of(r, kind), kind, L=64)["sigma0"]
    for kind in (core.PSI_EXP, core.PSI_ONEMINUS):
        slope = math.log(s[kind, 1.2] / s[kind, 1.1]) / math.log(0.2 / 0.1)
        assert abs(slope - 1.5) < 0.1
    pe = s[core.PSI_EXP, 1.1] / 0.1 ** 1.5
    po = s[core.PSI_ONEMINUS, 1.1] / 0.1 ** 1.5
    assert abs(pe / po - 1) < 0.05


# --------------------------------------------------------------------------------------------
# Surface of tension post-processing (Sec. 3)
# --------------------------------------------------------------------------------------------

def _sigma_direct(r, PT, P_in, P_out, R):
    """Eq. (gen_sigma) by brute-force quadrature on a fine grid, Heaviside included."""
    PJ = np.where(r < R, P_in, P_out)
    y = (r / R) ** 2 * (PJ - PT)
    return np.sum(0.5 * (y[1:] + y[:-1]) * np.diff(r))


def _dsigma_direct(r, PT, P_in, P_out, R):
    """Eq. (gen_d_sigma) by brute-force quadrature."""
    PJ = np.where(r < R, P_in, P_out)
    y = r * (r - R) * (PJ - PT)
    return -2.0 / R ** 3 * np.sum(0.5 * (y[1:] + y[:-1]) * np.diff(r))


def _equilibrium_profile(R0=10.0, width=1.0, P_in=0.3, P_out=0.1, rmax=40.0, h=2e-4):
    """A smooth normal-pressure profile and the tangential one that puts it in radial
    mechanical equilibrium in d = 3: dP_N/dr + (2/r)(P_N - P_T) = 0 (Eq. mech_eq_radial)."""
    r = np.arange(0.0, rmax + h / 2, h)
    PN = P_out + (P_in - P_out) * 0.5 * (1 - np.tanh((r - R0) / width))
    dPN = -(P_in - P_out) * 0.5 / width / np.cosh((r - R0) / width) ** 2
    PT = PN + 0.5 * r * dPN
    return r, PT


def test_closed_form_sigma_equals_definition_and_generalized_laplace():
    """For a profile in mechanical equilibrium: the split dP R/3 + C/R^2 equals Eq. (gen_sigma)
    evaluated by brute force; Eq. (gen_d_sigma) equals the derivative of sigma[R]; and the
    generalized Laplace law dP = 2 sigma[R]/R + d sigma/dR (Eq. LaplaceGen) holds for every R."""
    P_in, P_out = 0.3, 0.1
    r, PT = _equilibrium_profile(P_in=P_in, P_out=P_out)
    dP = P_in - P_out
    C = observe.sigma_C(r, PT, P_out)
    for R in (6.0, 9.0, 10.0, 12.5, 20.0):
        s_direct = _sigma_direct(r, PT, P_in, P_out, R)
        assert abs(observe.sigma_of_R(R, dP, C) - s_direct) < 2e-4 * abs(s_direct)
        ds = _dsigma_direct(r, PT, P_in, P_out, R)
        hR = 1e-3
        fd = (_sigma_direct(r, PT, P_in, P_out, R + hR)
              - _sigma_direct(r, PT, P_in, P_out, R - hR)) / (2 * hR)
        assert abs(ds - fd) < 2e-3 * max(abs(ds), 1e-3)
        assert abs(2 * s_direct / R + ds - dP) < 1e-3 * dP


def test_surface_of_tension_closed_form_numeric_and_universal_curve():
    P_in, P_out = 0.3, 0.1
    r, PT = _equilibrium_profile(P_in=P_in, P_out=P_out)
    dP = P_in - P_out
    C = observe.sigma_C(r, PT, P_out)
    Rs, ss = observe.surface_of_tension(dP, C)
    Rn, sn = observe.surface_of_tension_numeric(dP, C, 0.5 * Rs, 2.0 * Rs)
    assert abs(Rn - Rs) < 1e-8 * Rs
    assert abs(sn - ss) < 1e-12
    assert abs(ss - 0.5 * dP * Rs) < 1e-15
    # Laplace law at the minimum (Eq. f-statio-Rs); universal curve of Sec. 3
    for x in (0.5, 0.8, 1.0, 1.3, 2.0):
        R = x * Rs
        assert abs(observe.sigma_of_R(R, dP, C) / ss - (1 / 3 / x ** 2 + 2 * x / 3)) < 1e-12


def test_sharp_interface_surface_of_tension_is_its_radius():
    """P_T = P_J(r; R0) - sigma g(r - R0) with g a narrow normalised Gaussian of width s and
    dP = 2 sigma/R0: R_s^3 = R0^3 + 3 R0 s^2 exactly (R_s -> R0 as s -> 0)."""
    R0, sig, s = 12.0, 0.05, 0.02
    dP = 2 * sig / R0
    P_out = 0.1
    P_in = P_out + dP
    r = np.arange(0.0, 30.0, 1e-4)
    g = np.exp(-0.5 * ((r - R0) / s) ** 2) / (s * math.sqrt(2 * math.pi))
    PT = np.where(r < R0, P_in, P_out) - sig * g
    C = observe.sigma_C(r, PT, P_out)
    Rs, _ = observe.surface_of_tension(dP, C)
    # the trapezoid across the jump costs O(h) in C: 3h/R0 relative, a third of that in R_s
    assert abs(Rs - (R0 ** 3 + 3 * R0 * s * s) ** (1 / 3)) < 2e-5 * R0


def test_equimolar_radius_inverts_the_mass_balance():
    V, n_in, n_out, R = 41.0 ** 3, 2.5, 0.4, 10.25
    M = 4 * math.pi * R ** 3 * n_in / 3 + (V - 4 * math.pi * R ** 3 / 3) * n_out
    assert abs(observe.equimolar_radius(M, V, n_in, n_out) - R) < 1e-12
    # bubbles: n_in < n_out
    M = 4 * math.pi * R ** 3 * n_out / 3 + (V - 4 * math.pi * R ** 3 / 3) * n_in
    assert abs(observe.equimolar_radius(M, V, n_out, n_in) - R) < 1e-12


# --------------------------------------------------------------------------------------------
# Initial state and its noise
# --------------------------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    """SplitMix64 with state 0 yields 0xE220A8397B1DCDAF then 0x6E789E6AA1B965F4 (published
    test vector of the generator); the noise maps the top 53 bits to [-amp, amp)."""
    golden = 0x9E3779B97F4A7C15
    for state, out in ((0, 0xE220A8397B1DCDAF), (golden, 0x6E789E6AA1B965F4)):
        u = (out >> 11) * 2.0 ** -53
        assert core.noise(state, 0, 1.0) == 2.0 * u - 1.0
        assert core.noise(0, state, 1.0) == 2.0 * u - 1.0


def test_init_profile_geometry():
    """tanh profile of Sec. 4: liquid inside a droplet, gas inside a bubble, a slab of the given
    thickness; symmetric about the centre floor(L/2) without noise; noise bounded by its amp."""
    nl, ng = 2.5, 0.4
    n = core.init_density(33, 33, 33, core.DROPLET, 8.0, 1.0, nl, ng)
    c = 16
    assert abs(n[c, c, c] - nl) < 1e-6 and abs(n[0, 0, 0] - ng) < 1e-6
    # mirror about the centre node: index c + d <-> c - d
    idx = (2 * c - np.arange(33)) % 33
    assert np.abs(n - n[np.ix_(idx, idx, idx)]).max() < 1e-15
    # the interface (n = midpoint) sits at r = R
    mid = 0.5 * (nl + ng)
    assert abs(n[c, c, c + 8] - mid) < 1e-15
    nb = core.init_density(33, 33, 33, core.BUBBLE, 8.0, 1.0, ng, nl)
    assert abs(nb[c, c, c] - ng) < 1e-6 and abs(nb[0, 0, 0] - nl) < 1e-6
    ns = core.init_density(8, 8, 64, core.SLAB, 16.0, 2.0, nl, ng)  # half thickness 16
    assert abs(ns[32, 3, 5] - nl) < 1e-6 and abs(ns[0, 3, 5] - ng) < 1e-6
    assert abs(ns[16, 0, 0] - mid) < 1e-15 and abs(ns[48, 7, 7] - mid) < 1e-15
    nn = core.init_density(9, 10, 11, core.DROPLET, 3.0, 2.0, nl, ng, 1e-6, 1)
    n0 = core.init_density(9, 10, 11, core.DROPLET, 3.0, 2.0, nl, ng)
    d = nn - n0
    assert np.abs(d).max() <= 1e-6 and abs(d.mean()) < 2e-7 and d.std() > 4e-7


# --------------------------------------------------------------------------------------------
# Stencil radius (Sec. 2: streaming along the D3Q19 links, the force from the 18 nearest
# neighbours): one step reaches 2 nodes, two steps 4. The GPU's two-steps-per-pass launch is
# checked at full size against the oracle's two steps on 9^3 neighbourhoods, which rests on this.
# --------------------------------------------------------------------------------------------

def test_two_steps_reach_exactly_four_nodes():
    """The oracle's two whole-box steps at a node equal its two steps on the periodic 9^3
    neighbourhood of that node (to the bit), and not on the 7^3 one; a force or streaming
    stencil wider than nearest neighbours would break the first, a narrower one the second."""
    f = inputs.random_populations((14, 13, 12), 5, W_LAT * 1.5, amp=0.3)
    full = core.run(f.copy(), -6.0, 1.0, core.PSI_EXP, 2)
    for (x, y, z) in [(0, 0, 0), (13, 12, 11), (5, 6, 7), (2, 11, 3)]:
        for r, exact in ((4, True), (3, False)):
            ix, iy, iz = [(np.arange(-r, r + 1) + c) % n for c, n in ((x, 14), (y, 13), (z, 12))]
            sub = np.ascontiguousarray(f[:, iz][:, :, iy][:, :, :, ix])
            got = core.run(sub, -6.0, 1.0, core.PSI_EXP, 2)[:, r, r, r]
            diff = np.abs(got - full[:, z, y, x]).max()
            assert (diff == 0.0) if exact else (diff > 1e-8), (x, y, z, r, diff)
