"""Pins of the oracle's observables assembly (oracle/observe.py, observables()) against values
fixed independently of it: the bulk pressure of Eq. (bulkp) on uniform neighbourhoods, the
exact one- and two-dimensional reductions of the lattice pressure tensor Eq. (sm:pt) (the
independent D1Q3/D2Q9 codes of oracle/reduced.py), node counts of sharp spheres, translations of
a blob, and hand-made velocity fields.

Each test targets one choice of the assembly that the GPU observables are checked against: the
probe nodes (Sec. 4: P_in at the box centre, P_out at (L-1, L-1, L-1) for odd L), which diagonal
component is the tangential pressure along +x (Sec. 3: P^yy), the sigma[R] constant C on the nodes
r = 0..R_out, the plane averages and half-box sum of the flat sigma_0 (Sec. 4), the centre of mass
on a periodic box, R_e from the mass balance (Sec. 4), and the velocity-change measure (Sec. 4)
built from the physical velocity (Sec. 2).
"""
import numpy as np
import pytest

from oracle import core, eos, observe, reduced

KIND = core.PSI_EXP
G = eos.G_of(1.3, KIND)
XI, W_LAT, _ = core.tables()
CS2 = 1.0 / 3.0


def state_of_density(n):
    """Populations at rest (zero physical velocity) with density n; the pressure tensor of
    Eq. (sm:pt) depends on n alone."""
    return core.init_populations(np.ascontiguousarray(n), G, KIND)


def block(n, centre, value):
    """Set the 3 x 3 x 3 block of nodes around `centre` (periodic) to `value`: every D3Q19
    neighbour of the centre then holds that density."""
    nz, ny, nx = n.shape
    cx, cy, cz = centre
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                n[(cz + dz) % nz, (cy + dy) % ny, (cx + dx) % nx] = value


@pytest.mark.parametrize("L,far", [(21, 20), (20, 0), (9, 8)])
def test_probes_read_bulk_pressure_at_centre_and_far_node(L, far):
    """P_in and P_out are P^xx at the centre floor(L/2) and at the far node (L - 1 for odd L,
    (L/2 + L/2) mod L = 0 for even L); on a uniform neighbourhood P^xx is the bulk pressure of
    Eq. (bulkp) (e_2 = 1)."""
    n_a, n_c, n_b = 1.1, 2.4, 0.45
    n = np.full((L, L, L), n_a)
    c = L // 2
    block(n, (c, c, c), n_c)
    block(n, (far, far, far), n_b)
    o = observe.observables(state_of_density(n), G, KIND)
    assert abs(o["n_center"] - n_c) <= 1e-14 * n_c and abs(o["n_far"] - n_b) <= 1e-14 * n_b
    P_c, P_b = eos.pressure(n_c, G, KIND), eos.pressure(n_b, G, KIND)
    assert abs(o["P_in"] - P_c) <= 1e-14 * abs(P_c)
    assert abs(o["P_out"] - P_b) <= 1e-14 * abs(P_b)
    assert abs(o["dP"] - (P_c - P_b)) <= 1e-14 * abs(P_c)


def flat_pressures(n1d):
    """Normal and tangential pressure of a flat profile n1d (normal along the profile), from the
    independent D2Q9 code (the flat-interface reduction of the lattice pressure tensor)."""
    f1d = reduced.D1Q3.init_equilibrium(n1d, G, KIND)
    fl = reduced.flat_observables(f1d, G, KIND)
    return fl["PN"], fl["PT"]


def trapezoid_r2(R):
    """Trapezoid rule of r^2 on the nodes r = 0..R (unit spacing), summed by hand."""
    return R * (R + 1) * (2 * R + 1) / 6.0 - R * R / 2.0


@pytest.mark.parametrize("axis", [1, 2])
@pytest.mark.parametrize("L", [21, 16])
def test_tangential_pressure_is_pyy_along_x(axis, L):
    """A density that varies only along y (axis 1) or only along z (axis 2). On the line
    (x, c, c) every node is alike, so sigma[R]'s C = (P_out - P_T) times the trapezoid of r^2 on
    r = 0..R_out, with P_T = P^yy: the flat profile's normal pressure when the profile runs along
    y, its tangential pressure when it runs along z. P_in and P_out (P^xx) are tangential in both
    cases. Taking P^zz or P^xx for P_T, or another R_out, fails one of the two orientations."""
    c = L // 2
    far = (c + L // 2) % L
    coord = np.arange(L)
    n1d = 1.4 + 0.9 * np.tanh((np.abs(coord - c) - L / 4.0) / 1.5) * np.sign(np.cos(coord))
    n1d = n1d + 0.05 * coord / L
    PN, PT = flat_pressures(n1d)
    shape = [1, 1, 1]
    shape[2 - axis] = L
    n = np.broadcast_to(n1d.reshape(shape), (L, L, L)).copy()
    o = observe.observables(state_of_density(n), G, KIND)
    P_in, P_out = PT[c], PT[far]
    assert abs(o["P_in"] - P_in) <= 1e-14 and abs(o["P_out"] - P_out) <= 1e-14
    P_T = PN[c] if axis == 1 else PT[c]
    C = (P_out - P_T) * trapezoid_r2(L - 1 - c)
    assert abs(o["C"] - C) <= 1e-12 * max(abs(C), 1.0)
    if o["dP"] > 0 and o["C"] > 0:
        Rs, ss = observe.surface_of_tension(o["dP"], C)
        assert abs(o["R_s"] - Rs) <= 1e-12 * Rs and abs(o["sigma_s"] - ss) <= 1e-12 * ss
    else:
        assert np.isnan(o["R_s"]) and np.isnan(o["sigma_s"])
    # the line profile is the tangential (x) and y / z components along x
    assert np.abs(o["prof"][0] - n1d[c]).max() <= 1e-14 * n1d[c]
    assert np.abs(o["prof"][1] - PT[c]).max() <= 1e-14
    assert np.abs(o["prof"][2] - (PN[c] if axis == 1 else PT[c])).max() <= 1e-14
    assert np.abs(o["prof"][3] - (PT[c] if axis == 1 else PN[c])).max() <= 1e-14


@pytest.mark.parametrize("L,R", [(21, 5.0), (24, 7.3)])
def test_equimolar_radius_of_a_sharp_sphere(L, R):
    """A sharp sphere of n_in (nodes within R of the centre, minimum image) in n_out: the mass
    balance of Sec. 4 gives R_e^3 = 3 K / (4 pi) for K nodes inside, whatever n_in and n_out."""
    c = L // 2
    d = np.arange(L) - c
    r2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    inside = r2 <= R * R
    n_in, n_out = 2.3, 0.6
    n = np.where(inside, n_in, n_out)
    o = observe.observables(state_of_density(n), G, KIND)
    K = int(inside.sum())
    assert abs(o["R_e"] - (3.0 * K / (4.0 * np.pi)) ** (1.0 / 3.0)) <= 1e-12 * R
    assert abs(o["mass"] - (n_in * K + n_out * (L ** 3 - K))) <= 1e-12 * o["mass"]


@pytest.mark.parametrize("L", [21, 20])
@pytest.mark.parametrize("shift", [(0, 0, 0), (4, -3, 2), (-5, 6, -6)])
def test_centre_of_mass_follows_a_shifted_blob(L, shift):
    """A ball of excess density e on a uniform background, centred at c + s: the centre of mass is
    c + e K s / M (K nodes in the ball, M the total mass); the background adds nothing, also for
    even L, where the node half a box away counts 0 (it lies on both sides)."""
    c = L // 2
    n_bg, e, R = 0.5, 1.7, 3.2
    d = np.arange(L) - c
    n = np.full((L, L, L), n_bg)
    sx, sy, sz = shift
    dz, dy, dx = np.meshgrid(d - sz, d - sy, d - sx, indexing="ij")
    ball = dx ** 2 + dy ** 2 + dz ** 2 <= R * R
    n[ball] += e
    o = observe.observables(state_of_density(n), G, KIND)
    K = int(ball.sum())
    M = float(n.sum())
    for a, s in enumerate(shift):
        assert abs(o["com"][a] - (c + e * K * s / M)) <= 1e-12 * L


@pytest.mark.parametrize("L", [8, 7])
def test_centre_of_mass_of_a_uniform_box_is_its_centre(L):
    n = np.full((L, L, L), 1.3)
    o = observe.observables(state_of_density(n), G, KIND)
    assert np.abs(np.array(o["com"]) - L // 2).max() <= 1e-13


def test_centre_of_mass_half_a_box_away_counts_zero():
    """Even L: extra mass on the plane half a box from the centre (array index 0) moves the
    centre of mass along neither direction; one node nearer, at offset L/2 - 1, it does."""
    L, e = 10, 0.8
    c = L // 2
    for x, offset in ((0, 0), (L - 1, L // 2 - 1), (1, -(L // 2 - 1))):
        n = np.full((L, L, L), 1.0)
        n[c, c, x] += e
        o = observe.observables(state_of_density(n), G, KIND)
        M = float(n.sum())
        assert abs(o["com"][0] - (c + e * offset / M)) <= 1e-13, x
        assert abs(o["com"][1] - c) <= 1e-13 and abs(o["com"][2] - c) <= 1e-13


def equilibrium_state(n, u):
    """Populations w_i n (1 + 3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u) with density n and momentum n u at
    every node (inputs for the velocity measures)."""
    cu = np.einsum("ic,czyx->izyx", XI.astype(float), u)
    uu = (u * u).sum(axis=0)
    return W_LAT.reshape(19, 1, 1, 1) * n * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


def test_velocity_change_and_momentum_of_hand_made_velocities():
    """Uniform density (no force): the physical velocity is the given field. Changing the
    velocity of two nodes by d1 and d2 gives du_l1 = (|d1|_1 + |d2|_1) / N and du_max the largest
    component; the momentum sum is M u0."""
    nx, ny, nz = 6, 5, 4
    N = nx * ny * nz
    n = np.full((nz, ny, nx), 1.25)
    u0 = np.array([0.01, -0.02, 0.005])
    u = np.broadcast_to(u0.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy()
    a = observe.observables(equilibrium_state(n, u), G, KIND)
    assert abs(a["mass"] - 1.25 * N) <= 1e-13 * N
    for k in range(3):
        assert abs(a["mom"][k] - 1.25 * N * u0[k]) <= 1e-14 * N
    d1, d2 = np.array([3e-4, -1e-4, 2e-5]), np.array([-5e-5, 7e-4, 1e-4])
    u[:, 1, 2, 3] += d1
    u[:, 3, 0, 5] += d2
    b = observe.observables(equilibrium_state(n, u), G, KIND, u_prev=a["u"])
    want = (np.abs(d1).sum() + np.abs(d2).sum()) / N
    assert abs(b["du_l1"] - want) <= 1e-12 * want
    assert abs(b["du_max"] - 7e-4) <= 1e-12
    assert np.isnan(a["du_l1"]) and np.isnan(a["du_max"])


def test_velocity_change_uses_the_physical_velocity():
    """Populations at rest in a non-uniform density carry momentum -F/2 (Sec. 2: the physical
    velocity (sum xi f + F/2)/n is zero); their velocity change against a zero field is zero,
    while j/n alone is not."""
    n = core.init_density(9, 8, 7, core.DROPLET, 2.5, 1.0, 2.5, 0.4, 1e-3, 42)
    f = state_of_density(n)
    o = observe.observables(f, G, KIND, u_prev=np.zeros((3,) + n.shape))
    j, _ = core.velocity(f, G, KIND)
    assert np.abs(j / n).max() > 1e-3
    assert o["du_max"] <= 1e-15 and o["du_l1"] <= 1e-15


def embed_slab(f1d, axis, other=(4, 5)):
    """A D1Q3 state (rest, +, -) along `axis` embedded into D3Q19, uniform across: each 1D
    population is split over the 3D velocities with the same component along the axis, in
    proportion to their lattice weights."""
    L = f1d.shape[1]
    dims = [other[0], other[1]]
    dims.insert(axis, L)                      # (nx, ny, nz)
    shape = (dims[2], dims[1], dims[0])
    prof_shape = [1, 1, 1]
    prof_shape[2 - axis] = L
    f = np.empty((19,) + shape)
    idx = {0: 0, 1: 1, -1: 2}
    for i in range(19):
        k = idx[int(XI[i, axis])]
        members = [m for m in range(19) if int(XI[m, axis]) == int(XI[i, axis])]
        share = W_LAT[i] / sum(W_LAT[m] for m in members)
        f[i] = np.broadcast_to(share * f1d[k].reshape(prof_shape), shape)
    return f


@pytest.fixture(scope="module")
def relaxed_slab():
    f1d, _ = reduced.relax_flat(G, KIND, L=32, tol=1e-10)
    return f1d, reduced.flat_observables(f1d, G, KIND)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_slab_observables_equal_the_flat_reduction(relaxed_slab, axis):
    """A relaxed flat slab embedded with its normal along each axis: the plane-averaged profile
    is the flat profile (n, P_N on the normal component, P_T on both others), sigma_0 is the
    half-box sum of P_N - P_T and the P_N spread is that of the flat profile (independent D2Q9
    code of the paper's flat-interface geometry). Wrong plane axes, components or half box fail."""
    f1d, fl = relaxed_slab
    o = observe.observables(np.ascontiguousarray(embed_slab(f1d, axis)), G, KIND, geom=core.SLAB,
                            slab_axis=axis)
    prof = o["prof"]
    scale = np.abs(fl["PN"]).max()
    assert np.abs(prof[0] - fl["n"]).max() <= 1e-13 * fl["n_l"]
    for k in range(3):
        want = fl["PN"] if k == axis else fl["PT"]
        assert np.abs(prof[1 + k] - want).max() <= 1e-13 * scale, k
    assert abs(o["sigma0_flat"] - fl["sigma0"]) <= 1e-12 * fl["sigma0"]
    assert abs(o["pn_spread"] - fl["pn_spread"]) <= 1e-13 * scale
    assert fl["sigma0"] > 0.04      # a real interface: sigma_0 ~ 0.0498 at G/G_c = 1.3
    for k in ("C", "R_s", "sigma_s", "R_e"):
        assert np.isnan(o[k])
