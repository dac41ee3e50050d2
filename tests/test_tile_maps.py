"""CPU check of the fused step kernels' index maps (csrc/step_kernels.hpp), for every compiled tile
kind over ragged box sizes: the work items and threads of a launch are enumerated with the
kernels' index arithmetic written out again here, and each access is checked before any GPU runs
it. A buffer access out of range would not fault (buffer loads read 0 out of range), so an index
slip at an untested size would show only as wrong results; this test looks for it directly:

- every population load and store stays inside its population plane (loads of two nodes inside
  the row's pitch), and every LDS index inside the ring;
- each node of the box is stored exactly once per plane, and nothing is stored beyond the row
  pitch;
- in full-row tiles, every interior store lands at an address congruent to its thread slot
  modulo the 128-byte line (the lane window is aligned with the line grid), for rows padded to
  whole lines and for packed rows (pitch nx) alike;
- for each stored node, the 18 neighbours it reads from the LDS ring hold psi of the right
  (periodically wrapped) nodes, written by some thread of the workgroup;
- the pull sources of every population of a stored node are its upwind neighbours (wrapped).

The z direction (chunks of z_chunk planes marched from z0 - 1 to z1, planes wrapped) is checked
for coverage separately: it has no lane-dependent arithmetic.
"""
import itertools

import numpy as np
import pytest

Q = 19
CX = [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0]
CY = [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1]
NEIGH = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]


def row_pitch(nx, elem, packed=False):
    if packed:
        return nx
    per_line = 128 // elem
    return (nx + per_line - 1) // per_line * per_line


def pop_pitch(pxy, elem):
    s = (pxy + 63) // 64 * 64
    b = s * elem
    if b >= 64 << 10:
        s += b // 19 // 256 * 256 // elem
    return s


def wrap(v, L):
    return v % L


class Plane:
    """Accesses of one workgroup to one z-plane: psi written into the LDS ring, loads, stores."""

    def __init__(self, nx, ny, elem, lds_shape, packed=False):
        self.nx, self.ny, self.elem = nx, ny, elem
        self.px = row_pitch(nx, elem, packed)
        self.pp = pop_pitch(self.px * ny, elem)
        self.lds = {}
        self.lds_shape = lds_shape
        self.stores = []

    def load(self, voff, nbytes):
        assert voff % 4 == 0 and 0 <= voff and voff + nbytes <= self.pp * self.elem, voff
        return voff

    def node_of(self, voff):
        e = voff // self.elem
        return e % self.px, e // self.px

    def write_lds(self, idx, node):
        assert all(0 <= i < n for i, n in zip(idx, self.lds_shape)), idx
        self.lds[idx] = node

    def check_pull(self, node, sources):
        """sources[i] = (x, y) element the lane loaded for population i of `node`."""
        x, y = node
        for i in range(Q):
            want = (wrap(x - CX[i], self.nx), wrap(y - CY[i], self.ny))
            assert sources[i] == want, (node, i, sources[i], want)


def check_neighbours(pl, x, y, lds_of):
    """The LDS neighbourhood of stored node (x, y): lds_of(dx, dy) is its ring index."""
    for dx, dy in NEIGH:
        idx = lds_of(dx, dy)
        assert idx in pl.lds, (x, y, dx, dy, idx)
        assert pl.lds[idx] == (wrap(x + dx, pl.nx), wrap(y + dy, pl.ny)), (x, y, dx, dy)


def xy_tile(nx, ny, elem, R, waves, bxt, tix, tiy, stored, packed=False):
    """step_tile: tile (tix, tiy) of a BXT-wide x-y tiling."""
    sub = 64 // bxt
    by = waves * R * sub
    LX, LY = bxt + 2, by + 2
    NH = 2 * LX + 2 * by
    assert NH <= 64 * waves
    pl = Plane(nx, ny, elem, (LY, LX), packed)
    px, E = pl.px, elem
    x0, y0 = tix * bxt, tiy * by
    todo = []
    for t in range(64 * waves):
        lane, wv = t & 63, t >> 6
        lc, ls = lane % bxt, lane // bxt
        xg = x0 + lc
        xload, xstore = xg <= nx, xg < px
        x = wrap(xg, nx)
        xo = [wrap(x - 1, nx) * E, x * E, wrap(x + 1, nx) * E]
        for r in range(R):
            yg = y0 + (wv * R + r) * sub + ls
            yin, ld = yg < ny, xload and yg <= ny
            y = wrap(yg, ny)
            yo = [wrap(y - 1, ny) * px * E, y * px * E, wrap(y + 1, ny) * px * E]
            ly, lx = (wv * R + r) * sub + ls + 1, lc + 1
            node = None
            if ld:
                src = [pl.node_of(pl.load(yo[1 - CY[i]] + xo[1 - CX[i]], E)) for i in range(Q)]
                node = src[0]
                pl.check_pull(node, src)
            pl.write_lds((ly, lx), node)
            if xstore and yin:
                off = yo[1] + xg * E
                pl.stores.append(pl.node_of(pl.load(off, E)))
                if xg < nx:
                    todo.append((xg, yg, ly, lx))
        if t < NH:
            if t < LX:
                hx, hy = t, 0
            elif t < 2 * LX:
                hx, hy = t - LX, by + 1
            elif t < 2 * LX + by:
                hx, hy = 0, 1 + (t - 2 * LX)
            else:
                hx, hy = bxt + 1, 1 + (t - 2 * LX - by)
            hxg, hyg = wrap(x0 - 1 + hx, nx), wrap(y0 - 1 + hy, ny)
            hxo = [wrap(hxg - 1, nx) * E, hxg * E, wrap(hxg + 1, nx) * E]
            hyo = [wrap(hyg - 1, ny) * px * E, hyg * px * E, wrap(hyg + 1, ny) * px * E]
            src = [pl.node_of(pl.load(hyo[1 - CY[i]] + hxo[1 - CX[i]], E)) for i in range(Q)]
            pl.check_pull(src[0], src)
            pl.write_lds((hy, hx), src[0])
    for xg, yg, ly, lx in todo:
        check_neighbours(pl, xg, yg, lambda dx, dy: (ly + dy, lx + dx))
    stored.extend(pl.stores)


def row_tile_rows(npt, waves, px):
    """Interior rows of a full-row tile (kernels.hpp row_tile_rows): 31 slots are kept free to
    align the lane window when the pitch is not a whole number of 32-element lines."""
    slack = 31 if px % 32 else 0
    return (npt * 64 * waves - slack) // px - 2


def row_tile(nx, ny, elem, npt, waves, tiy, stored, packed=False):
    """step_rows: full-row tiles of by rows, npt nodes per thread."""
    NT = 64 * waves
    px = row_pitch(nx, elem, packed)
    by = row_tile_rows(npt, waves, px)
    assert by >= 1
    M = px * (by + 2)
    cap = npt * NT
    pl = Plane(nx, ny, elem, (cap,), packed)
    E = elem
    line = 128 // elem
    y0 = tiy * by
    al = ((y0 - 1) * px) % line      # Python's % is already non-negative
    todo = []
    for t in range(NT):
        for k in range(npt):
            m = t + k * NT - al
            valid = 0 <= m < M
            lx, ly = (m % px, m // px) if valid else (0, 0)
            yg = y0 - 1 + ly
            lxk, xk, yk = min(lx, nx - 1), lx, wrap(yg, ny)
            ldk = valid and lx < nx and yg <= ny
            stk = valid and 1 <= ly <= by and yg < ny
            x, y = lxk, yk
            xo = [(nx - 1 if x == 0 else x - 1) * E, x * E, (0 if x == nx - 1 else x + 1) * E]
            yo = [(ny - 1 if y == 0 else y - 1) * px * E, y * px * E,
                  (0 if y == ny - 1 else y + 1) * px * E]
            if ldk:
                src = [pl.node_of(pl.load(yo[1 - CY[i]] + xo[1 - CX[i]], E)) for i in range(Q)]
                pl.check_pull(src[0], src)
                pl.write_lds((ly * nx + xk,), src[0])
            if stk:
                off = yo[1] + xk * E
                assert xk < px
                # aligned lane window: the slot and the stored element agree modulo the line
                assert (off // E - (t + k * NT)) % line == 0, (t, k)
                pl.stores.append(pl.node_of(pl.load(off, E)))
                if xk < nx:
                    todo.append((xk, yg, ly, lxk))
    for x, yg, ly, lx in todo:
        def lds_of(dx, dy, ly=ly, lx=lx):
            xx = (nx - 1 if lx == 0 else lx - 1) if dx < 0 else (
                (0 if lx == nx - 1 else lx + 1) if dx > 0 else lx)
            return ((ly + dy) * nx + xx,)
        check_neighbours(pl, x, yg, lds_of)
    stored.extend(pl.stores)


def check_coverage(stored, nx, ny, px):
    seen = {}
    for node in stored:
        seen[node] = seen.get(node, 0) + 1
    for x, y in itertools.product(range(px), range(ny)):
        if x < nx:
            assert seen.get((x, y), 0) == 1, (x, y, seen.get((x, y), 0))
        else:
            assert seen.get((x, y), 0) <= 1, (x, y)
    assert all(x < px and y < ny for x, y in seen)


SIZES = [(1, 1), (2, 3), (5, 70), (31, 9), (33, 4), (37, 29), (63, 5), (64, 17), (65, 3),
         (100, 37), (127, 2), (128, 9), (129, 5), (130, 7), (191, 3), (256, 20), (257, 2)]


XY_SHAPES = [(R, waves, bxt) for (R, waves, bxt) in itertools.product((1, 2, 4), (4, 8), (64, 32))
             if not (waves == 8 and R == 4) and not (bxt == 32 and R == 4)]


@pytest.mark.parametrize("nx,ny", [s for s in SIZES if s[0] <= 130])
@pytest.mark.parametrize("R,waves,bxt", XY_SHAPES)
@pytest.mark.parametrize("elem", [4, 8])
@pytest.mark.parametrize("packed", [False, True])
def test_xy_tile_index_map(nx, ny, R, waves, bxt, elem, packed):
    by = waves * R * (64 // bxt)
    stored = []
    for tix in range((nx + bxt - 1) // bxt):
        for tiy in range((ny + by - 1) // by):
            xy_tile(nx, ny, elem, R, waves, bxt, tix, tiy, stored, packed)
    check_coverage(stored, nx, ny, row_pitch(nx, elem, packed))


@pytest.mark.parametrize("nx,ny", [s for s in SIZES if s[0] <= 130] + [(160, 11), (300, 4),
                                                                         (101, 37), (77, 50)])
@pytest.mark.parametrize("npt,waves", [(2, 8), (4, 8), (8, 8), (4, 4)])
@pytest.mark.parametrize("elem", [4, 8])
@pytest.mark.parametrize("packed", [False, True])
def test_row_tile_index_map(nx, ny, npt, waves, elem, packed):
    px = row_pitch(nx, elem, packed)
    by = row_tile_rows(npt, waves, px)
    if by < 1:
        pytest.skip("rows too long for this shape (the library refuses it)")
    stored = []
    for tiy in range((ny + by - 1) // by):
        row_tile(nx, ny, elem, npt, waves, tiy, stored, packed)
    check_coverage(stored, nx, ny, px)


@pytest.mark.parametrize("nz,zc", [(1, 1), (1, 8), (7, 3), (8, 8), (9, 8), (64, 6), (256, 64),
                                   (130, 33)])
def test_z_chunks_cover_every_plane_once(nz, zc):
    zc = min(zc, nz)
    planes = []
    for ch in range((nz + zc - 1) // zc):
        z0, z1 = ch * zc, min(ch * zc + zc, nz)
        planes += list(range(z0, z1))
        # the march pulls planes z0 - 1 .. z1 (wrapped), each with its two z neighbours
        for p in range(z0 - 1, z1 + 1):
            assert 0 <= wrap(p - 1, nz) < nz and 0 <= wrap(p + 1, nz) < nz
    assert sorted(planes) == list(range(nz))
