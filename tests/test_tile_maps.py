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


# ------------------------------------------------------------------------------------------
# Two steps per pass (k_step2 / k_step2_group: step_tile2). A workgroup of 64 * WAVES threads owns
# a BX x BY tile of the second step. Slot k of thread t pulls node s = t + k * NT of the
# (BX + 6) x (BY + 6) region (LDS position (s // LX, s % LX) of psa, global node x0 - 3 + lx,
# y0 - 3 + ly wrapped); in a tile cut by the box edge (wv x hv nodes inside) the slots beyond the
# (wv + 6) x (hv + 6) corner pull the corner's last column or row again. Pulled slots inside 1 <= lx <= BX + 4, 1 <= ly <= BY + 4 collide
# the first step into fs[.][ly - 1][lx - 1]. Own slot j of thread t is tile node o = t + j * NT at
# (o % BX, o // BX); ring slot h is ring node r = t + h * NT of the 2 (BX + 2) + 2 BY nodes
# around the tile (rows -1 and BY, then columns -1 and BX). Own and ring nodes gather their
# second-step populations from fs[i][by + 2 - cy_i][bx + 2 - cx_i] and write psi(t + 1) into
# psb[by + 1][bx + 1]; own nodes collide the second step with psb at their 18 neighbours and
# are stored when inside the row pitch and the box height.
# ------------------------------------------------------------------------------------------

SHAPES2 = [(64, 8, 8), (32, 16, 8), (32, 16, 4), (64, 16, 16)]   # (BX, BY, WAVES)


def two_step_maps(BX, BY, WAVES, nx, ny, px, tix, tiy):
    NT = 64 * WAVES
    NO = BX * BY // NT
    LX, LY, AX, AY, GX, GY = BX + 6, BY + 6, BX + 4, BY + 4, BX + 2, BY + 2
    NL = LX * LY
    NSA = -(-NL // NT)
    NHR = 2 * GX + 2 * BY
    NSH = -(-NHR // NT)
    x0, y0 = tix * BX, tiy * BY
    wv, hv = min(BX, nx - x0), min(BY, ny - y0)
    loaded, collided = {}, set()
    for t in range(NT):
        for k in range(NSA):
            s = t + k * NT
            if s >= NL:
                continue
            lx, ly = s % LX, s // LX
            assert (lx, ly) not in loaded, "an LDS position is pulled twice"
            loaded[(lx, ly)] = ((x0 - 3 + min(lx, wv + 5)) % nx, (y0 - 3 + min(ly, hv + 5)) % ny)
            if 1 <= lx <= AX and 1 <= ly <= AY:
                collided.add((lx, ly))
    own, ring = [], []
    for t in range(NT):
        for j in range(NO):
            o = t + j * NT
            own.append((o % BX, o // BX))
        for h in range(NSH):
            r = t + h * NT
            if r >= NHR:
                continue
            if r < GX:
                ring.append((r - 1, -1))
            elif r < 2 * GX:
                ring.append((r - GX - 1, BY))
            elif r < 2 * GX + BY:
                ring.append((-1, r - 2 * GX))
            else:
                ring.append((BX, r - 2 * GX - BY))
    return dict(NT=NT, LX=LX, LY=LY, AX=AX, AY=AY, GX=GX, GY=GY, wv=wv, hv=hv, x0=x0, y0=y0,
                loaded=loaded, collided=collided, own=own, ring=ring)


@pytest.mark.parametrize("shape", SHAPES2)
def test_two_step_tile_maps_cover_what_valid_outputs_need(shape):
    BX, BY, WAVES = shape
    for nx, ny, packed in ((1, 1, False), (3, 5, False), (37, 29, False), (65, 9, True),
                           (100, 100, False), (100, 37, True), (130, 17, False), (49, 52, True),
                           (BX, BY, False), (2 * BX + 1, 3 * BY - 1, True)):
        px = row_pitch(nx, 4, packed)
        plane_bytes = px * ny * 4
        for tix in range(-(-nx // BX)):
            for tiy in range(-(-ny // BY)):
                m = two_step_maps(BX, BY, WAVES, nx, ny, px, tix, tiy)
                wv, hv, loaded, collided = m["wv"], m["hv"], m["loaded"], m["collided"]
                # every LDS position of the region is pulled once; beyond the (wv + 6) x (hv + 6)
                # corner from the corner's last column or row
                assert set(loaded) == {(lx, ly) for lx in range(m["LX"]) for ly in range(m["LY"])}
                for (lx, ly), (x, y) in loaded.items():
                    if lx >= wv + 6 or ly >= hv + 6:
                        assert x == (m["x0"] + min(lx, wv + 5) - 3) % nx
                        assert y == (m["y0"] + min(ly, hv + 5) - 3) % ny
                # each loads a node of the box (offsets of it and its x/y neighbours in the plane)
                for (x, y) in loaded.values():
                    assert 0 <= x < nx and 0 <= y < ny
                    for dx, dy in NEIGH:
                        xo, yo = (x + dx) % nx, (y + dy) % ny
                        assert 0 <= yo * px * 4 + xo * 4 < plane_bytes
                # own nodes tile the whole BX x BY tile once; ring nodes the ring around it once
                assert sorted(m["own"]) == sorted((bx, by) for bx in range(BX) for by in range(BY))
                ring_want = ([(bx, -1) for bx in range(-1, BX + 1)] + [(bx, BY) for bx in range(-1, BX + 1)]
                             + [(-1, by) for by in range(BY)] + [(BX, by) for by in range(BY)])
                assert sorted(m["ring"]) == sorted(ring_want)
                # LDS bounds of every gather and psb write, valid or not
                for bx, by in m["own"] + m["ring"]:
                    assert 0 <= by + 1 < m["GY"] and 0 <= bx + 1 < m["GX"]
                    for i in range(Q):
                        gy, gx = by + 2 - CY[i], bx + 2 - CX[i]
                        assert 0 <= gy < m["AY"] and 0 <= gx < m["AX"]
                for lx, ly in collided:
                    assert 0 <= ly - 1 < m["AY"] and 0 <= lx - 1 < m["AX"]
                # stores: own nodes inside the row pitch and the box height, in the plane
                for bx, by in m["own"]:
                    xg, yg = m["x0"] + bx, m["y0"] + by
                    if xg < px and yg < ny:
                        assert yg * px * 4 + xg * 4 < plane_bytes
                # dependencies of the outputs inside the box: psi(t + 1) at the outputs and their
                # 18 neighbours, gathered by own or ring nodes from first-step nodes that
                # collided, whose psi neighbours and own moments were pulled
                own_ring = set(m["own"]) | set(m["ring"])
                gather = {(bx + dx, by + dy) for bx in range(wv) for by in range(hv)
                          for dx, dy in NEIGH}
                assert gather <= own_ring
                first = {(nx_ + 3 - CX[i], ny_ + 3 - CY[i]) for nx_, ny_ in gather for i in range(Q)}
                assert first <= collided, (shape, nx, ny, tix, tiy)
                assert {(lx + ex, ly + ey) for lx, ly in first for ex, ey in NEIGH} <= set(loaded)
                # each first-step node sits at the wrapped global position the outputs expect
                for lx, ly in first:
                    assert loaded[(lx, ly)] == ((m["x0"] + lx - 3) % nx, (m["y0"] + ly - 3) % ny)
