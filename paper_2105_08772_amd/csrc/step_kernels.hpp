// Fused step kernels (single box and multi-box) of the Shan-Chen D3Q19 lattice Boltzmann library
// (gfx950), with their launch-shape dispatch. Included by one translation unit per precision
// (step_f32.hip, step_m64.hip, step_f64.hip), each instantiating its storage and arithmetic types,
// so the three compile in parallel; kernels.hip includes it for the shared device helpers only.
//
// Population storage: plane-major, population i of node (x, y, z) at element
// (z * 19 + i) * pp + y * px + x, with the row pitch px >= nx (a whole number of 128-byte lines,
// whose padding is never read, or nx itself for packed rows) and the population pitch
// pp >= px * ny. Each z-plane is one
// contiguous block of 19 population planes, so a box is not limited by 32-bit offsets.
// The stored arrays hold the post-collision populations of the previous step, f*_i(x, t - 1), so
// the pre-collision state of time t is the pull f_i(x, t) = f*_i(x - xi_i, t - 1) (Eq. lbm of
// arXiv:2105.08772 read as pull streaming). FP32 storage keeps g_i = f_i - w_i rho_ref.
//
// Fused step (one launch per time step, or two: see the two-steps-per-pass kernel below; Sec. 2
// of the paper):
//   pull the 19 populations -> density n and momentum j -> psi(n) -> Shan-Chen force F from the
//   psi of the 18 neighbours (Eq. SCForce) -> u_eq = (j + F/2)/n -> BGK relaxation to the
//   second-order equilibrium plus the Guo term -> store. psi at the neighbours is needed at the
//   same time level, so each workgroup owns an x-y tile (64 or 32 nodes wide, or whole rows),
//   marches up a chunk of z-planes, pulls the densities of its tile plus a one-node halo into an
//   LDS ring of four psi planes, and collides plane q once the psi of plane q + 1 is in LDS. Only
//   the halo and the two end planes of each chunk are pulled twice; the repeated reads are meant
//   to hit L2 because neighbouring tiles run together on the same XCD.
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "d3q19.hpp"

namespace lbm {
namespace {

__device__ __forceinline__ int wrapi(int v, int L)
{
    int r = v % L;
    return r < 0 ? r + L : r;
}

// Stored element index of population i of node (x, y, z).
__device__ __forceinline__ unsigned long long pop_index(const BoxDesc& b, int i, int x, int y, int z)
{
    return (unsigned long long)((unsigned)z * (unsigned)Q + (unsigned)i) * b.pp +
           (unsigned)y * b.px + (unsigned)x;
}

template <typename T, int PSI>
__device__ __forceinline__ T psi_of(T n)
{
    if constexpr (sizeof(T) == 4) {
        if constexpr (PSI == 0) return expf(-1.0f / n);
        else return 1.0f - expf(-n);
    } else {
        if constexpr (PSI == 0) return exp(-1.0 / n);
        else return 1.0 - exp(-n);
    }
}

__device__ __forceinline__ double psi_rt(double n, int kind)
{
    return kind == 0 ? exp(-1.0 / n) : 1.0 - exp(-n);
}

// Logical tile for a workgroup id so that each XCD (the hardware deals workgroups round-robin
// over 8 XCDs) receives one contiguous run of logical tiles: neighbours share its L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb)
{
    constexpr unsigned NX = 8;
    const unsigned xcd = b % NX, k = b / NX, per = nb / NX, rem = nb % NX;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// Populations are addressed plane by plane: the 19 population planes of one z-plane (19 pp
// elements, under 4 GiB, checked by the host) form one buffer resource whose base is the plane's
// first byte. A load or store of population i is one buffer instruction with the node's in-plane
// byte offset in a vector register and i * pp * sizeof(T) as the scalar offset; out-of-range
// offsets read 0 and write nothing instead of faulting. Rebasing a resource per plane is scalar
// work, so the box size is limited by memory, not by 32-bit offsets.
constexpr unsigned RSRC_FLAGS = 0x00020000u;  // raw buffer, 32-bit dword format (gfx9 family)
// Population stores carry the non-temporal cache policy: a stored population is read again
// only in the next step, after the whole box has streamed through the caches.
constexpr int STORE_CPOL_NT = 2;
// Population loads skip the per-CU vector L1 (sc0): the data a tile reads twice (its halo) is
// reused across workgroups in L2, not within one CU (measured: about 1.5 % faster than default).
constexpr int LOAD_CPOL_SC0 = 1;

typedef __amdgpu_buffer_rsrc_t Rsrc;

struct PopBuf {
    char* base;
    unsigned pop_bytes;  // pp * sizeof(T): bytes between the population planes of one z-plane
};

template <typename T>
__device__ __forceinline__ PopBuf make_popbuf(const T* p, unsigned pp)
{
    return PopBuf{reinterpret_cast<char*>(const_cast<T*>(p)), pp * (unsigned)sizeof(T)};
}

// Resource of z-plane z (0 <= z < nz).
__device__ __forceinline__ Rsrc plane_rsrc(const PopBuf& b, int z)
{
    const unsigned plane_bytes = (unsigned)Q * b.pop_bytes;
    return __builtin_amdgcn_make_buffer_rsrc(b.base + (unsigned long long)(unsigned)z * plane_bytes,
                                             (short)0, (int)plane_bytes, (int)RSRC_FLAGS);
}

// Resources of the planes p - 1, p, p + 1 (periodic in z), indexed by dz + 1.
struct Planes {
    Rsrc m, c, p;
};

template <int D>
__device__ __forceinline__ Rsrc plane_at(const Planes& z)
{
    if constexpr (D == 0) return z.m;
    else if constexpr (D == 1) return z.c;
    else return z.p;
}

template <typename T, int I>
__device__ __forceinline__ T bload(Rsrc r, unsigned pop_bytes, unsigned voff)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff,
                                                                              (int)(I * pop_bytes), LOAD_CPOL_SC0));
    } else {
        typedef int v2i __attribute__((ext_vector_type(2)));
        const v2i v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)(I * pop_bytes), LOAD_CPOL_SC0);
        return __builtin_bit_cast(double, v);
    }
}

template <typename T, int I>
__device__ __forceinline__ void bstore(Rsrc r, unsigned pop_bytes, unsigned voff, T v)
{
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)voff,
                                              (int)(I * pop_bytes), STORE_CPOL_NT);
    } else {
        typedef int v2i __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, (int)voff,
                                              (int)(I * pop_bytes), STORE_CPOL_NT);
    }
}

// Compile-time loop over population indices.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

struct StepArgs {
    BoxDesc b;
    int s;      // source buffer (0 or 1): selects the step count b.tick[s] behind the dither
    int tiles_x, tiles_y, nchunks, zc, remap;
    int by;     // full-row tiles: interior rows per tile
};

// Load the 19 pre-collision populations of one node. The plane resources zr and the in-plane byte
// offsets yo/xo[d] address the plane/row/column at coordinate + d - 1; the source of velocity xi
// is the node - xi.
template <typename T>
__device__ __forceinline__ void load_node(const Planes& zr, unsigned pop_bytes,
                                          const unsigned (&yo)[3], const unsigned (&xo)[3],
                                          T (&f)[Q])
{
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        f[i] = bload<T, i>(plane_at<1 - CZ[i]>(zr), pop_bytes, yo[1 - CY[i]] + xo[1 - CX[i]]);
    });
}

// Reduce the populations of a node to (sum g, j), j in the arithmetic type C. The density deviation
// is accumulated in double precision: for FP32 storage the sum of the 19 stored values is then
// exact, so the density a node sees is exactly the mass it holds.
template <typename T, typename C>
__device__ __forceinline__ void moments(const T (&f)[Q], double& dn, C& jx, C& jy, C& jz)
{
    double s = (double)f[0];
    C ax = C(0), ay = C(0), az = C(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        s += (double)f[i] + (double)f[i + 1];
        const C d = (C)f[i] - (C)f[i + 1];
        if (CX[i] > 0) ax += d;
        if (CX[i] < 0) ax -= d;
        if (CY[i] > 0) ay += d;
        if (CY[i] < 0) ay -= d;
        if (CZ[i] > 0) az += d;
        if (CZ[i] < 0) az -= d;
    }
    dn = s;
    jx = ax;
    jy = ay;
    jz = az;
}

// Rounding of the rest population, which carries the node's mass closure. In double precision
// it is stored as computed. In single precision round-to-nearest is biased wherever many nodes
// hold the same value - the bulk of each phase - and the bias adds up coherently once the state
// is quasi-static (measured: mass drift growing by about 3e-10 per step at 256^3). The value is
// therefore rounded after adding a dither in [-1/2, 1/2) ulp, u = frac((k + s) phi) - 1/2, k the
// node's index (z ny + y) nx + x in the box (not its storage offset, so that the result does not
// depend on the row pitch) and phi the golden-ratio fraction (a Weyl sequence over the nodes): over
// the nodes of one step the dither is spread evenly, so the stored value is unbiased over a
// region. The offset s is a hash of the box's step count, so the pattern moves to an unrelated
// position every step: the rounding errors of a quasi-static state neither repeat (which makes
// the mass drift linearly) nor follow the previous step's pattern (a regular shift, e.g. a second
// Weyl sequence in time, correlates the dither with the state it produced and biases the
// rounding; measured 10x more drift than a fixed pattern). The caller passes key = k + s. The
// result is deterministic and depends neither on the launch shape, the row layout nor on
// grouping.
template <typename T>
__device__ __forceinline__ T round_rest(double v, unsigned key)
{
    if constexpr (sizeof(T) == 8) {
        return v;
    } else {
        const float fv = (float)v;
        const float ulp = __uint_as_float(__float_as_uint(fv) & 0x7F800000u) * 0x1p-23f;
        const float u = (float)(key * 0x9E3779B9u) * 0x1p-32f - 0.5f;
        return (float)(v + (double)(u * ulp));
    }
}

// Dither offset of step count t: the 32-bit finaliser of MurmurHash3 (A. Appleby), a bijection
// whose outputs for consecutive inputs look independent.
__device__ __forceinline__ unsigned dither_shift(unsigned t)
{
    t ^= t >> 16;
    t *= 0x85EBCA6Bu;
    t ^= t >> 13;
    t *= 0xC2B2AE35u;
    t ^= t >> 16;
    return t;
}

// Collide one node in the arithmetic type C and hand its 19 post-collision (shifted) populations,
// rounded to the storage type T, to sink(integral_constant<i>, value) in the order they are
// computed (pairs i, i + 1, then the rest population); key, the node's index (z ny + y) nx + x
// plus the dither offset of the box's step, sets the rest population's dither.
// dn64 = sum g (n - rho_ref, exact), j = sum xi g = sum xi f. Rest population: mass-exact
// closure g*_0 = dn - sum_{i>0} g*_i (the stored values summed in double precision), equal to
// the BGK value in exact arithmetic; the node's stored mass then changes only by the final
// rounding of g*_0. Every kernel collides through this routine, so that a node gets the same
// bits whichever kernel steps it.
template <typename T, typename C, bool TAU1, typename Sink>
__device__ __forceinline__ void collide_emit(Sink&& sink, unsigned key, C rho_ref, double dn64,
                                             C jx, C jy, C jz, C Fx, C Fy, C Fz, C inv_tau,
                                             C guo_pref, const T* fin)
{
    const C dn = (C)dn64;
    const C n = rho_ref + dn;
    const C inv_n = C(1) / n;
    const C ux = (jx + C(0.5) * Fx) * inv_n;
    const C uy = (jy + C(0.5) * Fy) * inv_n;
    const C uz = (jz + C(0.5) * Fz) * inv_n;
    const C uu = ux * ux + uy * uy + uz * uz;
    const C uF = ux * Fx + uy * Fy + uz * Fz;
    double sum = 0.0;
    static_for<0, (Q - 1) / 2>([&](auto K) {
        constexpr int i = 1 + 2 * decltype(K)::value;
        const C w = (C)weight(i);
        const C c = C(CX[i]) * ux + C(CY[i]) * uy + C(CZ[i]) * uz;
        const C cf = C(CX[i]) * Fx + C(CY[i]) * Fy + C(CZ[i]) * Fz;
        C gp, gm;
        if constexpr (TAU1) {
            // tau = 1: f* = f_eq + (1/2) Guo bracket
            const C even = w * (dn + n * (C(4.5) * c * c - C(1.5) * uu) + C(4.5) * c * cf - C(1.5) * uF);
            const C odd = w * (C(3) * n * c + C(1.5) * cf);
            gp = even + odd;
            gm = even - odd;
        } else {
            const C eq_e = w * (dn + n * (C(4.5) * c * c - C(1.5) * uu));
            const C eq_o = w * (C(3) * n * c);
            const C gu_e = guo_pref * w * (C(9) * c * cf - C(3) * uF);
            const C gu_o = guo_pref * w * (C(3) * cf);
            const C fp = (C)fin[i], fm = (C)fin[i + 1];
            gp = fp + (eq_e + eq_o - fp) * inv_tau + gu_e + gu_o;
            gm = fm + (eq_e - eq_o - fm) * inv_tau + gu_e - gu_o;
        }
        // the closure sums the values as stored (rounded to T)
        const T sp = (T)gp, sm = (T)gm;
        sink(std::integral_constant<int, i>{}, sp);
        sink(std::integral_constant<int, i + 1>{}, sm);
        sum += (double)sp + (double)sm;
    });
    sink(std::integral_constant<int, 0>{}, round_rest<T>(dn64 - sum, key));
}

// collide_emit storing the populations at in-plane byte offset off of plane resource dst, each
// as soon as it is computed.
template <typename T, typename C, bool TAU1>
__device__ __forceinline__ void collide_store(Rsrc dst, unsigned pop_bytes, unsigned off,
                                              unsigned key, C rho_ref,
                                              double dn64, C jx, C jy, C jz, C Fx, C Fy, C Fz,
                                              C inv_tau, C guo_pref, const T* fin)
{
    collide_emit<T, C, TAU1>([&](auto I, T v) { bstore<T, decltype(I)::value>(dst, pop_bytes, off, v); },
                             key, rho_ref, dn64, jx, jy, jz, Fx, Fy, Fz, inv_tau, guo_pref, fin);
}

// Shan-Chen force of Eq. (SCForce): F = -G c_s^2 psi(x) sum_a W_a psi(x + xi_a) xi_a
// = -G psi(x) S with S = sum_a w_a psi(x + xi_a) xi_a, since c_s^2 W_a equals the lattice weight
// w_a (1/18 for the six axis neighbours, 1/36 for the twelve diagonal ones). at(dx, dy, dz) returns psi of the
// neighbour at that offset (dz = -1, 0, 1 for the planes below, at and above the node). Every
// kernel evaluates the force through this routine (same expression, same rounding).
template <typename C, typename At>
__device__ __forceinline__ void sc_force(At&& at, C G, C& Fx, C& Fy, C& Fz)
{
    const C c_e = at(1, 0, 0), c_w = at(-1, 0, 0);
    const C c_n = at(0, 1, 0), c_s = at(0, -1, 0);
    const C c_ne = at(1, 1, 0), c_nw = at(-1, 1, 0);
    const C c_se = at(1, -1, 0), c_sw = at(-1, -1, 0);
    const C p_c = at(0, 0, 1), p_e = at(1, 0, 1), p_w = at(-1, 0, 1);
    const C p_n = at(0, 1, 1), p_s = at(0, -1, 1);
    const C m_c = at(0, 0, -1), m_e = at(1, 0, -1), m_w = at(-1, 0, -1);
    const C m_n = at(0, 1, -1), m_s = at(0, -1, -1);
    const C psi0 = at(0, 0, 0);
    const C w1 = (C)W1, w2 = (C)W2;
    const C Sx = w1 * (c_e - c_w) +
                 w2 * ((c_ne - c_nw) + (c_se - c_sw) + (p_e - p_w) + (m_e - m_w));
    const C Sy = w1 * (c_n - c_s) +
                 w2 * ((c_ne - c_se) + (c_nw - c_sw) + (p_n - p_s) + (m_n - m_s));
    const C Sz = w1 * (p_c - m_c) +
                 w2 * ((p_e - m_e) + (p_w - m_w) + (p_n - m_n) + (p_s - m_s));
    const C gp = -G * psi0;
    Fx = gp * Sx;
    Fy = gp * Sy;
    Fz = gp * Sz;
}

// Tile of a workgroup of WAVES wave64s: BXT (64 or 32) nodes wide; each wave covers R rows of
// 64 / BXT sub-rows, so the tile is WAVES * R * 64 / BXT rows high.
template <int R, int WAVES, int BXT>
constexpr int tile_rows()
{
    static_assert(BXT == 64 || BXT == 32, "tile width is 64 or 32");
    return WAVES * R * (64 / BXT);
}

// LDS ring of four psi planes of a (BXT + 2) x (BY + 2) tile, shared by the single-box and the
// multi-box kernels.
template <typename T, int BXT, int BY>
struct Ring {
    static constexpr int LX = BXT + 2, LY = BY + 2;
    T v[4][LY][LX];
};
// LDS ring of full-row tiles: four planes of up to CAP psi values (rows of nx, flattened).
template <typename T, int CAP>
struct RowRing {
    T v[4][CAP];
};

// Ring of a launch shape: BXT = 64 or 32 for x-y tiles; BXT = 0 for full-row tiles, where R is
// the number of nodes each thread holds per plane.
template <typename T, int R, int WAVES, int BXT>
struct RingSel {
    using type = Ring<T, BXT, tile_rows<R, WAVES, BXT>()>;
};
template <typename T, int R, int WAVES>
struct RingSel<T, R, WAVES, 0> {
    using type = RowRing<T, R * 64 * WAVES>;
};
template <typename T, int R, int WAVES, int BXT>
using RingOf = typename RingSel<T, R, WAVES, BXT>::type;

// One workgroup's share of a step: the tile (tix, tiy) of box b, planes [z0, z1), populations
// stored as T, arithmetic in C (C = T, or T = float with C = double). The caller provides the LDS
// ring; the routine ends with every thread past its last read of the ring.
template <typename T, typename C, int PSI, bool TAU1, int R, bool PF, int WAVES, int BXT>
__device__ __forceinline__ void step_tile(const BoxDesc& bd, const T* __restrict__ src,
                                          T* __restrict__ dst, int tix, int tiy, int z0, int z1,
                                          const unsigned* tick_in, unsigned* tick_out,
                                          RingOf<C, R, WAVES, BXT>& rg)
{
    constexpr int NT = 64 * WAVES;
    constexpr int SUB = 64 / BXT;
    constexpr int BY = tile_rows<R, WAVES, BXT>();
    constexpr int LX = BXT + 2;
    constexpr int NH = 2 * LX + 2 * BY;
    static_assert(NH <= NT, "halo ring larger than the workgroup");
    auto& ring = rg.v;

    const int nx = bd.nx, ny = bd.ny, nz = bd.nz;
    const PopBuf sbuf = make_popbuf(src, bd.pp);
    const PopBuf dbuf = make_popbuf(dst, bd.pp);
    const unsigned popb = sbuf.pop_bytes;
    const C rho_ref = (C)bd.rho_ref;
    const C G = (C)bd.G;
    const C inv_tau = (C)(1.0 / bd.tau);
    const C guo_pref = (C)(1.0 - 0.5 / bd.tau);
    const int x0 = tix * BXT, y0 = tiy * BY;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // lane -> (column lc, sub-row ls) of the wave's rows; row r of the wave is tile row
    // (wv * R + r) * SUB + ls
    const int lc = lane % BXT, ls = lane / BXT;

    // The thread's own column. In the last tile of a row, the lane at x = nx pulls node 0 (the
    // east neighbour of node nx - 1, wrapped) and only feeds psi to the LDS ring; lanes beyond it
    // load nothing. Lanes in the row's padding (nx <= x < px) store values nobody reads, so that
    // the row's last 128-byte line is written whole.
    constexpr unsigned E = sizeof(T);
    const unsigned rowb = bd.px * E;
    const int xg = x0 + lc;
    const bool xload = xg <= nx;
    const bool xstore = xg < (int)bd.px;
    const int x = wrapi(xg, nx);
    const unsigned xo[3] = {(unsigned)wrapi(x - 1, nx) * E, (unsigned)x * E,
                            (unsigned)wrapi(x + 1, nx) * E};
    const unsigned xso = (unsigned)xg * E;
    unsigned yo[R][3];
    bool yin[R], ld[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int yg = y0 + (wv * R + r) * SUB + ls;
        yin[r] = yg < ny;
        ld[r] = xload && yg <= ny;   // the row at y = ny is row 0, the north neighbour of ny - 1
        const int y = wrapi(yg, ny);
        yo[r][0] = (unsigned)wrapi(y - 1, ny) * rowb;
        yo[r][1] = (unsigned)y * rowb;
        yo[r][2] = (unsigned)wrapi(y + 1, ny) * rowb;
    }

    // Halo node of this thread (ring position hx, hy in LDS coordinates), if any.
    const int t = threadIdx.x;
    const bool has_halo = t < NH;
    int hx = 0, hy = 0;
    if (t < LX) {
        hx = t;
        hy = 0;
    } else if (t < 2 * LX) {
        hx = t - LX;
        hy = BY + 1;
    } else if (t < 2 * LX + BY) {
        hx = 0;
        hy = 1 + (t - 2 * LX);
    } else {
        hx = BXT + 1;
        hy = 1 + (t - 2 * LX - BY);
    }
    const int hxg = wrapi(x0 - 1 + hx, nx), hyg = wrapi(y0 - 1 + hy, ny);
    const unsigned hxo[3] = {(unsigned)wrapi(hxg - 1, nx) * E, (unsigned)hxg * E,
                             (unsigned)wrapi(hxg + 1, nx) * E};
    const unsigned hyo[3] = {(unsigned)wrapi(hyg - 1, ny) * rowb, (unsigned)hyg * rowb,
                             (unsigned)wrapi(hyg + 1, ny) * rowb};

    auto planes = [&](int p) {
        return Planes{plane_rsrc(sbuf, wrapi(p - 1, nz)), plane_rsrc(sbuf, wrapi(p, nz)),
                      plane_rsrc(sbuf, wrapi(p + 1, nz))};
    };

    // Raw populations of the plane being reduced. With PF the loads of plane k + 1 are issued
    // right after plane k has been reduced, so they are in flight during the barrier and the
    // collision of plane k - 1.
    T fr[R][Q];
    T fh[Q];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < Q; ++i) fr[r][i] = T(0);
    double pdn[R];
    C pjx[R], pjy[R], pjz[R];
    const int nplanes = (z1 - z0) + 2;
    // The step count behind the dither is read with a vector load (a relaxed atomic, so that it
    // is not turned into a scalar load, whose wait would also hold up the LDS traffic). It is
    // issued in every plane, behind that plane's population loads, so that it delays none of
    // them and the load counter waits stay exact (a load in the first plane only would leave
    // every later wait one load stricter); the first plane's value is used at the start of the
    // second, when it has long arrived.
    unsigned tkv = 0u, tk = 0u, seed = 0u;
    if constexpr (PF) {
        const Planes zr = planes(z0 - 1);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (ld[r]) load_node(zr, popb, yo[r], xo, fr[r]);
        if (has_halo) load_node(zr, popb, hyo, hxo, fh);
        tkv = __hip_atomic_load(tick_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    for (int k = 0; k < nplanes; ++k) {
        const int p = z0 - 1 + k;
        if (k == 1) {
            tk = __builtin_amdgcn_readfirstlane(tkv);
            seed = dither_shift(tk);
        }
        C(*slot)[LX] = ring[k & 3];
        double cdn[R];
        C cjx[R], cjy[R], cjz[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (!PF) {
                if (ld[r]) load_node(planes(p), popb, yo[r], xo, fr[r]);
            }
            moments(fr[r], cdn[r], cjx[r], cjy[r], cjz[r]);
            slot[(wv * R + r) * SUB + ls + 1][lc + 1] = psi_of<C, PSI>(rho_ref + (C)cdn[r]);
        }
        if (has_halo) {
            double hdn;
            C hjx, hjy, hjz;
            if constexpr (!PF) load_node(planes(p), popb, hyo, hxo, fh);
            moments(fh, hdn, hjx, hjy, hjz);
            slot[hy][hx] = psi_of<C, PSI>(rho_ref + (C)hdn);
        }
        if constexpr (PF) {
            if (k + 1 < nplanes) {
                const Planes zn = planes(p + 1);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (ld[r]) load_node(zn, popb, yo[r], xo, fr[r]);
                if (has_halo) load_node(zn, popb, hyo, hxo, fh);
                tkv = __hip_atomic_load(tick_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        } else {
            tkv = __hip_atomic_load(tick_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        __syncthreads();
        if (k >= 2) {
            // collide plane q = p - 1 with psi of planes q - 1, q, q + 1
            const C(*pm)[LX] = ring[(k - 2) & 3];
            const C(*pc)[LX] = ring[(k - 1) & 3];
            const C(*pp)[LX] = ring[k & 3];
            // plane q = p - 1 lies in [z0, z1): its resource needs no wrap
            const Rsrc qr = plane_rsrc(dbuf, p - 1);
            const unsigned qkey = (unsigned)(p - 1) * bd.nxy + seed;   // scalar: plane base + offset
            const int lx = lc + 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!(xstore && yin[r])) continue;
                const int ly = (wv * R + r) * SUB + ls + 1;
                C Fx, Fy, Fz;
                sc_force<C>([&](int dx, int dy, int dz) {
                    return (dz < 0 ? pm : dz > 0 ? pp : pc)[ly + dy][lx + dx];
                }, G, Fx, Fy, Fz);
                const unsigned off = yo[r][1] + xso;
                // stored rows lie inside the box (yg < ny): no wrap
                const unsigned yrow = (unsigned)(y0 + (wv * R + r) * SUB + ls);
                const unsigned key = qkey + yrow * (unsigned)nx + (unsigned)xg;
                if constexpr (TAU1) {
                    collide_store<T, C, true>(qr, popb, off, key, rho_ref, pdn[r], pjx[r], pjy[r],
                                              pjz[r], Fx, Fy, Fz, inv_tau, guo_pref,
                                              (const T*)nullptr);
                } else {
                    // the pre-collision populations of plane q, pulled again
                    T fin[Q];
                    load_node(planes(p - 1), popb, yo[r], xo, fin);
                    collide_store<T, C, false>(qr, popb, off, key, rho_ref, pdn[r], pjx[r], pjy[r],
                                               pjz[r], Fx, Fy, Fz, inv_tau, guo_pref, fin);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pdn[r] = cdn[r];
            pjx[r] = cjx[r];
            pjy[r] = cjy[r];
            pjz[r] = cjz[r];
        }
    }
    if (tick_out && threadIdx.x == 0) *tick_out = tk + 1u;
}

// Full-row tiles (for boxes whose rows are short): the workgroup owns rows [y0, y0 + by) of the
// whole x extent, z planes [z0, z1). Per plane it pulls by + 2 rows (one halo row on each side,
// wrapped) flattened over the row pitch: node m of the list is (m % px, m / px). There is no x
// halo (x neighbours wrap inside the LDS row). Thread t holds list nodes t + k NT - al, k < NPT,
// where al = (y0 - 1) px mod (elements per 128-byte line) puts the lane window on the line grid:
// every wave's loads and stores of the interior rows cover whole lines, whether the rows are
// padded to whole lines (al = 0; the padding lanes store values nobody reads, so that each row's
// last line is written whole) or packed (pitch nx: no idle lanes over padding, and only the two
// lines at the ends of the tile's rows are shared with the neighbouring tiles). The host chooses
// by so that px (by + 2) + al <= NPT NT (row_tile_rows).
template <typename T, typename C, int PSI, bool TAU1, int NPT, int WAVES>
__device__ __forceinline__ void step_rows(const BoxDesc& bd, const T* __restrict__ src,
                                          T* __restrict__ dst, int by, int tiy, int z0, int z1,
                                          const unsigned* tick_in, unsigned* tick_out,
                                          RowRing<C, NPT * 64 * WAVES>& rg)
{
    constexpr int NT = 64 * WAVES;
    auto& ring = rg.v;
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz;
    const int px = (int)bd.px;
    const PopBuf sbuf = make_popbuf(src, bd.pp);
    const PopBuf dbuf = make_popbuf(dst, bd.pp);
    const unsigned popb = sbuf.pop_bytes;
    const C rho_ref = (C)bd.rho_ref;
    const C G = (C)bd.G;
    const C inv_tau = (C)(1.0 / bd.tau);
    const C guo_pref = (C)(1.0 - 0.5 / bd.tau);
    constexpr unsigned E = sizeof(T);
    const unsigned rowb = bd.px * E;
    const int y0 = tiy * by;
    const int M = px * (by + 2);
    constexpr int LINE = 128 / (int)sizeof(T);
    const int al = (((y0 - 1) * px) % LINE + LINE) % LINE;

    // the thread's nodes: LDS position (lx, ly), box coordinates (x, y), load and store flags
    int lxk[NPT], lyk[NPT], xk[NPT], yk[NPT];
    bool ldk[NPT], stk[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int m = (int)threadIdx.x + k * NT - al;
        const bool valid = m >= 0 && m < M;
        const int lx = valid ? m % px : 0;
        const int ly = valid ? m / px : 0;
        const int yg = y0 - 1 + ly;
        lxk[k] = lx < nx ? lx : nx - 1;     // padding lanes read the last column's neighbourhood
        lyk[k] = ly;
        xk[k] = lx;                          // store column (padding included)
        yk[k] = wrapi(yg, ny);
        // rows past ny other than the first (row 0 again, the north neighbour of ny - 1) are
        // not needed
        ldk[k] = valid && lx < nx && yg <= ny;
        stk[k] = valid && ly >= 1 && ly <= by && yg < ny;
    }
    auto node_offsets = [&](int k, unsigned (&xo)[3], unsigned (&yo)[3]) {
        const int x = lxk[k], y = yk[k];
        xo[0] = (unsigned)(x == 0 ? nx - 1 : x - 1) * E;
        xo[1] = (unsigned)x * E;
        xo[2] = (unsigned)(x == nx - 1 ? 0 : x + 1) * E;
        yo[0] = (unsigned)(y == 0 ? ny - 1 : y - 1) * rowb;
        yo[1] = (unsigned)y * rowb;
        yo[2] = (unsigned)(y == ny - 1 ? 0 : y + 1) * rowb;
    };
    auto planes = [&](int p) {
        return Planes{plane_rsrc(sbuf, wrapi(p - 1, nz)), plane_rsrc(sbuf, wrapi(p, nz)),
                      plane_rsrc(sbuf, wrapi(p + 1, nz))};
    };

    double pdn[NPT];
    C pjx[NPT], pjy[NPT], pjz[NPT];
    const int nplanes = (z1 - z0) + 2;
    // step count behind the dither, loaded in every plane and used as in step_tile
    unsigned tkv = 0u, tk = 0u, seed = 0u;
    for (int kp = 0; kp < nplanes; ++kp) {
        const int p = z0 - 1 + kp;
        if (kp == 1) {
            tk = __builtin_amdgcn_readfirstlane(tkv);
            seed = dither_shift(tk);
        }
        const Planes zr = planes(p);
        C* slot = ring[kp & 3];
        double cdn[NPT];
        C cjx[NPT], cjy[NPT], cjz[NPT];
        // Each node's 19 loads are reduced before the next node's are issued: issuing all of the
        // thread's loads first (NPT * 19 in flight per lane) measured slower on the batched mix
        // (3.36 against 3.26 ms per step with 4 nodes per thread, 3.64 against 3.30 with 2).
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            cdn[k] = 0.0;
            cjx[k] = cjy[k] = cjz[k] = C(0);
            if (ldk[k]) {
                unsigned xo[3], yo[3];
                node_offsets(k, xo, yo);
                T f[Q];
                load_node(zr, popb, yo, xo, f);
                moments(f, cdn[k], cjx[k], cjy[k], cjz[k]);
                slot[lyk[k] * nx + xk[k]] = psi_of<C, PSI>(rho_ref + (C)cdn[k]);
            }
        }
        tkv = __hip_atomic_load(tick_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __syncthreads();
        if (kp >= 2) {
            // collide plane q = p - 1 with psi of planes q - 1, q, q + 1
            const C* pm = ring[(kp - 2) & 3];
            const C* pc = ring[(kp - 1) & 3];
            const C* pp = ring[kp & 3];
            // plane q = p - 1 lies in [z0, z1): its resource needs no wrap
            const Rsrc qr = plane_rsrc(dbuf, p - 1);
            const unsigned qkey = (unsigned)(p - 1) * bd.nxy + seed;   // scalar: plane base + offset
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (!stk[k]) continue;
                const int lx = lxk[k];
                const int xw = lx == 0 ? nx - 1 : lx - 1, xe = lx == nx - 1 ? 0 : lx + 1;
                const int r1 = lyk[k] * nx;
                const int xs[3] = {xw, lx, xe};
                C Fx, Fy, Fz;
                sc_force<C>([&](int dx, int dy, int dz) {
                    return (dz < 0 ? pm : dz > 0 ? pp : pc)[r1 + dy * nx + xs[dx + 1]];
                }, G, Fx, Fy, Fz);
                unsigned xo[3], yo[3];
                node_offsets(k, xo, yo);
                const unsigned off = yo[1] + (unsigned)xk[k] * E;
                const unsigned key = qkey + (unsigned)yk[k] * (unsigned)nx + (unsigned)xk[k];
                if constexpr (TAU1) {
                    collide_store<T, C, true>(qr, popb, off, key, rho_ref, pdn[k], pjx[k], pjy[k],
                                              pjz[k], Fx, Fy, Fz, inv_tau, guo_pref,
                                              (const T*)nullptr);
                } else {
                    // the pre-collision populations of plane q, pulled again
                    T fin[Q];
                    load_node(planes(p - 1), popb, yo, xo, fin);
                    collide_store<T, C, false>(qr, popb, off, key, rho_ref, pdn[k], pjx[k], pjy[k],
                                               pjz[k], Fx, Fy, Fz, inv_tau, guo_pref, fin);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            pdn[k] = cdn[k];
            pjx[k] = cjx[k];
            pjy[k] = cjy[k];
            pjz[k] = cjz[k];
        }
    }
    if (tick_out && threadIdx.x == 0) *tick_out = tk + 1u;
}

template <typename T, typename C, int PSI, bool TAU1, int R, bool PF, int WAVES, int BXT>
__global__ __launch_bounds__(64 * WAVES) void k_step(StepArgs a, const T* __restrict__ src,
                                                     T* __restrict__ dst)
{
    __shared__ RingOf<C, R, WAVES, BXT> ring;
    const unsigned logical = a.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tix = (int)(logical % (unsigned)a.tiles_x);
    const unsigned t2 = logical / (unsigned)a.tiles_x;
    const int tiy = (int)(t2 % (unsigned)a.tiles_y);
    const int ch = (int)(t2 / (unsigned)a.tiles_y);
    const int z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, a.b.nz);
    // the dither comes from the box's step count, kept per buffer (tick[s] counts the steps up to
    // the state in buffer s); one workgroup hands the next count to the step that reads the other
    // buffer
    const unsigned* tin = a.b.tick + a.s;
    unsigned* tout = logical == 0 ? a.b.tick + (1 - a.s) : nullptr;
    if constexpr (BXT == 0) step_rows<T, C, PSI, TAU1, R, WAVES>(a.b, src, dst, a.by, tiy, z0, z1, tin, tout, ring);
    else step_tile<T, C, PSI, TAU1, R, PF, WAVES, BXT>(a.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
}

// ------------------------------------------------------------------------------------------
// Two time steps per pass (FP32 storage and arithmetic, tau = 1). A single step streams every
// population in and out of HBM once; here a workgroup keeps the first step's post-collision
// populations of its region in LDS and applies the second step to them, so the box streams
// through HBM once per two steps. The workgroup owns a 64 x 8 tile of the second step's output
// and marches a z chunk. Per plane p it
//   1. pulls the populations of the tile plus a 3-node ring (70 x 14 nodes) from memory (loaded
//      during the previous plane's work): their density and momentum, and psi(t) into an LDS
//      ring of four planes;
//   2. collides plane p - 1 for the tile plus a 2-node ring (68 x 12): the first step, written
//      to LDS (one plane of 19 populations);
//   3. gathers from that plane the populations each node of the tile plus a 1-node ring
//      (66 x 10) pulls: f_i(x, t + 1) = f*_i(x - xi_i, t) comes from plane z - cz_i, so a node of
//      plane p - 2 is complete now (its cz = +1 populations were gathered two planes ago and its
//      cz = 0 ones one plane ago, held in registers), giving density, momentum and psi(t + 1);
//   4. collides plane p - 3 of the tile (the second step) and stores it.
// A chunk of planes [z0, z1) therefore pulls planes z0 - 3 .. z1 + 2. Both steps collide through
// the same routines as the single-step kernels (sc_force, collide_emit) on the same inputs, and
// the first step's values are rounded to FP32 exactly as they would be stored, so two steps here
// give the same bits as two single steps.
// ------------------------------------------------------------------------------------------
// Geometry of a two-step tile BX wide and BY rows high worked by WAVES waves: each thread owns
// BX BY / (64 WAVES) nodes of the second step's tile.
template <int BX_, int BY, int WAVES>
struct T2Geom {
    static constexpr int BX = BX_, NT = 64 * WAVES;
    static constexpr int NO = BX * BY / NT;                 // own nodes per thread
    static constexpr int LX = BX + 6, LY = BY + 6;          // pulled from memory: tile + 3
    static constexpr int AX = BX + 4, AY = BY + 4;          // first step: tile + 2
    static constexpr int GX = BX + 2, GY = BY + 2;          // second step's densities: tile + 1
    static constexpr int NL = LX * LY;
    static constexpr int NSA = (NL + NT - 1) / NT;          // pulled-node slots per thread
    static constexpr int NHR = 2 * GX + 2 * BY;             // ring nodes of the second step
    static constexpr int NSH = (NHR + NT - 1) / NT;         // ring slots per thread
    static constexpr int NB = NO + NSH;                     // gather slots per thread
    static_assert(NO * NT == BX * BY, "the tile must be a whole number of nodes per thread");
};

template <int BX, int BY, int WAVES>
struct Ring2 {
    using G = T2Geom<BX, BY, WAVES>;
    float psa[4][G::LY][G::LX];   // psi(t) of the pulled nodes, planes p - 3 .. p (mod 4)
    float fs[Q][G::AY][G::AX];    // first step's populations of plane p - 1
    float psb[4][G::GY][G::GX];   // psi(t + 1) of the tile plus one, planes p - 5 .. p - 2
};

template <int PSI, int BX, int BY, int WAVES, bool PF>
__device__ __forceinline__ void step_tile2(const BoxDesc& bd, const float* __restrict__ src,
                                           float* __restrict__ dst, int tix, int tiy, int z0,
                                           int z1, const unsigned* tick_in, unsigned* tick_out,
                                           Ring2<BX, BY, WAVES>& rg)
{
    using T = float;
    using C = float;
    using Gm = T2Geom<BX, BY, WAVES>;
    constexpr int NT = Gm::NT, NSA = Gm::NSA, NO = Gm::NO, NB = Gm::NB;
    constexpr int LX = Gm::LX, AX = Gm::AX, AY = Gm::AY, BCX = Gm::GX;
    constexpr unsigned E = sizeof(T);
    const int nx = bd.nx, ny = bd.ny, nz = bd.nz;
    const PopBuf sbuf = make_popbuf(src, bd.pp);
    const PopBuf dbuf = make_popbuf(dst, bd.pp);
    const unsigned popb = sbuf.pop_bytes;
    const C rho_ref = (C)bd.rho_ref;
    const C G = (C)bd.G;
    const unsigned rowb = bd.px * E;
    const unsigned nxy = bd.nxy;
    const int x0 = tix * Gm::BX, y0 = tiy * BY;
    const int t = threadIdx.x;

    // pulled nodes: slot k of thread t is node s = t + k NT of the (BX + 6) x (BY + 6) region, at
    // LDS position (ly, lx) of psa; nodes of the (BX + 4) x (BY + 4) region inside it also
    // collide (first step). A tile cut by the box edge (wv x hv nodes in the box) needs only the
    // (wv + 6) x (hv + 6) corner of the region: the slots beyond it load the corner's last column
    // or row again (lines the wave reads anyway, instead of nodes across the periodic wrap), and
    // what they compute reaches only tile nodes outside the box, which are not stored or land in
    // row padding that nothing reads
    const int wv = min(Gm::BX, nx - x0), hv = min(BY, ny - y0);
    int sx[NSA], sy[NSA];
    bool sin_[NSA], sa[NSA];
    unsigned sxo[NSA][3], syo[NSA][3], skey[NSA];
#pragma unroll
    for (int k = 0; k < NSA; ++k) {
        const int sidx = t + k * NT;
        sin_[k] = sidx < Gm::NL;
        const int lx = sin_[k] ? sidx % LX : 0, ly = sin_[k] ? sidx / LX : 0;
        sx[k] = lx;
        sy[k] = ly;
        sa[k] = sin_[k] && lx >= 1 && lx <= AX && ly >= 1 && ly <= AY;
        const int x = wrapi(x0 - 3 + min(lx, wv + 5), nx), y = wrapi(y0 - 3 + min(ly, hv + 5), ny);
        sxo[k][0] = (unsigned)wrapi(x - 1, nx) * E;
        sxo[k][1] = (unsigned)x * E;
        sxo[k][2] = (unsigned)wrapi(x + 1, nx) * E;
        syo[k][0] = (unsigned)wrapi(y - 1, ny) * rowb;
        syo[k][1] = (unsigned)y * rowb;
        syo[k][2] = (unsigned)wrapi(y + 1, ny) * rowb;
        skey[k] = (unsigned)y * (unsigned)nx + (unsigned)x;   // the node's index in its plane
    }
    // second step: slots j < NO are the thread's own nodes o = t + j NT of the tile, at
    // (o mod BX, o / BX), slots NO + h nodes of the ring around it (ring node t + h NT); (bx, by)
    // are tile coordinates
    int bx[NB], by[NB];
    bool bon[NB];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        const int o = t + j * NT;
        bx[j] = o % BX;
        by[j] = o / BX;
        bon[j] = true;
    }
#pragma unroll
    for (int h = 0; h < Gm::NSH; ++h) {
        const int r = t + h * NT;
        bon[NO + h] = r < Gm::NHR;
        int hx = 0, hy = 0;
        if (r < BCX) {
            hx = r - 1;
            hy = -1;
        } else if (r < 2 * BCX) {
            hx = r - BCX - 1;
            hy = BY;
        } else if (r < 2 * BCX + BY) {
            hx = -1;
            hy = r - 2 * BCX;
        } else if (r < Gm::NHR) {
            hx = Gm::BX;
            hy = r - 2 * BCX - BY;
        }
        bx[NO + h] = hx;
        by[NO + h] = hy;
    }
    // own nodes are stored if they lie in the box (lanes over row padding store values nobody
    // reads, so that every line is written whole)
    bool ost[NO];
    unsigned ooff[NO], okey[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        const int xg = x0 + bx[j], yg = y0 + by[j];
        ost[j] = xg < (int)bd.px && yg < ny;
        ooff[j] = (unsigned)(ost[j] ? yg : 0) * rowb + (unsigned)(ost[j] ? xg : 0) * E;
        okey[j] = (unsigned)(ost[j] ? yg : 0) * (unsigned)nx + (unsigned)(ost[j] ? xg : 0);
    }

    auto planes = [&](int p) {
        return Planes{plane_rsrc(sbuf, wrapi(p - 1, nz)), plane_rsrc(sbuf, wrapi(p, nz)),
                      plane_rsrc(sbuf, wrapi(p + 1, nz))};
    };

    double pdn[NSA];                           // pulled nodes: moments of the previous plane
    C pjx[NSA], pjy[NSA], pjz[NSA];
#pragma unroll
    for (int k = 0; k < NSA; ++k) {
        pdn[k] = 0.0;
        pjx[k] = pjy[k] = pjz[k] = C(0);
    }
    T stz[NB][Q] = {}, st1[NB][Q] = {}, st2[NB][Q] = {};   // gathered cz = 0 / cz = +1 values
    double bdn[NO];                            // own nodes: moments of the last completed plane
    C bjx[NO], bjy[NO], bjz[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        bdn[j] = 0.0;
        bjx[j] = bjy[j] = bjz[j] = C(0);
    }
    unsigned tkv = 0u, tk = 0u, seed_a = 0u, seed_b = 0u;
    const int nk = (z1 - z0) + 6;
    // PF: the populations of the next plane are loaded one iteration ahead, so that the loads are
    // in flight while the two collisions of the current iteration run
    T fnx[NSA][Q];
    if constexpr (PF) {
        const Planes zr = planes(z0 - 3);
#pragma unroll
        for (int k = 0; k < NSA; ++k)
            if (sin_[k]) load_node(zr, popb, syo[k], sxo[k], fnx[k]);
    }
    for (int kp = 0; kp < nk; ++kp) {
        const int p = z0 - 3 + kp;
        if (kp == 1) {
            tk = __builtin_amdgcn_readfirstlane(tkv);
            seed_a = dither_shift(tk);
            seed_b = dither_shift(tk + 1u);
        }
        // 1. plane p: moments and psi(t) of the pulled nodes, then the loads of plane p + 1
        double cdn[NSA];
        C cjx[NSA], cjy[NSA], cjz[NSA];
        {
            float(*ps)[LX] = rg.psa[p & 3];
            const Planes zc = planes(p);
#pragma unroll
            for (int k = 0; k < NSA; ++k) {
                cdn[k] = 0.0;
                cjx[k] = cjy[k] = cjz[k] = C(0);
                if (sin_[k]) {
                    if constexpr (!PF) load_node(zc, popb, syo[k], sxo[k], fnx[k]);
                    moments(fnx[k], cdn[k], cjx[k], cjy[k], cjz[k]);
                    ps[sy[k]][sx[k]] = psi_of<C, PSI>(rho_ref + (C)cdn[k]);
                }
            }
            if (PF && kp + 1 < nk) {
                const Planes zr = planes(p + 1);
#pragma unroll
                for (int k = 0; k < NSA; ++k)
                    if (sin_[k]) load_node(zr, popb, syo[k], sxo[k], fnx[k]);
            }
        }
        tkv = __hip_atomic_load(tick_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __syncthreads();
        // 2. first step on plane q = p - 1
        if (kp >= 2) {
            const float(*am)[LX] = rg.psa[(p - 2) & 3];
            const float(*ac)[LX] = rg.psa[(p - 1) & 3];
            const float(*ap)[LX] = rg.psa[p & 3];
            const unsigned qkey = (unsigned)wrapi(p - 1, nz) * nxy + seed_a;
#pragma unroll
            for (int k = 0; k < NSA; ++k) {
                if (!sa[k]) continue;
                const int lx = sx[k], ly = sy[k];
                C Fx, Fy, Fz;
                sc_force<C>([&](int dx, int dy, int dz) {
                    return (dz < 0 ? am : dz > 0 ? ap : ac)[ly + dy][lx + dx];
                }, G, Fx, Fy, Fz);
                collide_emit<T, C, true>(
                    [&](auto I, T v) { rg.fs[decltype(I)::value][ly - 1][lx - 1] = v; },
                    qkey + skey[k], rho_ref, pdn[k], pjx[k], pjy[k], pjz[k], Fx, Fy, Fz, C(1),
                    C(0.5), (const T*)nullptr);
            }
        }
        __syncthreads();
        // 3. gather from plane p - 1; plane c = p - 2 of the second step is then complete
        double ndn[NO];
        C njx[NO], njy[NO], njz[NO];
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            ndn[j] = 0.0;
            njx[j] = njy[j] = njz[j] = C(0);
        }
        if (kp >= 2) {
            float(*pb)[BCX] = rg.psb[(p - 2) & 3];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (!bon[k]) continue;
                const int gx = bx[k] + 2, gy = by[k] + 2;   // fs coordinates of the node
                T cur[Q];
                static_for<0, Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const T v = rg.fs[i][gy - CY[i]][gx - CX[i]];
                    if constexpr (CZ[i] < 0) {
                        cur[i] = v;
                    } else if constexpr (CZ[i] == 0) {
                        cur[i] = stz[k][i];
                        stz[k][i] = v;
                    } else {
                        cur[i] = st2[k][i];
                        st2[k][i] = st1[k][i];
                        st1[k][i] = v;
                    }
                });
                double dn;
                C jx, jy, jz;
                moments(cur, dn, jx, jy, jz);
                pb[by[k] + 1][bx[k] + 1] = psi_of<C, PSI>(rho_ref + (C)dn);
                if (k < NO) {
                    ndn[k] = dn;
                    njx[k] = jx;
                    njy[k] = jy;
                    njz[k] = jz;
                }
            }
        }
        __syncthreads();
        // 4. second step on plane r = p - 3, stored
        if (kp >= 6) {
            const float(*bm)[BCX] = rg.psb[(p - 4) & 3];
            const float(*bc)[BCX] = rg.psb[(p - 3) & 3];
            const float(*bp)[BCX] = rg.psb[(p - 2) & 3];
            const int r = p - 3;   // in [z0, z1): no wrap
            const Rsrc rr = plane_rsrc(dbuf, r);
            const unsigned rkey = (unsigned)r * nxy + seed_b;
#pragma unroll
            for (int j = 0; j < NO; ++j) {
                if (!ost[j]) continue;
                const int lx = bx[j] + 1, ly = by[j] + 1;
                C Fx, Fy, Fz;
                sc_force<C>([&](int dx, int dy, int dz) {
                    return (dz < 0 ? bm : dz > 0 ? bp : bc)[ly + dy][lx + dx];
                }, G, Fx, Fy, Fz);
                collide_store<T, C, true>(rr, popb, ooff[j], rkey + okey[j], rho_ref, bdn[j],
                                          bjx[j], bjy[j], bjz[j], Fx, Fy, Fz, C(1), C(0.5),
                                          (const T*)nullptr);
            }
        }
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            bdn[j] = ndn[j];
            bjx[j] = njx[j];
            bjy[j] = njy[j];
            bjz[j] = njz[j];
        }
#pragma unroll
        for (int k = 0; k < NSA; ++k) {
            pdn[k] = cdn[k];
            pjx[k] = cjx[k];
            pjy[k] = cjy[k];
            pjz[k] = cjz[k];
        }
    }
    if (tick_out && t == 0) *tick_out = tk + 2u;
}

// MINW: waves per SIMD the register allocation must allow (4: two 8-wave workgroups per CU, at
// most 128 VGPRs).
template <int PSI, int BX, int BY, int WAVES, bool PF, int MINW>
__global__ __launch_bounds__(64 * WAVES, MINW) void k_step2(StepArgs a, const float* __restrict__ src,
                                                            float* __restrict__ dst)
{
    __shared__ Ring2<BX, BY, WAVES> ring;
    const unsigned logical = a.remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tix = (int)(logical % (unsigned)a.tiles_x);
    const unsigned t2 = logical / (unsigned)a.tiles_x;
    const int tiy = (int)(t2 % (unsigned)a.tiles_y);
    const int ch = (int)(t2 / (unsigned)a.tiles_y);
    const int z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, a.b.nz);
    const unsigned* tin = a.b.tick + a.s;
    unsigned* tout = logical == 0 ? a.b.tick + (1 - a.s) : nullptr;
    step_tile2<PSI, BX, BY, WAVES, PF>(a.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
}

// ------------------------------------------------------------------------------------------
// Multi-box step: one launch advances every box of a group by one time step. Work items are
// (box, tile, z chunk) in box-major order; item_begin[b] is the first item of box b. Each box
// has its own size, psi, tau, G, rho_ref, population buffers and chunk length; the launch shape
// (rows, prefetch) is shared. Box b reads pop[(phase_b + parity) & 1] and writes the other.
// ------------------------------------------------------------------------------------------

// Box of a work item: the last box whose first item is <= item.
__device__ __forceinline__ const GroupBox& group_box_of(const GroupBox* __restrict__ boxes, int nbox,
                                                        unsigned item)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].item_begin <= item) lo = mid;
        else hi = mid - 1;
    }
    return boxes[lo];
}

template <typename T, typename C, int R, bool PF, int WAVES, int BXT>
__device__ __forceinline__ void group_item(const GroupBox* __restrict__ boxes, int nbox,
                                           unsigned item, int parity,
                                           RingOf<C, R, WAVES, BXT>& ring)
{
    const GroupBox& g = group_box_of(boxes, nbox, item);
    const unsigned local = item - g.item_begin;
    const int tix = (int)(local % (unsigned)g.tiles_x);
    const unsigned t2 = local / (unsigned)g.tiles_x;
    const int tiy = (int)(t2 % (unsigned)g.tiles_y);
    const int ch = (int)(t2 / (unsigned)g.tiles_y);
    const int z0 = ch * g.zc;
    const int z1 = min(z0 + g.zc, g.b.nz);
    const int s = (g.phase + parity) & 1;
    const T* src = (const T*)g.pop[s];
    T* dst = (T*)g.pop[1 - s];
    // step count behind the dither and its successor, as in the single-box kernel
    const unsigned* tin = g.b.tick + s;
    unsigned* tout = local == 0 ? g.b.tick + (1 - s) : nullptr;
    const bool tau1 = g.b.tau == 1.0;
    if constexpr (BXT == 0) {
        if (g.b.psi == 0) {
            if (tau1) step_rows<T, C, 0, true, R, WAVES>(g.b, src, dst, g.by, tiy, z0, z1, tin, tout, ring);
            else step_rows<T, C, 0, false, R, WAVES>(g.b, src, dst, g.by, tiy, z0, z1, tin, tout, ring);
        } else {
            if (tau1) step_rows<T, C, 1, true, R, WAVES>(g.b, src, dst, g.by, tiy, z0, z1, tin, tout, ring);
            else step_rows<T, C, 1, false, R, WAVES>(g.b, src, dst, g.by, tiy, z0, z1, tin, tout, ring);
        }
    } else {
        if (g.b.psi == 0) {
            if (tau1) step_tile<T, C, 0, true, R, PF, WAVES, BXT>(g.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
            else step_tile<T, C, 0, false, R, PF, WAVES, BXT>(g.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
        } else {
            if (tau1) step_tile<T, C, 1, true, R, PF, WAVES, BXT>(g.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
            else step_tile<T, C, 1, false, R, PF, WAVES, BXT>(g.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
        }
    }
}

// One workgroup per work item (the hardware dispatcher balances the uneven items).
template <typename T, typename C, int R, bool PF, int WAVES, int BXT>
__global__ __launch_bounds__(64 * WAVES) void k_step_group(const GroupBox* __restrict__ boxes,
                                                           int nbox, int parity, int remap)
{
    __shared__ RingOf<C, R, WAVES, BXT> ring;
    const unsigned item = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    group_item<T, C, R, PF, WAVES, BXT>(boxes, nbox, item, parity, ring);
}

// Persistent variant: a fixed grid whose workgroups take items from eight work queues, one per
// XCD (workgroup w runs on XCD w mod 8 and serves queue w mod 8, so the items of a queue - a
// contiguous, work-balanced run of the box-major list - share that XCD's L2). Every workgroup
// draws tickets until its queue is exhausted; the last workgroup to finish clears the queues and
// the finish counter for the next launch, so the kernel needs no host-side reset and can be
// replayed from a captured graph.
template <typename T, typename C, int R, bool PF, int WAVES, int BXT>
__global__ __launch_bounds__(64 * WAVES) void k_step_group_persistent(
    const GroupBox* __restrict__ boxes, int nbox, int parity, QueueState* __restrict__ q)
{
    __shared__ RingOf<C, R, WAVES, BXT> ring;
    __shared__ unsigned ticket;
    const unsigned xcd = blockIdx.x % 8u;
    const unsigned begin = q->range[xcd], end = q->range[xcd + 1];
    for (;;) {
        if (threadIdx.x == 0) ticket = begin + atomicAdd(&q->next[xcd], 1u);
        __syncthreads();
        const unsigned item = ticket;
        __syncthreads();
        if (item >= end) break;
        group_item<T, C, R, PF, WAVES, BXT>(boxes, nbox, item, parity, ring);
        __syncthreads();  // the next item rewrites the LDS ring
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&q->done, 1u);
        if (done == gridDim.x - 1) {
            for (int k = 0; k < 8; ++k) atomicExch(&q->next[k], 0u);
            atomicExch(&q->done, 0u);
            __threadfence();
        }
    }
}

// Two steps per pass over a group (FP32 storage and arithmetic, every box at tau = 1): one
// workgroup per (box, tile, z chunk) item of the list above, each marched by the two-step tile
// kernel's body; a launch moves every box from pop[(phase + parity) & 1] to the other buffer and
// advances its step count by two. With an item order (order != nullptr) the grid is 8 * per
// workgroups: workgroup w runs on XCD w mod 8 and takes order[(w mod 8) * per + w / 8], the XCD's
// share of the items in the order the host chose (NO_ITEM: nothing to do); without it, workgroup w
// takes item w.
template <int BX, int BY, int WAVES, bool PF, int MINW>
__global__ __launch_bounds__(64 * WAVES, MINW) void k_step2_group(const GroupBox* __restrict__ boxes,
                                                                  int nbox, int parity,
                                                                  const unsigned* __restrict__ order,
                                                                  unsigned per)
{
    __shared__ Ring2<BX, BY, WAVES> ring;
    const unsigned item = order ? order[(blockIdx.x % 8u) * per + blockIdx.x / 8u] : blockIdx.x;
    if (item == NO_ITEM) return;
    const GroupBox& g = group_box_of(boxes, nbox, item);
    const unsigned local = item - g.item_begin;
    const int tix = (int)(local % (unsigned)g.tiles_x);
    const unsigned t2 = local / (unsigned)g.tiles_x;
    const int tiy = (int)(t2 % (unsigned)g.tiles_y);
    const int ch = (int)(t2 / (unsigned)g.tiles_y);
    const int z0 = ch * g.zc;
    const int z1 = min(z0 + g.zc, g.b.nz);
    const int s = (g.phase + parity) & 1;
    const float* src = (const float*)g.pop[s];
    float* dst = (float*)g.pop[1 - s];
    const unsigned* tin = g.b.tick + s;
    unsigned* tout = local == 0 ? g.b.tick + (1 - s) : nullptr;
    if (g.b.psi == 0) step_tile2<0, BX, BY, WAVES, PF>(g.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
    else step_tile2<1, BX, BY, WAVES, PF>(g.b, src, dst, tix, tiy, z0, z1, tin, tout, ring);
}

template <typename T, typename C, int PSI, bool TAU1, int R, bool PF, int WAVES, int BXT>
hipError_t launch_step_t(const StepArgs& a, const void* src, void* dst, hipStream_t st)
{
    const unsigned grid = (unsigned)(a.tiles_x * a.tiles_y * a.nchunks);
    hipLaunchKernelGGL((k_step<T, C, PSI, TAU1, R, PF, WAVES, BXT>), dim3(grid), dim3(64 * WAVES),
                       0, st, a, (const T*)src, (T*)dst);
    return hipGetLastError();
}

// Supported launch shapes (checked by shape_supported): 4 waves with rows 1, 2 or 4 and either
// prefetch setting; 8 waves with rows 1 or 2 and no prefetch; tile width 32 with rows 1 or 2;
// full-row tiles (tile width 0) without prefetch, with 8 waves and 2, 4 or 8 nodes per thread, or
// with 4 waves and 4 nodes per thread.
template <typename T, typename C, int PSI, bool TAU1>
hipError_t dispatch_pf(const StepShape& s, const StepArgs& a, const void* src, void* dst,
                       hipStream_t st)
{
#define LBM_STEP(R, PF, WV, BXT) launch_step_t<T, C, PSI, TAU1, R, PF, WV, BXT>(a, src, dst, st)
    if (s.tile_x == 0) {
        if (s.waves == 4) return LBM_STEP(4, false, 4, 0);
        if (s.rows == 2) return LBM_STEP(2, false, 8, 0);
        // 8 nodes per thread only with single-precision arithmetic (in double it spills)
        if constexpr (sizeof(C) == 8) return s.rows == 4 ? LBM_STEP(4, false, 8, 0) : hipErrorInvalidValue;
        else return s.rows == 4 ? LBM_STEP(4, false, 8, 0) : LBM_STEP(8, false, 8, 0);
    }
    if (s.waves == 8) {
        if (s.tile_x == 32) return s.rows == 1 ? LBM_STEP(1, false, 8, 32) : LBM_STEP(2, false, 8, 32);
        return s.rows == 1 ? LBM_STEP(1, false, 8, 64) : LBM_STEP(2, false, 8, 64);
    }
    if (s.tile_x == 32) {
        if (s.prefetch) return s.rows == 1 ? LBM_STEP(1, true, 4, 32) : LBM_STEP(2, true, 4, 32);
        return s.rows == 1 ? LBM_STEP(1, false, 4, 32) : LBM_STEP(2, false, 4, 32);
    }
    if (s.prefetch) {
        switch (s.rows) {
            case 1: return LBM_STEP(1, true, 4, 64);
            case 2: return LBM_STEP(2, true, 4, 64);
            default: return LBM_STEP(4, true, 4, 64);
        }
    }
    switch (s.rows) {
        case 1: return LBM_STEP(1, false, 4, 64);
        case 2: return LBM_STEP(2, false, 4, 64);
        default: return LBM_STEP(4, false, 4, 64);
    }
#undef LBM_STEP
}

template <typename T, typename C>
hipError_t dispatch_step(const StepShape& s, const StepArgs& a, const void* src, void* dst,
                         hipStream_t st)
{
    const bool tau1 = a.b.tau == 1.0;
    if (a.b.psi == 0)
        return tau1 ? dispatch_pf<T, C, 0, true>(s, a, src, dst, st)
                    : dispatch_pf<T, C, 0, false>(s, a, src, dst, st);
    return tau1 ? dispatch_pf<T, C, 1, true>(s, a, src, dst, st)
                : dispatch_pf<T, C, 1, false>(s, a, src, dst, st);
}

// One step of one box in the storage type T and arithmetic type C.
template <typename T, typename C>
hipError_t launch_step_impl(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                            void* dst, hipStream_t st)
{
    StepArgs a;
    a.b = b;
    a.s = sbuf;
    a.by = 0;
    if (s.tile_x == 0) {
        a.by = row_tile_rows(s, b.px);
        if (a.by < 1) return hipErrorInvalidValue;
        a.tiles_x = 1;
        a.tiles_y = (b.ny + a.by - 1) / a.by;
    } else {
        a.tiles_x = (b.nx + s.tile_x - 1) / s.tile_x;
        const int by = tile_height(s);
        a.tiles_y = (b.ny + by - 1) / by;
    }
    a.zc = s.z_chunk < b.nz ? s.z_chunk : b.nz;
    a.nchunks = (b.nz + a.zc - 1) / a.zc;
    a.remap = s.xcd_remap;
    return dispatch_step<T, C>(s, a, src, dst, st);
}

template <typename T, typename C, int R, bool PF, int WAVES, int BXT>
hipError_t launch_group_t(const GroupBox* boxes, int nbox, unsigned nitems, int parity,
                          int persistent, int remap, unsigned workers, QueueState* q,
                          hipStream_t st)
{
    if (persistent)
        hipLaunchKernelGGL((k_step_group_persistent<T, C, R, PF, WAVES, BXT>), dim3(workers),
                           dim3(64 * WAVES), 0, st, boxes, nbox, parity, q);
    else
        hipLaunchKernelGGL((k_step_group<T, C, R, PF, WAVES, BXT>), dim3(nitems), dim3(64 * WAVES), 0,
                           st, boxes, nbox, parity, remap);
    return hipGetLastError();
}

template <typename T, typename C>
hipError_t launch_group_shape(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                              int parity, int persistent, unsigned workers, QueueState* q,
                              hipStream_t st)
{
#define LBM_GROUP(R, PF, WV, BXT) \
    launch_group_t<T, C, R, PF, WV, BXT>(boxes, nbox, nitems, parity, persistent, s.xcd_remap, workers, q, st)
    if (s.tile_x == 0) {
        if (s.waves == 4) return LBM_GROUP(4, false, 4, 0);
        if (s.rows == 2) return LBM_GROUP(2, false, 8, 0);
        if constexpr (sizeof(C) == 8) return s.rows == 4 ? LBM_GROUP(4, false, 8, 0) : hipErrorInvalidValue;
        else return s.rows == 4 ? LBM_GROUP(4, false, 8, 0) : LBM_GROUP(8, false, 8, 0);
    }
    if (s.waves == 8) {
        if (s.tile_x == 32) return s.rows == 1 ? LBM_GROUP(1, false, 8, 32) : LBM_GROUP(2, false, 8, 32);
        return s.rows == 1 ? LBM_GROUP(1, false, 8, 64) : LBM_GROUP(2, false, 8, 64);
    }
    if (s.tile_x == 32) {
        if (s.prefetch) return s.rows == 1 ? LBM_GROUP(1, true, 4, 32) : LBM_GROUP(2, true, 4, 32);
        return s.rows == 1 ? LBM_GROUP(1, false, 4, 32) : LBM_GROUP(2, false, 4, 32);
    }
    if (s.prefetch) {
        switch (s.rows) {
            case 1: return LBM_GROUP(1, true, 4, 64);
            case 2: return LBM_GROUP(2, true, 4, 64);
            default: return LBM_GROUP(4, true, 4, 64);
        }
    }
    switch (s.rows) {
        case 1: return LBM_GROUP(1, false, 4, 64);
        case 2: return LBM_GROUP(2, false, 4, 64);
        default: return LBM_GROUP(4, false, 4, 64);
    }
#undef LBM_GROUP
}

}  // namespace
}  // namespace lbm
