// Device kernels of the Shan-Chen D3Q19 lattice Boltzmann library (gfx950) other than the fused
// step: initial state, conversion between the stored and the canonical FP64 layout, FP64
// observation, the streaming-copy reference and the allocation-free step's work-list writers; plus
// the host launchers, which dispatch the fused step to the translation unit of each precision
// (step_f32.hip, step_m64.hip, step_f64.hip). The step kernels and the shared device helpers are
// in step_kernels.hpp.
#include <mutex>
#include <type_traits>

#include "step_kernels.hpp"

// Work list and queue state of the allocation-free multi-box step (lbm_sc_step_boxes_noalloc):
// one fixed array per GPU, held until the process ends. Host code never uses this name as an
// address (it is a host-side stand-in there); it reads the device address once per device with
// hipGetSymbolAddress (noalloc_scratch_address) and passes that to the kernels.
static __device__ __align__(256) unsigned char scratch[lbm::noalloc_queue_offset() +
                                                       sizeof(lbm::QueueState)];

namespace lbm {
namespace {


// ------------------------------------------------------------------------------------------
// Initial state
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long s)
{
    unsigned long long z = s + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int min_image(int v, int c, int L)
{
    int d = v - c;
    if (2 * d > L) d -= L;
    if (2 * d < -L) d += L;
    return d;
}

__global__ void k_init_density(BoxDesc b, InitDesc d, double* __restrict__ dn,
                               double* __restrict__ dpsi)
{
    const unsigned k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n) return;
    const int x = (int)(k % (unsigned)b.nx);
    const int y = (int)((k / (unsigned)b.nx) % (unsigned)b.ny);
    const int z = (int)(k / b.nxy);
    const double dx = min_image(x, b.nx / 2, b.nx);
    const double dy = min_image(y, b.ny / 2, b.ny);
    const double dz = min_image(z, b.nz / 2, b.nz);
    double r;
    if (d.geom == 2) {
        const double dd = d.slab_axis == 0 ? dx : (d.slab_axis == 1 ? dy : dz);
        r = fabs(dd);
    } else {
        r = sqrt(dx * dx + dy * dy + dz * dz);
    }
    double n = 0.5 * (d.n_in + d.n_out) - 0.5 * (d.n_in - d.n_out) * tanh((r - d.radius) / d.width);
    if (d.noise_amp != 0.0) {
        const double u = (double)(splitmix64(d.seed ^ (unsigned long long)k) >> 11) *
                         (1.0 / 9007199254740992.0);
        n += d.noise_amp * (2.0 * u - 1.0);
    }
    dn[k] = n;
    dpsi[k] = psi_rt(n, b.psi);
}

// S = sum_a w_a psi(x + xi_a) xi_a from a psi field with periodic wrap.
__device__ __forceinline__ void sc_sum(const BoxDesc& b, const double* __restrict__ psi, int x,
                                       int y, int z, double& Sx, double& Sy, double& Sz)
{
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const unsigned k = ((unsigned)wrapi(z + CZ[i], b.nz) * (unsigned)b.ny +
                            (unsigned)wrapi(y + CY[i], b.ny)) * (unsigned)b.nx +
                           (unsigned)wrapi(x + CX[i], b.nx);
        const double v = weight(i) * psi[k];
        sx += CX[i] * v;
        sy += CY[i] * v;
        sz += CZ[i] * v;
    }
    Sx = sx;
    Sy = sy;
    Sz = sz;
}

template <typename T>
__global__ void k_init_pops(BoxDesc b, const double* __restrict__ dn,
                            const double* __restrict__ dpsi, T* __restrict__ dst)
{
    const unsigned k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n) return;
    const int x = (int)(k % (unsigned)b.nx);
    const int y = (int)((k / (unsigned)b.nx) % (unsigned)b.ny);
    const int z = (int)(k / b.nxy);
    double Sx, Sy, Sz;
    sc_sum(b, dpsi, x, y, z, Sx, Sy, Sz);
    const double n = dn[k];
    const double g = -b.G * dpsi[k];
    // zero physical velocity: u = -F/(2n)
    const double ux = -0.5 * g * Sx / n, uy = -0.5 * g * Sy / n, uz = -0.5 * g * Sz / n;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double c = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const double f = weight(i) * n * (1.0 + 3.0 * c + 4.5 * c * c - 1.5 * uu);
        // f_i(x, 0) is the pull of the stored slot at x - xi_i
        dst[pop_index(b, i, wrapi(x - CX[i], b.nx), wrapi(y - CY[i], b.ny), wrapi(z - CZ[i], b.nz))] =
            (T)(f - weight(i) * b.rho_ref);
    }
}

// ------------------------------------------------------------------------------------------
// Canonical FP64 <-> stored conversion (one population per launch)
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ void k_get(BoxDesc b, int i, int cx, int cy, int cz, double w, const T* __restrict__ src,
                      double* __restrict__ out)
{
    const unsigned k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n) return;
    const int x = (int)(k % (unsigned)b.nx);
    const int y = (int)((k / (unsigned)b.nx) % (unsigned)b.ny);
    const int z = (int)(k / b.nxy);
    out[k] = (double)src[pop_index(b, i, wrapi(x - cx, b.nx), wrapi(y - cy, b.ny), wrapi(z - cz, b.nz))] +
             w * b.rho_ref;
}

template <typename T>
__global__ void k_set(BoxDesc b, int i, int cx, int cy, int cz, double w, const double* __restrict__ in,
                      T* __restrict__ dst)
{
    const unsigned k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n) return;
    const int x = (int)(k % (unsigned)b.nx);
    const int y = (int)((k / (unsigned)b.nx) % (unsigned)b.ny);
    const int z = (int)(k / b.nxy);
    // the slot at x holds the population that arrives at x + xi_i
    const unsigned s = ((unsigned)wrapi(z + cz, b.nz) * (unsigned)b.ny +
                        (unsigned)wrapi(y + cy, b.ny)) * (unsigned)b.nx +
                       (unsigned)wrapi(x + cx, b.nx);
    dst[pop_index(b, i, x, y, z)] = (T)(in[s] - w * b.rho_ref);
}

// ------------------------------------------------------------------------------------------
// Observation (FP64)
// ------------------------------------------------------------------------------------------

template <typename T>
__global__ void k_obs_pull(BoxDesc b, const T* __restrict__ src, double* __restrict__ dn,
                           double* __restrict__ dpsi, double* __restrict__ dj)
{
    for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < b.n;
         k += gridDim.x * blockDim.x) {
        const int x = (int)(k % (unsigned)b.nx);
        const int y = (int)((k / (unsigned)b.nx) % (unsigned)b.ny);
        const int z = (int)(k / b.nxy);
        double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const unsigned long long o = pop_index(b, i, wrapi(x - CX[i], b.nx), wrapi(y - CY[i], b.ny),
                                                   wrapi(z - CZ[i], b.nz));
            const double f = (double)src[o] + weight(i) * b.rho_ref;
            s += f;
            jx += CX[i] * f;
            jy += CY[i] * f;
            jz += CZ[i] * f;
        }
        dn[k] = s;
        dpsi[k] = psi_rt(s, b.psi);
        dj[k] = jx;
        dj[b.n + k] = jy;
        dj[2 * (unsigned long long)b.n + k] = jz;
    }
}

enum { P_MASS = 0, P_MX, P_MY, P_MZ, P_CX, P_CY, P_CZ, P_DU, P_DMAX, P_BAD, P_NMIN, P_NMAX };
static_assert(P_NMAX < OBS_PARTS, "partials");

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
    return v;
}

// Offset from the centre used by the centre of mass: minimum image, and 0 for the node exactly
// half a box away (it lies on both sides).
__device__ __forceinline__ double com_offset(int v, int L)
{
    const int d = min_image(v, L / 2, L);
    return (2 * d == L || 2 * d == -L) ? 0.0 : (double)d;
}

// Force, physical velocity and the FP64 reductions of one observation. dj holds the momentum
// sum_i xi_i f_i (from k_obs_pull); uprev holds the velocity of the previous observation and is
// overwritten, node by node, with this one's (each node is read and written by one thread).
__global__ __launch_bounds__(256) void k_obs_reduce(BoxDesc b, const double* __restrict__ dn,
                                                    const double* __restrict__ dpsi,
                                                    const double* __restrict__ dj,
                                                    double* __restrict__ uprev,
                                                    int has_prev, double* __restrict__ parts)
{
    double acc[OBS_PARTS];
#pragma unroll
    for (int q = 0; q < OBS_PARTS; ++q) acc[q] = 0.0;
    acc[P_NMIN] = 1.0e300;
    acc[P_NMAX] = -1.0e300;
    const unsigned long long N = b.n;
    for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < b.n;
         k += gridDim.x * blockDim.x) {
        const int x = (int)(k % (unsigned)b.nx);
        const int y = (int)((k / (unsigned)b.nx) % (unsigned)b.ny);
        const int z = (int)(k / b.nxy);
        double Sx, Sy, Sz;
        sc_sum(b, dpsi, x, y, z, Sx, Sy, Sz);
        const double g = -b.G * dpsi[k];
        const double Fx = g * Sx, Fy = g * Sy, Fz = g * Sz;
        const double n = dn[k];
        const double px = dj[k] + 0.5 * Fx, py = dj[N + k] + 0.5 * Fy, pz = dj[2 * N + k] + 0.5 * Fz;
        const double ux = px / n, uy = py / n, uz = pz / n;
        acc[P_MASS] += n;
        acc[P_MX] += px;
        acc[P_MY] += py;
        acc[P_MZ] += pz;
        acc[P_CX] += n * com_offset(x, b.nx);
        acc[P_CY] += n * com_offset(y, b.ny);
        acc[P_CZ] += n * com_offset(z, b.nz);
        if (has_prev) {
            const double ex = fabs(ux - uprev[k]), ey = fabs(uy - uprev[N + k]),
                         ez = fabs(uz - uprev[2 * N + k]);
            acc[P_DU] += ex + ey + ez;
            acc[P_DMAX] = fmax(acc[P_DMAX], fmax(ex, fmax(ey, ez)));
        }
        uprev[k] = ux;
        uprev[N + k] = uy;
        uprev[2 * N + k] = uz;
        const bool ok = (n > 0.0) && isfinite(n) && isfinite(ux) && isfinite(uy) && isfinite(uz);
        if (!ok) acc[P_BAD] += 1.0;
        acc[P_NMIN] = fmin(acc[P_NMIN], n);
        acc[P_NMAX] = fmax(acc[P_NMAX], n);
    }
    __shared__ double red[4][OBS_PARTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < OBS_PARTS; ++q) {
        double v;
        if (q == P_DMAX || q == P_NMAX) v = wave_max(acc[q]);
        else if (q == P_NMIN) v = wave_min(acc[q]);
        else v = wave_sum(acc[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < OBS_PARTS) {
        const int q = threadIdx.x;
        double v = red[0][q];
        for (int w = 1; w < 4; ++w) {
            if (q == P_DMAX || q == P_NMAX) v = fmax(v, red[w][q]);
            else if (q == P_NMIN) v = fmin(v, red[w][q]);
            else v += red[w][q];
        }
        parts[blockIdx.x * OBS_PARTS + q] = v;
    }
}

__global__ void k_obs_final(const double* __restrict__ parts, int nblocks, double* __restrict__ scal)
{
    const int q = threadIdx.x;
    if (q >= OBS_PARTS) return;
    double v = parts[q];
    for (int blk = 1; blk < nblocks; ++blk) {
        const double p = parts[blk * OBS_PARTS + q];
        if (q == P_DMAX || q == P_NMAX) v = fmax(v, p);
        else if (q == P_NMIN) v = fmin(v, p);
        else v += p;
    }
    scal[q] = v;
}

// Diagonal of the lattice pressure tensor, Eq. (sm:pt):
//   P^aa = n c_s^2 + (G c_s^2/2) psi(x) sum_a W_a psi(x + xi_a) (xi_a^a)^2
//        = n/3 + (G/2) psi(x) sum_a w_a psi(x + xi_a) (xi_a^a)^2.
__device__ __forceinline__ void pt_diag(const BoxDesc& b, const double* __restrict__ dn,
                                        const double* __restrict__ psi, int x, int y, int z,
                                        double& n, double& Pxx, double& Pyy, double& Pzz)
{
    double sxx = 0.0, syy = 0.0, szz = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const unsigned k = ((unsigned)wrapi(z + CZ[i], b.nz) * (unsigned)b.ny +
                            (unsigned)wrapi(y + CY[i], b.ny)) * (unsigned)b.nx +
                           (unsigned)wrapi(x + CX[i], b.nx);
        const double v = weight(i) * psi[k];
        sxx += CX[i] * CX[i] * v;
        syy += CY[i] * CY[i] * v;
        szz += CZ[i] * CZ[i] * v;
    }
    const unsigned k0 = ((unsigned)z * (unsigned)b.ny + (unsigned)y) * (unsigned)b.nx + (unsigned)x;
    n = dn[k0];
    const double h = 0.5 * b.G * psi[k0];
    Pxx = n / 3.0 + h * sxx;
    Pyy = n / 3.0 + h * syy;
    Pzz = n / 3.0 + h * szz;
}

// probes[0..3] = n and P^xx at the centre, n and P^xx at the far probe.
__global__ void k_probes(BoxDesc b, const double* __restrict__ dn, const double* __restrict__ dpsi,
                         double* __restrict__ probes)
{
    const int t = threadIdx.x;
    if (t >= 2) return;
    const int cx = b.nx / 2, cy = b.ny / 2, cz = b.nz / 2;
    const int x = t == 0 ? cx : (cx + b.nx / 2) % b.nx;
    const int y = t == 0 ? cy : (cy + b.ny / 2) % b.ny;
    const int z = t == 0 ? cz : (cz + b.nz / 2) % b.nz;
    double n, pxx, pyy, pzz;
    pt_diag(b, dn, dpsi, x, y, z, n, pxx, pyy, pzz);
    probes[2 * t] = n;
    probes[2 * t + 1] = pxx;
}

__global__ void k_profile_line(BoxDesc b, const double* __restrict__ dn,
                               const double* __restrict__ dpsi, double* __restrict__ prof)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= b.nx) return;
    double n, pxx, pyy, pzz;
    pt_diag(b, dn, dpsi, x, b.ny / 2, b.nz / 2, n, pxx, pyy, pzz);
    prof[x] = n;
    prof[b.nx + x] = pxx;
    prof[2 * b.nx + x] = pyy;
    prof[3 * b.nx + x] = pzz;
}

// One workgroup per plane normal to `axis`; plane averages of n, P^xx, P^yy, P^zz.
__global__ __launch_bounds__(256) void k_profile_planes(BoxDesc b, int axis,
                                                       const double* __restrict__ dn,
                                                       const double* __restrict__ dpsi,
                                                       double* __restrict__ prof)
{
    const int s = blockIdx.x;
    const int L = axis == 0 ? b.nx : (axis == 1 ? b.ny : b.nz);
    const int A = axis == 0 ? b.ny : b.nx;  // first in-plane axis length
    const int B = axis == 2 ? b.ny : b.nz;  // second in-plane axis length
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < A * B; t += blockDim.x) {
        const int a = t % A, c = t / A;
        int x, y, z;
        if (axis == 0) { x = s; y = a; z = c; }
        else if (axis == 1) { x = a; y = s; z = c; }
        else { x = a; y = c; z = s; }
        double n, pxx, pyy, pzz;
        pt_diag(b, dn, dpsi, x, y, z, n, pxx, pyy, pzz);
        acc[0] += n;
        acc[1] += pxx;
        acc[2] += pyy;
        acc[3] += pzz;
    }
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        const double v = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
        prof[q * L + s] = v / (double)(A * B);
    }
}

unsigned blocks_for(unsigned n, unsigned bs) { return (n + bs - 1) / bs; }

// Streaming copy used as the achievable-bandwidth reference: each lane moves V (4, 8 or 16
// bytes: one, two or four floats) per access; each workgroup copies one contiguous block of
// 4 * 256 elements (four loads in flight per thread), with non-temporal stores, and the grid
// covers the whole range once, so the workgroups in flight touch one compact, advancing window
// of addresses. Measured on MI355X with 2 GiB: 6.47 TB/s (4-byte lanes), 6.23 (8), 5.70 (16),
// against 5.64 TB/s for a grid-stride loop over 1024 workgroups (4.31 with 16-byte lanes) and
// 4.86 TB/s for hipMemcpy.
typedef float CopyV2 __attribute__((ext_vector_type(2)));
typedef float CopyV4 __attribute__((ext_vector_type(4)));

template <typename V>
__global__ __launch_bounds__(256) void k_stream_copy(const V* __restrict__ src,
                                                     V* __restrict__ dst, size_t n)
{
    constexpr int U = 4;
    const size_t base = (size_t)blockIdx.x * (256 * U) + threadIdx.x;
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
}

// Copy a batch of work-list descriptors, passed by value as a kernel argument, to their slots in
// the allocation-free step's array (word by word; the batch is a few KB).
__global__ __launch_bounds__(256) void k_put_descs(DescBatch b, GroupBox* __restrict__ dst)
{
    static_assert(sizeof(GroupBox) % 4 == 0, "descriptors are copied in 32-bit words");
    constexpr int WORDS = (int)(sizeof(GroupBox) / 4);
    const unsigned* src = reinterpret_cast<const unsigned*>(b.d);
    unsigned* out = reinterpret_cast<unsigned*>(dst + b.first);
    for (int k = threadIdx.x; k < b.count * WORDS; k += blockDim.x) out[k] = src[k];
}

__global__ void k_put_queue(QueueState q, QueueState* __restrict__ dst)
{
    if (threadIdx.x == 0) *dst = q;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

// Device address of `scratch` on the current device. Each GPU holds its own copy of the array at
// its own address, so the address is looked up once per device (with that device current) and
// kept; every later call returns the kept address.
hipError_t noalloc_scratch_address(void** ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_put_descs(const DescBatch& b, void* scratch_dev, hipStream_t st)
{
    if (b.count < 1 || b.count > NOALLOC_BATCH || b.first < 0 ||
        b.first + b.count > NOALLOC_MAX_BOXES)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_put_descs, dim3(1), dim3(256), 0, st, b,
                       reinterpret_cast<GroupBox*>(scratch_dev));
    return hipGetLastError();
}

hipError_t launch_put_queue(const QueueState& q, void* scratch_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_put_queue, dim3(1), dim3(64), 0, st, q,
                       reinterpret_cast<QueueState*>(static_cast<char*>(scratch_dev) +
                                                     noalloc_queue_offset()));
    return hipGetLastError();
}

hipError_t launch_step(bool fp32, bool math64, const BoxDesc& b, const StepShape& s, int sbuf,
                       const void* src, void* dst, hipStream_t st)
{
    if (!shape_supported(s) || (sbuf & ~1)) return hipErrorInvalidValue;
    if (!fp32) return launch_step_f64(b, s, sbuf, src, dst, st);
    return math64 ? launch_step_m64(b, s, sbuf, src, dst, st) : launch_step_f32(b, s, sbuf, src, dst, st);
}

hipError_t launch_step_group(bool fp32, bool math64, const StepShape& s, const GroupBox* boxes, int nbox,
                             unsigned nitems, int parity, int persistent, unsigned workers,
                             QueueState* q, hipStream_t st)
{
    if (!shape_supported(s)) return hipErrorInvalidValue;
    if (nbox <= 0 || nitems == 0) return hipSuccess;
    if (!fp32) return launch_group_f64(s, boxes, nbox, nitems, parity, persistent, workers, q, st);
    return math64 ? launch_group_m64(s, boxes, nbox, nitems, parity, persistent, workers, q, st)
                  : launch_group_f32(s, boxes, nbox, nitems, parity, persistent, workers, q, st);
}


hipError_t launch_init(bool fp32, const BoxDesc& b, const InitDesc& d, double* dn, double* dpsi,
                       void* dst, hipStream_t st)
{
    const unsigned g = blocks_for(b.n, 256);
    hipLaunchKernelGGL(k_init_density, dim3(g), dim3(256), 0, st, b, d, dn, dpsi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fp32)
        hipLaunchKernelGGL(k_init_pops<float>, dim3(g), dim3(256), 0, st, b, (const double*)dn,
                           (const double*)dpsi, (float*)dst);
    else
        hipLaunchKernelGGL(k_init_pops<double>, dim3(g), dim3(256), 0, st, b, (const double*)dn,
                           (const double*)dpsi, (double*)dst);
    return hipGetLastError();
}

hipError_t launch_get(bool fp32, const BoxDesc& b, int i, const void* src, double* out,
                      hipStream_t st)
{
    const unsigned g = blocks_for(b.n, 256);
    if (fp32)
        hipLaunchKernelGGL(k_get<float>, dim3(g), dim3(256), 0, st, b, i, CX[i], CY[i], CZ[i],
                           weight(i), (const float*)src, out);
    else
        hipLaunchKernelGGL(k_get<double>, dim3(g), dim3(256), 0, st, b, i, CX[i], CY[i], CZ[i],
                           weight(i), (const double*)src, out);
    return hipGetLastError();
}

hipError_t launch_set(bool fp32, const BoxDesc& b, int i, const double* in, void* dst,
                      hipStream_t st)
{
    const unsigned g = blocks_for(b.n, 256);
    if (fp32)
        hipLaunchKernelGGL(k_set<float>, dim3(g), dim3(256), 0, st, b, i, CX[i], CY[i], CZ[i],
                           weight(i), in, (float*)dst);
    else
        hipLaunchKernelGGL(k_set<double>, dim3(g), dim3(256), 0, st, b, i, CX[i], CY[i], CZ[i],
                           weight(i), in, (double*)dst);
    return hipGetLastError();
}

hipError_t launch_observe(bool fp32, const BoxDesc& b, const void* src, double* dn, double* dpsi,
                          double* dj, double* uprev, int has_prev, double* parts,
                          double* scal, hipStream_t st)
{
    const unsigned g = blocks_for(b.n, 256) < 4096u ? blocks_for(b.n, 256) : 4096u;
    if (fp32)
        hipLaunchKernelGGL(k_obs_pull<float>, dim3(g), dim3(256), 0, st, b, (const float*)src, dn,
                           dpsi, dj);
    else
        hipLaunchKernelGGL(k_obs_pull<double>, dim3(g), dim3(256), 0, st, b, (const double*)src,
                           dn, dpsi, dj);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_reduce, dim3(OBS_BLOCKS), dim3(256), 0, st, b, (const double*)dn,
                       (const double*)dpsi, (const double*)dj, uprev, has_prev, parts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(64), 0, st, (const double*)parts, OBS_BLOCKS,
                       scal);
    return hipGetLastError();
}

template <typename V>
hipError_t launch_copy_t(const void* src, void* dst, size_t bytes, hipStream_t st)
{
    const size_t n = bytes / sizeof(V);
    if (n == 0) return hipSuccess;
    const size_t grid = (n + 1023) / 1024;
    if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy<V>, dim3((unsigned)grid), dim3(256), 0, st, (const V*)src,
                       (V*)dst, n);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int lane_bytes,
                              hipStream_t st)
{
    switch (lane_bytes) {
        case 4: return launch_copy_t<float>(src, dst, bytes, st);
        case 8: return launch_copy_t<CopyV2>(src, dst, bytes, st);
        case 16: return launch_copy_t<CopyV4>(src, dst, bytes, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_profile_line(const BoxDesc& b, const double* dn, const double* dpsi,
                               double* prof, double* probes, hipStream_t st)
{
    hipLaunchKernelGGL(k_profile_line, dim3(blocks_for(b.nx, 256)), dim3(256), 0, st, b, dn, dpsi,
                       prof);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probes, dim3(1), dim3(64), 0, st, b, dn, dpsi, probes);
    return hipGetLastError();
}

hipError_t launch_profile_planes(const BoxDesc& b, int axis, const double* dn, const double* dpsi,
                                 double* prof, double* probes, hipStream_t st)
{
    const int L = axis == 0 ? b.nx : (axis == 1 ? b.ny : b.nz);
    hipLaunchKernelGGL(k_profile_planes, dim3(L), dim3(256), 0, st, b, axis, dn, dpsi, prof);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probes, dim3(1), dim3(64), 0, st, b, dn, dpsi, probes);
    return hipGetLastError();
}

}  // namespace lbm
