// Host-side declarations of the device launchers (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Geometry and physics of one box, passed by value to every kernel.
struct BoxDesc {
    int nx, ny, nz;
    unsigned nxy;            // nx * ny
    unsigned n;              // nx * ny * nz (nodes; canonical index (z * ny + y) * nx + x)
    unsigned px;             // row pitch of the stored populations (elements, >= nx, whole
                             // 128-byte lines)
    unsigned pxy;            // px * ny
    unsigned pp;             // population pitch: elements between the population planes of one
                             // z-plane (>= pxy); population i of node (x, y, z) is stored at
                             // element (z * 19 + i) * pp + y * px + x
    unsigned* tick;          // device: step counts that seed the FP32 rest-population dither;
                             // tick[s] belongs to the state held in population buffer s
    int psi;                 // 0: exp(-1/n), 1: 1 - exp(-n)
    double G;
    double tau;
    double rho_ref;          // 0 for FP64 storage
};

// Launch shape of the fused step kernel. The workgroup is 64 * waves threads (waves wave64s); the
// tile is tile_x nodes wide (64, or 32 with each wave row split into two sub-rows), tile_height()
// rows high and z_chunk planes deep. tile_x = 0 selects full-row tiles: the whole x extent and
// row_tile_rows() rows, with `rows` nodes per thread and plane.
struct StepShape {
    int rows;        // rows of the tile per wave (1, 2 or 4); full-row tiles: nodes per thread (4, 8)
    int waves;       // wave64s per workgroup (4 or 8)
    int z_chunk;     // planes marched per workgroup
    int xcd_remap;   // 1: map consecutive logical tiles to one XCD
    int prefetch;    // 1: issue the next plane's loads before the barrier (software pipelining)
    int tile_x;      // tile width: 64, 32, or 0 for full-row tiles
};

// The compiled shapes: 4 waves with rows 1, 2 or 4 (rows 1 or 2 at tile width 32), either
// prefetch setting; 8 waves with rows 1 or 2 and no prefetch; full-row tiles (tile width 0)
// without prefetch, 8 waves with 2, 4 or 8 nodes per thread or 4 waves with 4.
inline bool shape_supported(const StepShape& s)
{
    if (s.z_chunk < 1 || (s.xcd_remap & ~1) || (s.prefetch & ~1)) return false;
    if (s.tile_x == 0)
        return s.prefetch == 0 && ((s.waves == 8 && (s.rows == 2 || s.rows == 4 || s.rows == 8)) ||
                                   (s.waves == 4 && s.rows == 4));
    if (s.tile_x != 64 && s.tile_x != 32) return false;
    if (s.waves == 4) return s.rows == 1 || s.rows == 2 || (s.rows == 4 && s.tile_x == 64);
    if (s.waves == 8) return (s.rows == 1 || s.rows == 2) && s.prefetch == 0;
    return false;
}

inline int tile_height(const StepShape& s) { return s.waves * s.rows * (64 / s.tile_x); }

// Shapes of the two-steps-per-pass kernel: tiles tile_x wide and 8 * rows high with one node of
// the second step per thread, i.e. waves = tile_x * 8 * rows / 64: 64 x 8 (rows 1, waves 8) or
// 32 x 16 (rows 2, waves 8), either prefetch setting, or 64 x 16 (rows 2, waves 16, prefetch 0).
inline bool step2_shape_supported(const StepShape& s)
{
    if (s.z_chunk < 1 || (s.xcd_remap & ~1) || (s.prefetch & ~1)) return false;
    return (s.tile_x == 64 && s.rows == 1 && s.waves == 8) ||
           (s.tile_x == 32 && s.rows == 2 && s.waves == 8) ||
           (s.tile_x == 32 && s.rows == 2 && s.waves == 4 && s.prefetch == 0) ||
           (s.tile_x == 64 && s.rows == 2 && s.waves == 16 && s.prefetch == 0);
}

// Interior rows of a full-row tile for row pitch px: the tile pulls by + 2 rows of px nodes into
// rows * 64 * waves thread slots, less up to 31 slots that align the lane window with the line
// grid when the pitch is not a whole number of 128-byte lines (packed rows; a line holds 32 FP32
// or 16 FP64 values, so 31 covers both). < 1: the rows are too long for full-row tiles.
inline int row_tile_rows(const StepShape& s, unsigned px)
{
    const unsigned slack = px % 32u ? 31u : 0u;
    return (int)((unsigned)(s.rows * 64 * s.waves - slack) / px) - 2;
}

// One box of a multi-box step.
struct GroupBox {
    BoxDesc b;
    const void* pop[2];     // the box's two population buffers
    int phase;              // pop[phase] holds the box's current state when the group's step
                            // counter is even
    int tiles_x, tiles_y, zc;
    int by;                 // full-row tiles: interior rows per tile
    unsigned item_begin;    // first work item of the box
    unsigned items;         // tiles_x * tiles_y * ceil(nz / zc)
};

// Empty slot of a group's item order.
constexpr unsigned NO_ITEM = 0xFFFFFFFFu;

// Work queues of the persistent multi-box kernel (device memory, zero-initialised once).
struct QueueState {
    unsigned next[8];       // next ticket of each XCD's queue
    unsigned done;          // workgroups finished in the current launch
    unsigned range[9];      // queue x serves items [range[x], range[x+1])
};

struct InitDesc {
    int geom;            // 0 droplet, 1 bubble, 2 slab
    int slab_axis;
    double radius;       // R (droplet/bubble) or half thickness (slab)
    double width;
    double n_in, n_out;
    double noise_amp;
    unsigned long long seed;
};

// Allocation-free multi-box step: the work list (at most NOALLOC_MAX_BOXES descriptors) and the
// persistent kernel's queue state live in one fixed device array per GPU, written by small
// stream-ordered kernels that take the descriptors as kernel arguments (no host staging, no
// device allocation).
constexpr int NOALLOC_MAX_BOXES = 1024;
constexpr int NOALLOC_BATCH = 16;     // descriptors per writing launch (kernel-argument size)
struct DescBatch {
    GroupBox d[NOALLOC_BATCH];
    int count;                        // descriptors used in d
    int first;                        // index of d[0] in the device work list
};
// Device address of the current device's array (looked up with hipGetSymbolAddress on the
// first call on each device and kept). Its first NOALLOC_MAX_BOXES * sizeof(GroupBox) bytes hold
// the work list, followed by the queue state at noalloc_queue_offset().
hipError_t noalloc_scratch_address(void** ptr);
constexpr size_t noalloc_queue_offset()
{
    return ((size_t)NOALLOC_MAX_BOXES * sizeof(GroupBox) + 255) / 256 * 256;
}
// Write a batch of descriptors / the queue state into the array at `scratch` (a device address
// returned by noalloc_scratch_address).
hipError_t launch_put_descs(const DescBatch& b, void* scratch, hipStream_t st);
hipError_t launch_put_queue(const QueueState& q, void* scratch, hipStream_t st);

// Number of per-block partial sums written by the observation reduction.
constexpr int OBS_PARTS = 14;
// Fixed grid of the observation reduction (deterministic order of the partial sums).
constexpr int OBS_BLOCKS = 512;

// One step of one box. fp32: populations stored as float (shifted); math64: with fp32, the step's
// arithmetic is done in double precision (storage and traffic unchanged).
// sbuf: index (0 or 1) of the source buffer, which selects the dither seed b.tick[sbuf].
hipError_t launch_step(bool fp32, bool math64, const BoxDesc& b, const StepShape& s, int sbuf,
                       const void* src, void* dst, hipStream_t st);
// The same per precision (step_f32.hip: FP32 storage and arithmetic; step_m64.hip: FP32 storage,
// FP64 arithmetic; step_f64.hip: FP64), called by launch_step / launch_step_group after the shape
// check.
#define LBM_STEP_DECL(tag)                                                                          \
    hipError_t launch_step_##tag(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,  \
                                 void* dst, hipStream_t st);                                       \
    hipError_t launch_group_##tag(const StepShape& s, const GroupBox* boxes, int nbox,             \
                                  unsigned nitems, int parity, int persistent, unsigned workers,   \
                                  QueueState* q, hipStream_t st);
LBM_STEP_DECL(f32)
LBM_STEP_DECL(m64)
LBM_STEP_DECL(f64)
#undef LBM_STEP_DECL
// Two time steps per pass for FP32 storage and arithmetic at tau = 1 (shape s, see
// step2_shape_supported): the state in src after t steps becomes the state in dst after t + 2.
hipError_t launch_step2_f32(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                            void* dst, hipStream_t st);
// The same over a group's work list (tiles tile_x wide and 8 * rows high, one workgroup per item):
// nitems workgroups taking items 0 .. nitems - 1, or, with an item order, 8 * per workgroups of
// which workgroup w takes order[(w mod 8) * per + w / 8] (NO_ITEM: none).
hipError_t launch_group2_f32(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                             const unsigned* order, unsigned per, int parity, hipStream_t st);
// Multi-box step. nitems work items; persistent: grid of `workers` workgroups over the queues.
hipError_t launch_step_group(bool fp32, bool math64, const StepShape& s, const GroupBox* boxes, int nbox,
                             unsigned nitems, int parity, int persistent, unsigned workers,
                             QueueState* q, hipStream_t st);
hipError_t launch_init(bool fp32, const BoxDesc& b, const InitDesc& d, double* dn, double* dpsi,
                       void* dst, hipStream_t st);
hipError_t launch_get(bool fp32, const BoxDesc& b, int i, const void* src, double* out,
                      hipStream_t st);
hipError_t launch_set(bool fp32, const BoxDesc& b, int i, const double* in, void* dst,
                      hipStream_t st);
// Observation: pull moments (dn, dpsi, dj: N, N and 3N doubles of workspace), then force,
// velocity and reductions; uprev (3N doubles, the box's own) holds the previous observation's
// velocity on entry and this one's on return.
hipError_t launch_observe(bool fp32, const BoxDesc& b, const void* src, double* dn, double* dpsi,
                          double* dj, double* uprev, int has_prev, double* parts,
                          double* scal, hipStream_t st);
hipError_t launch_profile_line(const BoxDesc& b, const double* dn, const double* dpsi,
                               double* prof, double* probes, hipStream_t st);
// lane_bytes: bytes each lane moves per access (4, 8 or 16).
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int lane_bytes,
                              hipStream_t st);
hipError_t launch_profile_planes(const BoxDesc& b, int axis, const double* dn, const double* dpsi,
                                 double* prof, double* probes, hipStream_t st);

}  // namespace lbm
