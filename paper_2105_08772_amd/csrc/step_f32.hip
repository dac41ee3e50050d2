// Fused step kernels instantiated for FP32 storage and arithmetic.
#include "step_kernels.hpp"

namespace lbm {

hipError_t launch_step_f32(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                           void* dst, hipStream_t st)
{
    return launch_step_impl<float, float>(b, s, sbuf, src, dst, st);
}

// Two time steps per pass (FP32 storage and arithmetic, tau = 1): tiles tile_x wide and 8 * rows
// high, worked by tile_x * 8 * rows / 64 waves (one node of the second step per thread): 64 x 8
// with 8 waves or 32 x 16 with 8 waves, either prefetch setting, or 64 x 16 with 16 waves; z
// chunks of zc planes (clamped to nz).
template <int BX, int BY, int WAVES, bool PF, int MINW = 1>
hipError_t launch_step2_t(const BoxDesc& b, int zc, int remap, int sbuf, const void* src, void* dst,
                          hipStream_t st)
{
    StepArgs a;
    a.b = b;
    a.s = sbuf;
    a.by = 0;
    a.tiles_x = (b.nx + BX - 1) / BX;
    a.tiles_y = (b.ny + BY - 1) / BY;
    a.zc = zc < b.nz ? zc : b.nz;
    if (a.zc < 1) return hipErrorInvalidValue;
    a.nchunks = (b.nz + a.zc - 1) / a.zc;
    a.remap = remap;
    const unsigned grid = (unsigned)(a.tiles_x * a.tiles_y * a.nchunks);
    if (b.psi == 0)
        hipLaunchKernelGGL((k_step2<0, BX, BY, WAVES, PF, MINW>), dim3(grid), dim3(64 * WAVES), 0, st, a,
                           (const float*)src, (float*)dst);
    else
        hipLaunchKernelGGL((k_step2<1, BX, BY, WAVES, PF, MINW>), dim3(grid), dim3(64 * WAVES), 0, st, a,
                           (const float*)src, (float*)dst);
    return hipGetLastError();
}

hipError_t launch_step2_f32(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                            void* dst, hipStream_t st)
{
    const int zc = s.z_chunk, remap = s.xcd_remap;
    if (s.tile_x == 64 && s.rows == 1 && s.waves == 8)
        return s.prefetch ? launch_step2_t<64, 8, 8, true>(b, zc, remap, sbuf, src, dst, st)
                          : launch_step2_t<64, 8, 8, false>(b, zc, remap, sbuf, src, dst, st);
    if (s.tile_x == 32 && s.rows == 2 && s.waves == 8)
        return s.prefetch ? launch_step2_t<32, 16, 8, true>(b, zc, remap, sbuf, src, dst, st)
                          : launch_step2_t<32, 16, 8, false, 4>(b, zc, remap, sbuf, src, dst, st);
    if (s.tile_x == 32 && s.rows == 2 && s.waves == 4 && !s.prefetch)
        return launch_step2_t<32, 16, 4, false, 2>(b, zc, remap, sbuf, src, dst, st);
    if (s.tile_x == 64 && s.rows == 2 && s.waves == 16 && !s.prefetch)
        return launch_step2_t<64, 16, 16, false>(b, zc, remap, sbuf, src, dst, st);
    return hipErrorInvalidValue;
}

template <int BX, int BY, int WAVES, bool PF, int MINW = 1>
hipError_t launch_group2_t(const GroupBox* boxes, int nbox, unsigned nitems, const unsigned* order,
                           unsigned per, int parity, hipStream_t st)
{
    const unsigned grid = order ? 8u * per : nitems;
    hipLaunchKernelGGL((k_step2_group<BX, BY, WAVES, PF, MINW>), dim3(grid), dim3(64 * WAVES), 0, st,
                       boxes, nbox, parity, order, per);
    return hipGetLastError();
}

// Two steps per pass over a group: the shapes of launch_step2_f32, one workgroup per work item
// (the work list built for tiles tile_x wide and 8 * rows high).
hipError_t launch_group2_f32(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                             const unsigned* order, unsigned per, int parity, hipStream_t st)
{
#define LBM_G2(BX, BY, WV, PF, ...) \
    launch_group2_t<BX, BY, WV, PF, ##__VA_ARGS__>(boxes, nbox, nitems, order, per, parity, st)
    if (s.tile_x == 64 && s.rows == 1 && s.waves == 8)
        return s.prefetch ? LBM_G2(64, 8, 8, true) : LBM_G2(64, 8, 8, false);
    if (s.tile_x == 32 && s.rows == 2 && s.waves == 8)
        return s.prefetch ? LBM_G2(32, 16, 8, true) : LBM_G2(32, 16, 8, false, 4);
    if (s.tile_x == 32 && s.rows == 2 && s.waves == 4 && !s.prefetch) return LBM_G2(32, 16, 4, false, 2);
    if (s.tile_x == 64 && s.rows == 2 && s.waves == 16 && !s.prefetch) return LBM_G2(64, 16, 16, false);
    return hipErrorInvalidValue;
#undef LBM_G2
}

hipError_t launch_group_f32(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                            int parity, int persistent, unsigned workers, QueueState* q,
                            hipStream_t st)
{
    return launch_group_shape<float, float>(s, boxes, nbox, nitems, parity, persistent, workers, q, st);
}

}  // namespace lbm
