// Fused step kernels instantiated for FP32 storage and arithmetic.
#include "step_kernels.hpp"

namespace lbm {

hipError_t launch_step_f32(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                           void* dst, hipStream_t st)
{
    return launch_step_impl<float, float>(b, s, sbuf, src, dst, st);
}

// Two time steps per pass (FP32 storage and arithmetic, tau = 1): 64-wide tiles of rows x 8 rows
// worked by waves wave64s (rows 1 with waves 8, either prefetch setting; rows 2 with waves 16), z
// chunks of zc planes (clamped to nz).
template <int BY, int WAVES, bool PF>
hipError_t launch_step2_t(const BoxDesc& b, int zc, int remap, int sbuf, const void* src, void* dst,
                          hipStream_t st)
{
    StepArgs a;
    a.b = b;
    a.s = sbuf;
    a.by = 0;
    a.tiles_x = (b.nx + 63) / 64;
    a.tiles_y = (b.ny + BY - 1) / BY;
    a.zc = zc < b.nz ? zc : b.nz;
    if (a.zc < 1) return hipErrorInvalidValue;
    a.nchunks = (b.nz + a.zc - 1) / a.zc;
    a.remap = remap;
    const unsigned grid = (unsigned)(a.tiles_x * a.tiles_y * a.nchunks);
    if (b.psi == 0)
        hipLaunchKernelGGL((k_step2<0, BY, WAVES, PF>), dim3(grid), dim3(64 * WAVES), 0, st, a,
                           (const float*)src, (float*)dst);
    else
        hipLaunchKernelGGL((k_step2<1, BY, WAVES, PF>), dim3(grid), dim3(64 * WAVES), 0, st, a,
                           (const float*)src, (float*)dst);
    return hipGetLastError();
}

hipError_t launch_step2_f32(const BoxDesc& b, int rows, int waves, int prefetch, int zc, int remap,
                            int sbuf, const void* src, void* dst, hipStream_t st)
{
    if (rows == 1 && waves == 8)
        return prefetch ? launch_step2_t<8, 8, true>(b, zc, remap, sbuf, src, dst, st)
                        : launch_step2_t<8, 8, false>(b, zc, remap, sbuf, src, dst, st);
    if (rows == 2 && waves == 16 && !prefetch)
        return launch_step2_t<16, 16, false>(b, zc, remap, sbuf, src, dst, st);
    return hipErrorInvalidValue;
}

hipError_t launch_group_f32(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                            int parity, int persistent, unsigned workers, QueueState* q,
                            hipStream_t st)
{
    return launch_group_shape<float, float>(s, boxes, nbox, nitems, parity, persistent, workers, q, st);
}

}  // namespace lbm
