// Fused step kernels instantiated for FP32 storage, FP64 arithmetic.
#include "step_kernels.hpp"

namespace lbm {

hipError_t launch_step_m64(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                           void* dst, hipStream_t st)
{
    return launch_step_impl<float, double>(b, s, sbuf, src, dst, st);
}

hipError_t launch_group_m64(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                            int parity, int persistent, unsigned workers, QueueState* q,
                            hipStream_t st)
{
    return launch_group_shape<float, double>(s, boxes, nbox, nitems, parity, persistent, workers, q, st);
}

}  // namespace lbm
