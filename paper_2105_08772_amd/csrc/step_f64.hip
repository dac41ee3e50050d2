// Fused step kernels instantiated for FP64 storage and arithmetic.
#include "step_kernels.hpp"

namespace lbm {

hipError_t launch_step_f64(const BoxDesc& b, const StepShape& s, int sbuf, const void* src,
                           void* dst, hipStream_t st)
{
    return launch_step_impl<double, double>(b, s, sbuf, src, dst, st);
}

hipError_t launch_group_f64(const StepShape& s, const GroupBox* boxes, int nbox, unsigned nitems,
                            int parity, int persistent, unsigned workers, QueueState* q,
                            hipStream_t st)
{
    return launch_group_shape<double, double>(s, boxes, nbox, nitems, parity, persistent, workers, q, st);
}

}  // namespace lbm
