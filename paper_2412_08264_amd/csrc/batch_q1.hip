// Batched residual, apply and fused-step kernels, and the stand-alone Hessian-vector product, on tiles of
// 32 x 8 pixels.
#include "batch_tile.h"

namespace bl {

template hipError_t launch_b_residual_q<1>(const Stencil&, bool, const Slot*, const BatchMap&, int, hipStream_t);
template hipError_t launch_b_apply_q<1>(const Stencil&, bool, bool, const Slot*, const BatchMap&, StepRef,
                                             hipStream_t);
template hipError_t launch_f_step_q<1>(const Stencil&, bool, const Slot*, const BatchMap&, StepRef, const Slot*,
                                       hipStream_t);
template hipError_t launch_hvp_q<1>(const Stencil&, bool, const double*, const double*, double*, int,
                                          hipStream_t);

}  // namespace bl
