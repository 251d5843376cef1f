// 3D adjoint step kernels (every adjoint mode) and their batched form.
#include "step_kernels.h"

namespace stride {

void launch_family_3d_adj(int R, int mode, const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                          const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    R == 4 ? launch_mode_r<true, true, 4>(mode, d, cf, sp, ls, p, s)
           : launch_mode_r<true, true, 5>(mode, d, cf, sp, ls, p, s);
}

void launch_batched_3d_adj(int R, int mode, const Dims& d, const StencilCoef& cf,
                           const LaunchShape& ls, const SlotStep* table, int nslots, int max_samples,
                           hipStream_t s)
{
    R == 4 ? batched_mode_r<true, true, 4>(mode, d, cf, ls, table, nslots, max_samples, s)
           : batched_mode_r<true, true, 5>(mode, d, cf, ls, table, nslots, max_samples, s);
}

}  // namespace stride
