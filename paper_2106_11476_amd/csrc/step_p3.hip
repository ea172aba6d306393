// 3D pressure-phase kernels of the time step, instantiated for every mechanism count,
// memory scheme, stencil mode and kernel variant.
#include "step_kernels.hpp"

namespace fw2 {

hipError_t launch_pressure_3d(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    return dispatch_L<true, 3>(a, L, scheme, kc, st);
}

}  // namespace fw2
