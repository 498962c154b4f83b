// Rollout kernels of the quad5 model (the standalone tile kernels and the
// batched persistent kernels), compiled in a unit of their own.
#include "mppi_device.hpp"

namespace dbas {

hipError_t launch_rollout_quad5(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    return launch_rollout_m<MPPI_QUAD5>(p, a, lds, s);
}

BatchRolloutKernel batch_rollout_kernel_quad5(int key) { return batch_kernel_of<MPPI_QUAD5>(key); }

}  // namespace dbas
