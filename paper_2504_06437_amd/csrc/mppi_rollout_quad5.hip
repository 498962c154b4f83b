// Rollout kernels of the quad5 model (the standalone tile kernels and the
// batched persistent kernel), compiled in a unit of their own.
#include "mppi_device.hpp"

namespace dbas {

hipError_t launch_rollout_quad5(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    return launch_rollout_m<MPPI_QUAD5>(p, a, lds, s);
}

BatchRolloutKernel batch_rollout_kernel_quad5(int key)
{
    switch (key) {
    case 0: return k_batch_rollout_layout<MPPI_QUAD5, 16>;
    case 1: return k_batch_rollout_layout<MPPI_QUAD5, 32>;
    case 2: return k_batch_rollout_layout<MPPI_QUAD5, 64>;
    case 3: return k_batch_rollout_layout<MPPI_QUAD5, 128>;
    case 4: return k_batch_rollout_layout<MPPI_QUAD5, 256>;
    default: return k_batch_rollout<MPPI_QUAD5>;
    }
}

}  // namespace dbas
