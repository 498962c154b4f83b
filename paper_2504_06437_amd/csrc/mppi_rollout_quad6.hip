// Rollout kernels of the quad6 model (the standalone tile kernels and the
// batched persistent kernel), compiled in a unit of their own.
#include "mppi_device.hpp"

namespace dbas {

hipError_t launch_rollout_quad6(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    return launch_rollout_m<MPPI_QUAD6>(p, a, lds, s);
}

BatchRolloutKernel batch_rollout_kernel_quad6(int key)
{
    switch (key) {
    case 0: return k_batch_rollout_layout<MPPI_QUAD6, 16>;
    case 1: return k_batch_rollout_layout<MPPI_QUAD6, 32>;
    case 2: return k_batch_rollout_layout<MPPI_QUAD6, 64>;
    case 3: return k_batch_rollout_layout<MPPI_QUAD6, 128>;
    case 4: return k_batch_rollout_layout<MPPI_QUAD6, 256>;
    default: return k_batch_rollout<MPPI_QUAD6>;
    }
}

}  // namespace dbas
