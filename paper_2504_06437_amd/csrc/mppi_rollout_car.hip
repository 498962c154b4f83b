// Rollout kernels of the car model (the standalone tile kernels and the
// batched persistent kernel), compiled in a unit of their own.
#include "mppi_device.hpp"

namespace dbas {

hipError_t launch_rollout_car(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    return launch_rollout_m<MPPI_CAR>(p, a, lds, s);
}

BatchRolloutKernel batch_rollout_kernel_car(int key)
{
    switch (key) {
    case 0: return k_batch_rollout_layout<MPPI_CAR, 16>;
    case 1: return k_batch_rollout_layout<MPPI_CAR, 32>;
    case 2: return k_batch_rollout_layout<MPPI_CAR, 64>;
    case 3: return k_batch_rollout_layout<MPPI_CAR, 128>;
    case 4: return k_batch_rollout_layout<MPPI_CAR, 256>;
    default: return k_batch_rollout<MPPI_CAR>;
    }
}

}  // namespace dbas
