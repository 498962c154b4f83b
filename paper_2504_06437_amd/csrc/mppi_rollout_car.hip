// Rollout kernels of the car model (the standalone tile kernels and the
// batched persistent kernels), compiled in a unit of their own.
#include "mppi_device.hpp"

namespace dbas {

hipError_t launch_rollout_car(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    return launch_rollout_m<MPPI_CAR>(p, a, lds, s);
}

BatchRolloutKernel batch_rollout_kernel_car(int key) { return batch_kernel_of<MPPI_CAR>(key); }

}  // namespace dbas
