// Serving layer (placeholder until the scheduler lands).
#include <hip/hip_runtime.h>

#include "mppi_internal.hpp"
#include "mppi_runtime.hpp"

struct mppi_server {
    int dummy;
};

extern "C" int mppi_server_create(const mppi_server_config*, mppi_server_t** out)
{
    if (out) *out = nullptr;
    set_global_error("mppi_server_create: serving is not built yet");
    return MPPI_E_INVALID;
}
extern "C" void mppi_server_destroy(mppi_server_t*) {}
extern "C" int mppi_server_add_robot(mppi_server_t*, const mppi_config*, int32_t, const float*, int32_t*) { return MPPI_E_INVALID; }
extern "C" int mppi_server_submit(mppi_server_t*, int32_t, const float*, const float*, double, int64_t*) { return MPPI_E_INVALID; }
extern "C" int mppi_server_poll(mppi_server_t*, int64_t, float*, double*, int32_t*) { return MPPI_E_INVALID; }
extern "C" int mppi_server_wait(mppi_server_t*, int64_t, float*, double*, int32_t*) { return MPPI_E_INVALID; }
extern "C" double mppi_server_now(const mppi_server_t*) { return 0.0; }
extern "C" int mppi_server_get_stats(mppi_server_t*, mppi_server_stats*) { return MPPI_E_INVALID; }
extern "C" int mppi_server_get_robot(mppi_server_t*, int32_t, float*, uint64_t*) { return MPPI_E_INVALID; }
extern "C" const char* mppi_server_last_error(const mppi_server_t*) { return global_error(); }
