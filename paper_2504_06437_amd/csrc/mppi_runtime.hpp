// Host-side handle of one controller (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "mppi_internal.hpp"

struct mppi_ctrl {
    mppi_config cfg{};
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    bool tiles_fixed = false;
    bool external_scratch = false;   // sample buffers supplied per launch by the owner
    uint64_t version = 0;            // bumps whenever DevParams change (batches re-upload)
    uint32_t iter = 0;               // iterations launched; U[iter & 1] holds the warm start
    std::string err;
    dbas::DevParams p{};
    std::vector<void*> allocations;
    float* d_obs = nullptr;
    int obs_cap = 0;
    float* d_sdf = nullptr;
    size_t sdf_bytes = 0;
    float4* d_sdf4 = nullptr;        // four-texel records of the costmap
    size_t sdf4_bytes = 0;
    dbas::HostResult* h_res = nullptr;
    // kernel timing (mppi_profile_*): event triples per recorded iteration
    bool profiling = false;
    int prof_every = 1;                    // record every n-th iteration
    int64_t prof_seen = 0;                 // iterations since profiling was turned on
    std::vector<hipEvent_t> prof_events;   // 3 per slot
    int prof_used = 0;
    int64_t prof_dropped = 0;

    ~mppi_ctrl();
    int fail(int status, const char* fmt, ...);
    int hip_fail(hipError_t e, const char* what);
    void* dalloc(size_t bytes, int* status);
    int sync();
    int read_state(dbas::CtrlState* out);
    int write_state_field(size_t offset, const void* src, size_t bytes);
    int configure_tiles(int S);
    int alloc_tile_buffers();
    int retile();
    int launch_step(const float* x0_host, const float* x0_dev, float* u0_dev, bool mark = false);
};

namespace dbas {
std::string validate_config(const mppi_config* c);
void params_from_config(const mppi_config* cfg, DevParams& p);
int heuristic_tile_samples(int K, int J, int T, int n, int sgf_m);
bool any_tile_fits(int K, int J, int T, int n, int sgf_m);
// Samples per tile for this controller's (model, K, T, J, P, costmap,
// smoothing); 0 when no tile shape fits.
int choose_tile_samples(mppi_ctrl* h);
int create_ctrl(const mppi_config* cfg, const mppi_device* dev, bool external_scratch, mppi_ctrl** out);
}  // namespace dbas

void set_global_error(const std::string& s);
const char* global_error();
