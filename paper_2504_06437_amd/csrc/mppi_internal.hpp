// Internal structures of the DBaS-Log-MPPI HIP library, shared by its host
// runtime and its kernels (never by the CPU oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dbas_mppi.h"

namespace dbas {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)
constexpr int kWave = 64;
constexpr int kM = MPPI_M;
constexpr int kRowsPerBlock = kBlock / kWave;   // update kernel: one wave per control row

// Mutable per-controller state, resident in device memory.
struct CtrlState {
    uint64_t counter;        // Philox step counter of the next iteration
    uint64_t last_counter;   // counter used by the last iteration
    double rho, eta;         // last iteration's min cost and normaliser
    double cshift;           // last iteration's common barrier-state cost (every S_k includes it)
    float S_e;               // exploration rate
    int32_t status;          // status of the last iteration
    float beta0, beta_d;     // fused barrier at x0 and at x_d
    uint32_t tiles_done;     // completion ticket of the running iteration
    uint32_t iter;           // iterations run; U[iter & 1] is the warm start
    int32_t fp64_tiles;      // tiles of the last iteration whose weights ran in FP64
    int32_t pad;
};

// Written by the update kernel into pinned host memory.
struct HostResult {
    float u0[kM];
    int32_t status;
    int32_t pad;
    uint64_t counter;
};

// Everything a kernel needs to run one controller's iteration.  Passed by
// value to the single-controller kernels, held in an array for the batch.
struct DevParams {
    int32_t model, K, Kp, T, P, J, G, spt, tiles, n;
    int32_t normaliser, init_mode;
    float dt, mass, gravity, arm, inertia, wheelbase;
    float u_min[kM], u_max[kM], sigma[kM];
    float mu_ln, sigma_ln, lambda, gamma_u, gamma_b, r_b, h_eps;
    float Q[MPPI_NMAX], Qf[MPPI_NMAX];
    float shape[MPPI_PMAX][2];
    uint32_t seed_lo, seed_hi;
    int32_t map_w, map_h;
    float map_x0, map_y0, map_res;
    int32_t pad;
    const float* obs;        // [J][3] cx, cy, r (world frame)
    const float* sdf;        // [map_h][map_w] or null
    const float* xref;       // [T+1][n] world frame
    float* U;                // [2][T][2] warm start, double-buffered by iteration parity
    float* Ustar;            // [T][2] optimal sequence of the last iteration (before the shift)
    float* du;               // [T][2][Kp] noise
    float* S;                // [2][Kp] compensated cost: hi at [k], lo at [Kp + k]
    float* e;                // [Kp] tile-local exponentials exp(-(S_k - rho_tile)/lambda)
    double* rho_b;           // [tiles] tile minimum cost
    double* eta_b;           // [tiles] tile sum of exponentials
    double* f_b;             // [tiles] exp(-(rho_b - rho)/lambda)
    int32_t* flag_b;         // [tiles] 1 when the tile ran its weights in FP64
    double* partN;           // [2T][tiles] tile sums of e_k du[t][c][k]
    CtrlState* st;
    HostResult* res;         // device-visible pointer to pinned host memory (may be null)
};

// Per-launch arguments of the single-controller kernels.
struct StepArgs {
    float x0[MPPI_NMAX + 2];
    const float* x0_ptr;     // device x0 (overrides x0[] when non-null)
    float* u0_dev;           // optional device u0 output
};

// One unit of the batched rollout: sample tile `tile` of controller `ctrl`.
struct BatchUnit {
    int32_t ctrl;
    int32_t tile;
};

// One unit of the batched update: control rows [row0, row0 + 4) of `ctrl`.
struct RowUnit {
    int32_t ctrl;
    int32_t row0;
};

inline int state_dim(int model) { return model == MPPI_QUAD6 ? 6 : model == MPPI_QUAD5 ? 5 : 4; }

// Dynamic LDS bytes one rollout tile of this controller needs.
inline size_t tile_lds_bytes(int J, int T, int n)
{
    size_t b = 0;
    b += (size_t)(J > 0 ? J : 1) * 16;          // obstacles, local frame
    b += (size_t)T * 8;                         // U
    b += (size_t)(T + 1) * n * 4;               // reference, local frame
    b = (b + 15) & ~(size_t)15;
    b += (size_t)kBlock * 8;                    // tile exponentials
    b += 16 * 8;                                // block-reduction slots
    return b;
}

// Kernel launchers (mppi_kernels.hip).
hipError_t launch_rollout(const DevParams& p, const StepArgs& a, hipStream_t s);
hipError_t launch_update(const DevParams& p, const StepArgs& a, hipStream_t s);
hipError_t launch_batch_rollout(const DevParams* d_params, const BatchUnit* d_units, int nunits,
                                const float* d_x0s, uint32_t* d_queue, int grid, size_t lds,
                                hipStream_t s);
hipError_t launch_batch_update(const DevParams* d_params, const RowUnit* d_units, int nunits,
                               float* d_u0s, hipStream_t s);
hipError_t launch_weights(const DevParams& p, double* d_w, hipStream_t s);
hipError_t launch_philox_words(const DevParams& p, uint64_t counter, uint32_t* d_words, hipStream_t s);
int batch_rollout_blocks_per_cu(size_t lds);
bool tile_lanes_supported(int G);

}  // namespace dbas
