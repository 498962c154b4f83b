// Internal structures of the DBaS-Log-MPPI HIP library, shared by its host
// runtime and its kernels (never by the CPU oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/dbas_mppi.h"

namespace dbas {

constexpr int kWave = 64;
constexpr int kRollBlock = 1024;     // rollout workgroup: 16 wave64s, one tile of S samples
constexpr int kUpdBlock = 256;       // update workgroup: 4 wave64s, one control row each
constexpr int kMaxTiles = 4096;      // most sample tiles per controller
constexpr int kMaxTile = 256;        // largest S
constexpr int kM = MPPI_M;

// Mutable per-controller state, resident in device memory.
struct CtrlState {
    uint64_t counter;        // Philox step counter of the next iteration
    uint64_t last_counter;   // counter used by the last iteration
    double rho, eta;         // last iteration's min cost and normaliser
    double cshift;           // last iteration's common barrier-state cost (every S_k includes it)
    float S_e;               // exploration rate
    int32_t status;          // status of the last iteration
    float beta0, beta_d;     // fused barrier at x0 and at x_d
    float cost_b;            // C_B of the last U* (adaptive exploration)
    uint32_t iter;           // iterations run (the host tracks the same count)
    int32_t fp64_tiles;      // tiles of the last iteration whose weights ran in FP64
    int32_t pad;
};

// Written by the update kernel into pinned host memory.  When the launch asks
// for it (StepArgs::mark), seq (the number of iterations completed) is
// written last, after system-scope fences, so a host thread that sees it
// change may read u0 and status.
struct HostResult {
    float u0[kM];
    int32_t status;
    int32_t pad;
    uint64_t counter;
    uint64_t seq;
};

// Everything a kernel needs to run one controller's iteration.  Passed by
// value to the single-controller kernels, held in an array for the batch.
struct DevParams {
    int32_t model, K, Kp, T, P, J, spt, tiles, n;   // spt: samples per tile (S)
    int32_t normaliser, init_mode;
    float dt, mass, gravity, arm, inertia, wheelbase;
    float u_min[kM], u_max[kM], sigma[kM];
    float mu_ln, sigma_ln, lambda, gamma_u, gamma_b, r_b, h_eps;
    float Q[MPPI_NMAX], Qf[MPPI_NMAX];
    float shape[MPPI_PMAX][2];
    uint32_t seed_lo, seed_hi;
    int32_t map_w, map_h;
    float map_x0, map_y0, map_res;
    int32_t export_noise;    // 1: the rollout also stores the noise into du
    int32_t adaptive;        // 1: S_e follows the barrier cost of U*
    float explore_mu;
    int32_t sgf_m;           // Savitzky-Golay half window (0: no smoothing)
    int32_t sampling;        // MPPI_SAMPLE_NLN or MPPI_SAMPLE_NORMAL (the normal part alone)
    int32_t cost_mode;       // MPPI_COST_DBAS or MPPI_COST_INDICATOR (no barrier state)
    float collision_weight;  // weight of the collision indicator
    int32_t shape_kind;      // ShapeForm: the layout form the model's fixed-P tile may use
    int32_t lg_pack;         // the rollout's barrier splits (tile_lg_pack | kLgPackSet), or 0:
                             //   the kernel forms them itself
    double beta_d_weight;    // R_B sum_{t=1..T} c_t / beta_d, the common barrier-state cost per unit of beta_d
    const float* sgf_coef;   // [T][2m+1] smoothing weights of step t over its window
    const float* obs;        // [J][3] cx, cy, r (world frame)
    const float* sdf;        // [map_h][map_w] or null
    const float4* sdf4;      // [map_h-1][map_w-1] four-texel records of sdf (null: read sdf itself)
    const float* xref;       // [T+1][n] world frame
    float* U;                // [2][T][2] warm start, double-buffered by iteration parity
    float* Unext;            // [T][2] where the update writes the shifted warm start instead of the
                             //   other half of U (null: the other half; the handle-free entry point)
    float* Ustar;            // [T][2] optimal sequence of the last iteration (before the shift)
    float* du;               // [T][2][Kp] noise (only with export_noise)
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
    uint32_t parity;         // iterations run & 1: the half of U that holds the warm start
    uint32_t mark;           // 1: publish u0, status and the completion mark to the host
                             //    at once (system-scope fences), for a host thread spinning
    int32_t* status_dev;     // optional device copy of the iteration's status
};

// Per-step input of one controller of a batch (staged by the host).
struct BatchIn {
    float x0[MPPI_NMAX + 2];
    uint32_t parity;
    uint32_t pad[3];
};

// One unit of the batched update: control rows [row0, row0 + 4) of `ctrl`.
struct RowUnit {
    int32_t ctrl;
    int32_t row0;
};

// One unit of the batched rollout: sample tile `tile` of controller `ctrl`.
struct BatchUnit {
    int32_t ctrl;
    int32_t tile;
};

constexpr int kModels = 3;          // MPPI_QUAD6, MPPI_QUAD5, MPPI_CAR

// Kernels of the batched rollout, per model: one persistent kernel per tile
// size and tile kind, each holding the one tile the standalone kernel of that
// shape holds (a kernel holding many tiles has the registers of the largest
// and spills).  Kinds: the layout form of the paper's bodies, the runtime-P
// form and the indicator tile, each without and with a costmap.
constexpr int kTileSizes = 5;       // S = 16, 32, 64, 128, 256
constexpr int kTileKinds = 6;
constexpr int kBatchKeys = kTileSizes * kTileKinds;
constexpr int kBatchGroups = kModels * kBatchKeys;

// The rollout units of a batched launch, grouped by kernel: one persistent
// launch per group present.  Group g (model g / kBatchKeys, kernel
// g % kBatchKeys) is units [begin[g], begin[g] + count[g]) of the list,
// longest first; lds[g] is the dynamic LDS its kernel needs and
// work[g] the sum of its units' estimates.  The queue of group g is words
// 2g and 2g + 1.
struct UnitGroups {
    int begin[kBatchGroups];
    int count[kBatchGroups];
    size_t lds[kBatchGroups];
    double work[kBatchGroups];
};

// A rollout unit before grouping, with its group, its estimated work and the
// dynamic LDS of its tile.
struct BatchWork {
    double cost;
    int32_t group;
    size_t lds;
    BatchUnit unit;
};

// Per-tile work estimate for longest-first ordering: samples x steps x
// (pairs + a fixed part).
inline double tile_cost(int S, int K, int T, int P, int J)
{
    return (double)(S < K ? S : K) * T * ((double)P * J + 64.0);
}

// Sort `work` by model, then longest first (stable), write the units to `out`
// and return the groups.
UnitGroups group_units(std::vector<BatchWork>& work, BatchUnit* out);

// Shape points of the model's compile-time tile (the paper's bodies): 8 for
// the vehicle, 7 for the quadrotors.
constexpr int fixed_points(int model) { return model == MPPI_CAR ? 8 : 7; }

// Which layout form of the fixed-P tile the shape allows (0: none; the
// runtime-P tile's general form is used).  Vehicle, 1: the corners and side
// midpoints of a rectangle centred on the reference point, in the order
// (a, b), (a, -b), (-a, b), (-a, -b), (a, 0), (-a, 0), (0, b), (0, -b).
// Quadrotors, 1: every point on the body axis (b = 0); 2: moreover points
// 0, 1, 2 are the mirror images of points 6, 5, 4 (a_i = -a_{6-i}) and point
// 0 lies farthest from the centre (|a_0| >= |a_i|).
enum ShapeForm : int32_t { kShapeGeneral = 0, kShapeLayout = 1, kShapeMirroredAxis = 2 };

inline int32_t shape_form(int model, int P, const float (*sh)[2])
{
    if (P != fixed_points(model)) return kShapeGeneral;
    if (model == MPPI_CAR) {
        const float a = sh[0][0], b = sh[0][1];
        const float want[8][2] = {{a, b}, {a, -b}, {-a, b}, {-a, -b}, {a, 0.0f}, {-a, 0.0f}, {0.0f, b}, {0.0f, -b}};
        for (int i = 0; i < 8; ++i)
            if (sh[i][0] != want[i][0] || sh[i][1] != want[i][1]) return kShapeGeneral;
        return kShapeLayout;
    }
    for (int i = 0; i < P; ++i)
        if (sh[i][1] != 0.0f) return kShapeGeneral;
    for (int i = 0; i < 3; ++i)
        if (sh[i][0] != -sh[6 - i][0]) return kShapeLayout;
    const float a0 = sh[0][0] < 0.0f ? -sh[0][0] : sh[0][0];
    for (int i = 1; i < 4; ++i)
        if ((sh[i][0] < 0.0f ? -sh[i][0] : sh[i][0]) > a0) return kShapeLayout;
    return kShapeMirroredAxis;
}

inline int state_dim(int model) { return model == MPPI_QUAD6 ? 6 : model == MPPI_QUAD5 ? 5 : 4; }

// LDS obstacle slots (at least one, so the carve-up never has a zero-size array).
__host__ __device__ inline int obstacle_slots(int J) { return J > 0 ? J : 1; }

constexpr size_t kLdsLimit = 65536;     // dynamic LDS budget of one rollout workgroup
constexpr int kChunkSlotsMax = 2048;    // most (step, sample) slots in one horizon chunk

// Per (step, sample) slot, double-buffered: inputs (float4), pose (float4),
// fused barrier (float).
constexpr int kSlotBytes = 2 * (16 + 16 + 4);
// Each chunk buffer holds two slots beyond its (step, sample) items: chunk 0
// carries the poses of x0 and x_d = x_ref[T] there, whose fused barriers are
// beta_0 and beta_d.
constexpr int kXSlots = 2;

// LDS bytes of a rollout tile apart from the chunk slots.
__host__ __device__ inline size_t tile_fixed_lds(int J, int T, int n)
{
    size_t b = 0;
    b += (size_t)obstacle_slots(J) * 16;        // obstacles, local frame
    b += (size_t)T * 8;                         // U
    b += (size_t)(T + 1) * n * 4;               // reference, local frame
    b = (b + 15) & ~(size_t)15;
    b += (size_t)kMaxTile * 8;                  // tile exponentials
    b += 16 * 8;                                // block-reduction slots
    b += 64;                                    // pool waves per SIMD, owner SIMD, the largest |o|^2
    b += (size_t)kXSlots * kSlotBytes;          // two extra slots per chunk buffer (x0, x_d)
    return b;
}

// First chunk of the rollout pipeline: about a tenth of the horizon.
__host__ __device__ inline int tile_first_chunk(int T) { return (T + 9) / 10; }

// Steps per horizon chunk of the rollout pipeline after the first: a third
// of the rest of the horizon, within the LDS budget and kChunkSlotsMax.
// 0 when even one step does not fit (such a configuration is rejected).
__host__ __device__ inline int tile_chunk_steps(int J, int T, int n, int S)
{
    const size_t fixed = tile_fixed_lds(J, T, n);
    if (fixed + (size_t)S * kSlotBytes > kLdsLimit) return 0;
    long fit = (long)((kLdsLimit - fixed) / ((size_t)S * kSlotBytes));
    if (fit > kChunkSlotsMax / S) fit = kChunkSlotsMax / S;
    long tc = (T - tile_first_chunk(T) + 2) / 3;
    if (tc > fit) tc = fit;
    if (tc < 1) tc = 1;
    return (int)tc;
}

// Split of the fused-barrier items of a chunk of `items` (step, sample)
// items over nsp = 2^lg lanes each, for a tile whose first DW waves own its
// samples: among the splits that give every wave of the noise pool a unit,
// the one whose units, spread over the CU's four SIMDs, cost least:
// ceil(units / 4) units, each of ceil(J / nsp) obstacles x P pairs plus a
// fixed part (pose, shape transform, reduction: about 8 pairs' worth).
// Without such a split, the finest.
__host__ __device__ inline int tile_split_lg(int items, int J, int P, int DW)
{
    int lg = 0;
    long best = -1;
    for (int l = 0; l <= 6 && (1 << l) <= (J > 1 ? J : 1); ++l) {
        const long units = ((long)items * (1L << l) + kWave - 1) / kWave;
        if (units < kRollBlock / kWave - DW) {
            if (best < 0) lg = l;                        // the finest so far
            continue;
        }
        const long per_lane = (J + (1 << l) - 1) >> l;
        const long cost = (units + 3) / 4 * (per_lane * P + 8);
        if (best < 0 || cost < best) {
            best = cost;
            lg = l;
        }
    }
    return lg;
}

constexpr int kLgPackSet = 1 << 12;

// The splits of a tile's chunks, which have at most three lengths (the
// first, the middle ones, the last), packed 4 bits each, with kLgPackSet.
__host__ __device__ inline int tile_lg_pack(int J, int T, int n, int S, int P)
{
    const int tc = tile_chunk_steps(J, T, n, S);
    if (tc == 0) return kLgPackSet;
    const int tc0 = tile_first_chunk(T) < tc ? tile_first_chunk(T) : tc;
    const int nch = 1 + (T - tc0 + tc - 1) / tc;
    const int DW = (S + kWave - 1) / kWave;
    const int last = nch == 1 ? tc0 : T - (tc0 + (nch - 2) * tc);
    return kLgPackSet | tile_split_lg(tc0 * S, J, P, DW) | (nch > 2 ? tile_split_lg(tc * S, J, P, DW) << 4 : 0) |
           (nch > 1 ? tile_split_lg(last * S, J, P, DW) << 8 : 0);
}

// Does a tile of S samples fit the rollout's LDS budget: at least one horizon
// step per chunk and, with Savitzky-Golay smoothing (sgf_m > 0), room for the
// 2T FP64 update sums that the tile smooths in the space of its spent chunk
// inputs (two buffers of tc x S float4)?  Every place that picks or accepts a
// tile shape asks this one question.
__host__ __device__ inline bool tile_fits(int J, int T, int n, int S, int sgf_m)
{
    const int tc = tile_chunk_steps(J, T, n, S);
    if (tc == 0) return false;
    return sgf_m <= 0 || (size_t)2 * T * 8 <= (size_t)2 * tc * S * 16;
}

// Does the tile keep its whole noise (T x S float2) in LDS for the epilogue,
// or draw it again there?
__host__ __device__ inline bool tile_keeps_noise(int J, int T, int n, int S)
{
    return tile_fixed_lds(J, T, n) + (size_t)tile_chunk_steps(J, T, n, S) * S * kSlotBytes + (size_t)T * S * 8 <=
           kLdsLimit;
}

// Dynamic LDS bytes of the adaptive-exploration kernel: obstacles, the T+1
// poses of the U* rollout, their fused barriers.
inline size_t explore_lds_bytes(int J, int T)
{
    return (size_t)obstacle_slots(J) * 16 + (size_t)(T + 1) * 16 + (size_t)(T + 1) * 4;
}

// Dynamic LDS bytes one rollout tile of this controller needs.
inline size_t tile_lds_bytes(int J, int T, int n, int S)
{
    return tile_fixed_lds(J, T, n) + (size_t)tile_chunk_steps(J, T, n, S) * S * kSlotBytes +
           (tile_keeps_noise(J, T, n, S) ? (size_t)T * S * 8 : 0);
}

// Kernel launchers (mppi_kernels.hip).  The rollout kernels of each model
// live in their own unit (mppi_rollout_<model>.hip).
using BatchRolloutKernel = void (*)(const DevParams*, const BatchUnit*, int, const BatchIn*, uint32_t*);
// The batched rollout kernel of `key` (kind key / kTileSizes, tile size
// 16 << key % kTileSizes) of each model.
hipError_t launch_rollout_quad6(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s);
hipError_t launch_rollout_quad5(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s);
hipError_t launch_rollout_car(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s);
BatchRolloutKernel batch_rollout_kernel_quad6(int key);
BatchRolloutKernel batch_rollout_kernel_quad5(int key);
BatchRolloutKernel batch_rollout_kernel_car(int key);
hipError_t launch_rollout(const DevParams& p, const StepArgs& a, hipStream_t s);
hipError_t launch_update(const DevParams& p, const StepArgs& a, hipStream_t s);
// One persistent rollout launch per group, in order of decreasing work, each
// over min(units, cus x resident blocks) workgroups.
hipError_t launch_batch_rollouts(const DevParams* d_params, const BatchUnit* d_units, const UnitGroups& g,
                                 const BatchIn* d_in, uint32_t* d_queue, int cus, hipStream_t s);
hipError_t launch_batch_update(const DevParams* d_params, const RowUnit* d_units, int nunits, const BatchIn* d_in,
                               float* d_u0s, hipStream_t s);
hipError_t launch_explore(const DevParams& p, const StepArgs& a, hipStream_t s);
hipError_t launch_batch_explore(const DevParams* d_params, const int32_t* d_ids, int n, const BatchIn* d_in,
                                size_t lds, hipStream_t s);
hipError_t launch_weights(const DevParams& p, double* d_w, hipStream_t s);
hipError_t launch_philox_words(const DevParams& p, uint64_t counter, uint32_t* d_words, hipStream_t s);
hipError_t launch_sdf_cells(const float* sdf, int W, int H, float4* out, hipStream_t s);
int batch_rollout_blocks_per_cu(int group, size_t lds);
// The batch group of a controller's tiles (see UnitGroups).
int batch_group(const DevParams& p);
bool tile_samples_supported(int S);

}  // namespace dbas
