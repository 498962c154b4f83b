// HIP kernels (gfx950) of one DBaS-Log-MPPI iteration apart from the rollout
// (whose kernels are compiled per model, in mppi_rollout_<model>.hip, from
// the templates of mppi_device.hpp):
//   update kernel   -- one workgroup per four control rows (t, c).  Every
//                      workgroup merges the tile minima and normalisers
//                      itself (eq. control_update: rho = min S, eta), then
//                      one wave per row forms U*[t][c] = U[t][c] +
//                      sum_b f_b N_b[t][c] / eta, coalesced over tiles, and
//                      writes U* and the shifted warm start (Alg. 1 closing
//                      loop) into the other half of a double buffer, and u0*.
//   explore kernel  -- the noise-free rollout of U* and its barrier cost
//                      (Sec. IV-B eq. scaling factor), the next S_e.
//   the weights and Philox-word inspection kernels, and the host launchers.
#include "mppi_device.hpp"

#include <algorithm>

namespace dbas {
namespace {

// ---------------------------------------------------------------------------
// Update of control rows [row0, row0 + 4) of one controller, one wave per row.
// Every workgroup first merges the tile minima and normalisers itself
// (eq. control_update: rho = min_b rho_b, f_b = exp(-(rho_b - rho)/lambda),
// eta = sum_b f_b eta_b), then U*[t][c] = U[t][c] + sum_b f_b N_b[t][c] / eta,
// coalesced over tiles; it writes U*, the shifted warm start (Alg. 1 closing
// loop) into the other half of the double buffer and u0*; the workgroup of
// row 0 also records the iteration in the controller's state.
// host: what goes to the pinned host result block -- kHostNone: nothing;
// kHostPlain: u0, status and counter, seen by the host after the launch
// completes; kHostMark: the same, then the completion mark behind one
// system-scope fence, for a host thread that spins on the mark.
// ---------------------------------------------------------------------------
enum HostOut { kHostNone = 0, kHostPlain = 1, kHostMark = 2 };

__device__ void update_rows(const DevParams& p, int row0, uint32_t parity, float* u0_dev, int32_t* status_dev,
                            int host, double* sf, double* slots)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int T = p.T, nt = p.tiles;
    CtrlState* st = p.st;
    const float* Uin = p.U + (size_t)(parity & 1u) * T * kM;
    float* Uout = p.Unext ? p.Unext : p.U + (size_t)((parity + 1u) & 1u) * T * kM;
    const bool first = row0 == 0;

    // Every load that does not depend on the merge is issued first: this
    // wave's row of partN (its first kPre elements per lane), U_r, and, with
    // at most one tile per thread, the tile's scalars.
    constexpr int kPre = 8;
    const int r = row0 + wave;
    const bool has_row = r < 2 * T;
    const double* row = p.partN + (size_t)(has_row ? r : 0) * nt;
    double pre[kPre];
#pragma unroll
    for (int i = 0; i < kPre; ++i) pre[i] = (has_row && lane + i * kWave < nt) ? row[lane + i * kWave] : 0.0;
    const float u_in = has_row ? Uin[r] : 0.0f;
    // the state words the first workgroup updates at the end (the rollout
    // does not write them)
    uint64_t ctr = 0;
    uint32_t it0 = 0;
    if (first && tid == 0) {
        ctr = st->counter;
        it0 = st->iter;
    }
    HostResult* res = host != kHostNone ? p.res : nullptr;
    const bool one = nt <= kUpdBlock;
    double rb1 = INFINITY, eb1 = 0.0, fl1 = 0.0;
    if (one && tid < nt) {
        rb1 = p.rho_b[tid];
        eb1 = p.eta_b[tid];
        fl1 = (double)p.flag_b[tid];
    }

    double m = rb1;
    if (!one)
        for (int b = tid; b < nt; b += kUpdBlock) m = fmin(m, p.rho_b[b]);
    const double rho = block_min_d<kUpdWaves>(m, slots);
    double es = 0.0, n64 = 0.0;
    if (one) {
        if (tid < nt) {
            const double f = (isfinite(rho) && isfinite(rb1)) ? exp(-(rb1 - rho) / (double)p.lambda) : 0.0;
            sf[tid] = f;
            if (first) p.f_b[tid] = f;
            es = f * eb1;
            n64 = fl1;
        }
    } else {
        for (int b = tid; b < nt; b += kUpdBlock) {
            const double rb = p.rho_b[b];
            const double f = (isfinite(rho) && isfinite(rb)) ? exp(-(rb - rho) / (double)p.lambda) : 0.0;
            sf[b] = f;
            if (first) p.f_b[b] = f;
            es += f * p.eta_b[b];
            n64 += (double)p.flag_b[b];
        }
    }
    const double2 sums = block_sum_d2<kUpdWaves>(es, n64, slots);     // also publishes sf to the block
    const double eta = sums.x, n64s = sums.y;
    const bool ok = isfinite(rho) && isfinite(eta) && eta > 0.0;

    if (has_row) {
        float us;
        if (ok) {
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < kPre; ++i)
                if (lane + i * kWave < nt) a += sf[lane + i * kWave] * pre[i];
            for (int b = lane + kPre * kWave; b < nt; b += kWave) a += sf[b] * row[b];
            a = wave_sum_d(a);
            us = (float)((double)u_in + a / eta);
        } else {
            us = u_in;
        }
        if (lane == 0) {
            p.Ustar[r] = us;
            const int t = r >> 1;
            if (ok) {
                if (t >= 1) Uout[r - 2] = us;
                if (t == T - 1) Uout[r] = p.init_mode == MPPI_INIT_ZERO ? 0.0f : us;
            } else {
                Uout[r] = us;
            }
            if (t == 0) {
                if (u0_dev) u0_dev[r] = us;
                if (first) reinterpret_cast<float*>(slots)[2 * kUpdWaves * 2 + r] = us;   // for thread 0
            }
        }
    }
    if (first) {
        __syncthreads();                        // rows 0 and 1 (u0) are in LDS
        if (tid == 0) {
            const int status = ok ? MPPI_OK : MPPI_E_NUMERIC;
            st->last_counter = ctr;
            if (ok) st->counter = ctr + 1u;
            st->rho = rho;
            st->eta = eta;
            st->status = status;
            st->fp64_tiles = (int32_t)n64s;
            if (status_dev) *status_dev = status;
            const uint32_t it = it0 + 1u;
            st->iter = it;
            if (res) {
                const float* u0l = reinterpret_cast<const float*>(slots) + 2 * kUpdWaves * 2;
                res->u0[0] = u0l[0];
                res->u0[1] = u0l[1];
                res->status = status;
                res->counter = ctr;
                if (host == kHostMark) {
                    // u0, status and counter are this thread's own stores: one
                    // fence orders them before the mark
                    __threadfence_system();
                    res->seq = it;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adaptive exploration (Sec. IV-B eq. scaling factor; closing loop of
// Algorithm 1), one workgroup per controller: U* is rolled out once without
// noise from x0 (one lane; inputs saturated inside f), the fused barrier of
// every pose is summed by one wave per pose, then one lane runs
// eq. barrier_update from beta_0 in FP64, forms C_B = sum_{t=1..T} R_B beta_t
// and sets the next iteration's S_e = mu ln(e + max(C_B, 0)).
// ---------------------------------------------------------------------------
constexpr int kExpBlock = 256;

template <int MODEL>
__device__ void explore_poses(const DevParams& p, const X0& xs, float4* pose)
{
    constexpr int NS = Model<MODEL>::NS;
    float x[NS];
    x[0] = 0.0f;
    x[1] = 0.0f;
#pragma unroll
    for (int a = 2; a < NS; ++a) x[a] = xs.v[a];
    float sth, cth;
    heading_sincos(x[2], sth, cth);
    pose[0] = make_float4(0.0f, 0.0f, cth, sth);
    for (int t = 0; t < p.T; ++t) {
        const float s0 = fminf(fmaxf(p.Ustar[2 * t], p.u_min[0]), p.u_max[0]);
        const float s1 = fminf(fmaxf(p.Ustar[2 * t + 1], p.u_min[1]), p.u_max[1]);
        float f0, f1;
        Model<MODEL>::inputs(p, s0, s1, f0, f1);
        Model<MODEL>::step(p, x, f0, f1, sth, cth);
        heading_sincos(x[2], sth, cth);
        pose[t + 1] = make_float4(x[0], x[1], cth, sth);
    }
}

__device__ void explore_ctrl(const DevParams& p, const X0& xs, unsigned char* smem)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const int T = p.T, J = p.J, P = p.P;
    float4* obs = reinterpret_cast<float4*>(smem);
    float4* pose = reinterpret_cast<float4*>(smem + (size_t)obstacle_slots(J) * 16);
    float* bv = reinterpret_cast<float*>(smem + (size_t)obstacle_slots(J) * 16 + (size_t)(T + 1) * 16);
    // the rollout's local frame, centred on the start position
    const double ox = (double)xs.v[0], oy = (double)xs.v[1];
    for (int j = tid; j < J; j += kExpBlock) {
        const double cx = (double)p.obs[3 * j], cy = (double)p.obs[3 * j + 1], r = (double)p.obs[3 * j + 2];
        obs[j] = make_float4((float)(cx - ox), (float)(cy - oy), (float)(-(r * r)), 0.0f);
    }
    float inv_res = 0.0f, offx = 0.0f, offy = 0.0f;
    const bool has_map = p.sdf != nullptr;
    if (has_map) {
        inv_res = (float)(1.0 / (double)p.map_res);
        offx = (float)((ox - (double)p.map_x0) / (double)p.map_res - 0.5);
        offy = (float)((oy - (double)p.map_y0) / (double)p.map_res - 0.5);
    }
    if (tid == 0) {
        switch (p.model) {
        case MPPI_QUAD6: explore_poses<MPPI_QUAD6>(p, xs, pose); break;
        case MPPI_QUAD5: explore_poses<MPPI_QUAD5>(p, xs, pose); break;
        default: explore_poses<MPPI_CAR>(p, xs, pose); break;
        }
    }
    __syncthreads();
    for (int t = wave; t <= T; t += kExpBlock / kWave) {
        const float4 q = pose[t];
        float acc = 0.0f;
        for (int idx = lane; idx < P * J; idx += kWave) {
            const int i = idx / J, j = idx - i * J;
            const float px = fmaf(p.shape[i][0], q.z, fmaf(-p.shape[i][1], q.w, q.x));
            const float py = fmaf(p.shape[i][0], q.w, fmaf(p.shape[i][1], q.z, q.y));
            const float4 o = obs[j];
            const float dx = px - o.x, dy = py - o.y;
            acc += barrier_rcp(fmaf(dx, dx, fmaf(dy, dy, o.z)), p.h_eps);
        }
        if (has_map && lane < P) {
            const float px = fmaf(p.shape[lane][0], q.z, fmaf(-p.shape[lane][1], q.w, q.x));
            const float py = fmaf(p.shape[lane][0], q.w, fmaf(p.shape[lane][1], q.z, q.y));
            acc += barrier_rcp(sdf_sample(p, fmaf(px, inv_res, offx), fmaf(py, inv_res, offy)),
                               p.h_eps);
        }
        acc = wave_sum_f(acc);
        if (lane == 0) bv[t] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        CtrlState* st = p.st;
        const double g = (double)p.gamma_b, bd = (double)st->beta_d;
        double beta = (double)bv[0], cb = 0.0;
        for (int t = 1; t <= T; ++t) {
            beta = (double)bv[t] - g * (bd - beta);
            cb += (double)p.r_b * beta;
        }
        st->cost_b = (float)cb;
        st->S_e = (float)((double)p.explore_mu * log(2.718281828459045 + fmax(cb, 0.0)));
    }
}

__global__ __launch_bounds__(kUpdBlock) void k_update(DevParams p, StepArgs a)
{
    __shared__ double sf[kMaxTiles];
    __shared__ double slots[2 * kUpdWaves + 1];       // + u0 of rows 0 and 1
    update_rows(p, blockIdx.x * kUpdWaves, a.parity, a.u0_dev, a.status_dev, a.mark ? kHostMark : kHostNone, sf,
                slots);
}

// One workgroup per (controller, four control rows) of the batch.
__global__ __launch_bounds__(kUpdBlock) void k_batch_update(const DevParams* __restrict__ ps,
                                                            const RowUnit* __restrict__ units,
                                                            const BatchIn* __restrict__ in, float* u0s)
{
    __shared__ double sf[kMaxTiles];
    __shared__ double slots[2 * kUpdWaves + 1];       // + u0 of rows 0 and 1
    const RowUnit ru = units[blockIdx.x];
    update_rows(ps[ru.ctrl], ru.row0, in[ru.ctrl].parity, u0s ? u0s + (size_t)ru.ctrl * kM : nullptr, nullptr,
                kHostPlain, sf, slots);
}

__global__ __launch_bounds__(kExpBlock) void k_explore(DevParams p, StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    X0 xs;
#pragma unroll
    for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = a.x0_ptr ? (i < p.n ? a.x0_ptr[i] : 0.0f) : a.x0[i];
    xs.parity = a.parity;
    explore_ctrl(p, xs, smem);
}

// One workgroup per listed controller of a batch.
__global__ __launch_bounds__(kExpBlock) void k_batch_explore(const DevParams* __restrict__ ps,
                                                             const int32_t* __restrict__ ids,
                                                             const BatchIn* __restrict__ in)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int c = ids[blockIdx.x];
    X0 xs;
#pragma unroll
    for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = in[c].x0[i];
    xs.parity = in[c].parity;
    explore_ctrl(ps[c], xs, smem);
}

// The four-texel records of a costmap: record (i, j), 0 <= i < W-1,
// 0 <= j < H-1, holds the values at cell centres (i, j), (i+1, j), (i, j+1),
// (i+1, j+1).
__global__ __launch_bounds__(256) void k_sdf_cells(const float* __restrict__ sdf, int W, int H, float4* out)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= (W - 1) * (H - 1)) return;
    const int j = idx / (W - 1), i = idx - j * (W - 1);
    const float* r0 = sdf + (size_t)j * W + i;
    out[idx] = make_float4(r0[0], r0[1], r0[W], r0[W + 1]);
}

// w_k = e_k f_b(k) / eta: the weights the update used.
__global__ __launch_bounds__(256) void k_weights(DevParams p, double* w)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= p.K) return;
    const CtrlState* st = p.st;
    w[k] = st->status == MPPI_OK ? (double)p.e[k] * p.f_b[k / p.spt] / st->eta : 0.0;
}

__global__ __launch_bounds__(256) void k_philox_words(DevParams p, uint64_t counter, uint32_t* out)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= p.K * p.T) return;
    const int k = idx / p.T, t = idx - k * p.T;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)t, (uint32_t)counter, (uint32_t)(counter >> 32)),
                                  p.seed_lo, p.seed_hi);
    uint4* o = reinterpret_cast<uint4*>(out) + idx;
    *o = r;
}
}  // namespace

bool tile_samples_supported(int S) { return S >= 16 && S <= kMaxTile && (S & (S - 1)) == 0; }

hipError_t launch_rollout(const DevParams& p0, const StepArgs& a, hipStream_t s)
{
    DevParams p = p0;
    p.lg_pack = tile_lg_pack(p.J, p.T, p.n, p.spt, p.P);
    const size_t lds = tile_lds_bytes(p.J, p.T, p.n, p.spt);
    switch (p.model) {
    case MPPI_QUAD6: return launch_rollout_quad6(p, a, lds, s);
    case MPPI_QUAD5: return launch_rollout_quad5(p, a, lds, s);
    case MPPI_CAR: return launch_rollout_car(p, a, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_update(const DevParams& p, const StepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3((2 * p.T + kUpdWaves - 1) / kUpdWaves), dim3(kUpdBlock), 0, s, p, a);
    return hipGetLastError();
}

namespace {

BatchRolloutKernel batch_rollout_kernel(int group)
{
    const int key = group % kBatchKeys;
    switch (group / kBatchKeys) {
    case MPPI_QUAD6: return batch_rollout_kernel_quad6(key);
    case MPPI_QUAD5: return batch_rollout_kernel_quad5(key);
    default: return batch_rollout_kernel_car(key);
    }
}

}  // namespace

UnitGroups group_units(std::vector<BatchWork>& work, BatchUnit* out)
{
    std::stable_sort(work.begin(), work.end(), [](const BatchWork& a, const BatchWork& b) {
        return a.group != b.group ? a.group < b.group : a.cost > b.cost;
    });
    UnitGroups g{};
    for (int m = 0; m < kBatchGroups; ++m) g.begin[m] = -1;
    for (size_t i = 0; i < work.size(); ++i) {
        const int m = work[i].group;
        if (g.begin[m] < 0) g.begin[m] = (int)i;
        ++g.count[m];
        g.work[m] += work[i].cost;
        if (work[i].lds > g.lds[m]) g.lds[m] = work[i].lds;
        out[i] = work[i].unit;
    }
    for (int m = 0; m < kBatchGroups; ++m)
        if (g.begin[m] < 0) g.begin[m] = 0;
    return g;
}

hipError_t launch_batch_rollouts(const DevParams* d_params, const BatchUnit* d_units, const UnitGroups& g,
                                 const BatchIn* d_in, uint32_t* d_queue, int cus, hipStream_t s)
{
    int order[kBatchGroups];
    for (int i = 0; i < kBatchGroups; ++i) order[i] = i;
    std::stable_sort(order, order + kBatchGroups, [&](int a, int b) { return g.work[a] > g.work[b]; });
    for (int i = 0; i < kBatchGroups; ++i) {
        const int m = order[i];
        if (g.count[m] == 0) continue;
        const int grid = std::max(1, std::min(g.count[m], cus * batch_rollout_blocks_per_cu(m, g.lds[m])));
        hipLaunchKernelGGL(batch_rollout_kernel(m), dim3(grid), dim3(kRollBlock), g.lds[m], s, d_params,
                           d_units + g.begin[m], g.count[m], d_in, d_queue + 2 * m);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_update(const DevParams* d_params, const RowUnit* d_units, int nunits, const BatchIn* d_in,
                               float* d_u0s, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_update, dim3(nunits), dim3(kUpdBlock), 0, s, d_params, d_units, d_in, d_u0s);
    return hipGetLastError();
}

hipError_t launch_explore(const DevParams& p, const StepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_explore, dim3(1), dim3(kExpBlock), explore_lds_bytes(p.J, p.T), s, p, a);
    return hipGetLastError();
}

hipError_t launch_batch_explore(const DevParams* d_params, const int32_t* d_ids, int n, const BatchIn* d_in,
                                size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_explore, dim3(n), dim3(kExpBlock), lds, s, d_params, d_ids, d_in);
    return hipGetLastError();
}

hipError_t launch_weights(const DevParams& p, double* d_w, hipStream_t s)
{
    hipLaunchKernelGGL(k_weights, dim3((p.K + 255) / 256), dim3(256), 0, s, p, d_w);
    return hipGetLastError();
}

hipError_t launch_sdf_cells(const float* sdf, int W, int H, float4* out, hipStream_t s)
{
    const int n = (W - 1) * (H - 1);
    hipLaunchKernelGGL(k_sdf_cells, dim3((n + 255) / 256), dim3(256), 0, s, sdf, W, H, out);
    return hipGetLastError();
}

hipError_t launch_philox_words(const DevParams& p, uint64_t counter, uint32_t* d_words, hipStream_t s)
{
    const int n = p.K * p.T;
    hipLaunchKernelGGL(k_philox_words, dim3((n + 255) / 256), dim3(256), 0, s, p, counter, d_words);
    return hipGetLastError();
}

int batch_group(const DevParams& p)
{
    int size = 0;
    for (int k = 0; k < kTileSizes; ++k)
        if (p.spt == (16 << k)) size = k;
    const int map = p.sdf != nullptr;
    int kind;
    if (p.cost_mode == MPPI_COST_INDICATOR) kind = 4 + map;
    else if (p.P == fixed_points(p.model) && p.shape_kind != kShapeGeneral) kind = map;
    else kind = 2 + map;
    return p.model * kBatchKeys + kind * kTileSizes + size;
}

int batch_rollout_blocks_per_cu(int group, size_t lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_rollout_kernel(group), kRollBlock, lds) !=
        hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace dbas
