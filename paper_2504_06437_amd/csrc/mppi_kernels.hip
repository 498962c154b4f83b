// HIP kernels (gfx950) of one DBaS-Log-MPPI iteration.
//
//   rollout kernel  -- one workgroup per sample tile.  Each sample is owned by
//                      a group of G lanes (G = 1: one sample per lane).  Per
//                      step: Philox4x32-10 + normal x log-normal noise (Sec.
//                      IV-C, shared across the group), the dynamics (eq.
//                      veh_dyn) with saturated inputs, the fused barrier over
//                      the obstacles (staged in LDS, split across the group)
//                      and the costmap, the barrier-state recursion (eq.
//                      barrier_update) and the running cost (Alg. 1, eq.
//                      cost-to-go_bas) in a compensated FP32 sum.  The tile
//                      then forms its own min-shifted exponentials and the
//                      tile sums  eta_b = sum e_k,  N_b[t][c] = sum e_k du_k,
//                      and the last tile to finish merges the tile minima and
//                      normalisers (eq. control_update: rho = min S, eta).
//   update kernel   -- one wave per control row (t, c): U*[t][c] = U[t][c] +
//                      sum_b f_b N_b[t][c] / eta, coalesced over tiles; writes
//                      U* and the shifted warm start (Alg. 1 closing loop)
//                      into the other half of a double buffer, and u0*.
//
// All positions are handled in a frame centred on the iteration's start
// position (obstacles, reference and costmap offset are translated once in
// FP64), so FP32 rounding is relative to the rollout's extent, not the world's.
#include "mppi_internal.hpp"

#include <math.h>

namespace dbas {
namespace {

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32-10 (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 23 high bits centred in their cell: ((r >> 9) + 1/2) 2^-23, exact in FP32.
__device__ __forceinline__ float word_to_uniform(uint32_t r)
{
    return fmaf((float)(r >> 9), 0x1p-23f, 0x1p-24f);
}

// Normal x log-normal pair for inputs (0, 1) from one Philox block: Box-Muller
// normals n from words (0, 1), z from words (2, 3);
// du_c = sqrt(S_e) sigma_c n_c exp(mu_ln + sigma_ln z_c).
__device__ __forceinline__ float2 nln_pair(uint4 r, float scale0, float scale1, float mu_ln, float sigma_ln)
{
    const float u0 = word_to_uniform(r.x), u1 = word_to_uniform(r.y);
    const float u2 = word_to_uniform(r.z), u3 = word_to_uniform(r.w);
    const float rn = sqrtf(-2.0f * logf(u0));
    const float rz = sqrtf(-2.0f * logf(u2));
    float sn, cn, sz, cz;
    sincospif(2.0f * u1, &sn, &cn);
    sincospif(2.0f * u3, &sz, &cz);
    float2 o;
    o.x = scale0 * (rn * cn) * expf(fmaf(sigma_ln, rz * cz, mu_ln));
    o.y = scale1 * (rn * sn) * expf(fmaf(sigma_ln, rz * sz, mu_ln));
    return o;
}

// ---------------------------------------------------------------------------
// Cross-lane helpers.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over a group of G adjacent lanes (G <= 16, inside one DPP row).  Every
// lane of the group ends with the same bits: each stage adds a lane's value
// to its partner's, and IEEE addition is commutative.
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (G >= 2) v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    if constexpr (G >= 4) v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    if constexpr (G >= 8) v += dpp<0x141>(v);   // row_half_mirror
    if constexpr (G >= 16) v += dpp<0x140>(v);  // row_mirror
    return v;
}

__device__ __forceinline__ float lane_read(float v, int src_lane)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ double wave_min_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m));
    return v;
}

// Block reductions (256 threads); every thread gets the result.
__device__ __forceinline__ double block_min_d(double v, double* slots)
{
    v = wave_min_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = slots[0];
#pragma unroll
    for (int i = 1; i < kBlock / kWave; ++i) r = fmin(r, slots[i]);
    return r;
}

__device__ __forceinline__ double block_sum_d(double v, double* slots)
{
    v = wave_sum_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = slots[0];
#pragma unroll
    for (int i = 1; i < kBlock / kWave; ++i) r += slots[i];
    return r;
}

__device__ __forceinline__ float block_sum_f(float v, double* slots)
{
    v = wave_sum_f(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = (double)v;
    __syncthreads();
    float r = (float)slots[0];
#pragma unroll
    for (int i = 1; i < kBlock / kWave; ++i) r += (float)slots[i];
    return r;
}

// Compensated accumulation (Knuth's TwoSum): hi + lo carries the sum exactly
// up to the rounding of lo.
__device__ __forceinline__ void two_sum_acc(float& hi, float& lo, float x)
{
    const float s = hi + x;
    const float bp = s - hi;
    const float err = (hi - (s - bp)) + (x - bp);
    hi = s;
    lo += err;
}

__device__ __forceinline__ float barrier_rcp(float h, float eps)
{
    return __builtin_amdgcn_rcpf(fmaxf(h, eps));
}

// Bilinear costmap sample between cell centres, clamped to the edge cells.
// (gx, gy) are continuous cell coordinates; any float input stays in bounds.
__device__ __forceinline__ float sdf_sample(const float* __restrict__ sdf, int W, int H, float gx, float gy)
{
    gx = fminf(fmaxf(gx, 0.0f), (float)(W - 1));
    gy = fminf(fmaxf(gy, 0.0f), (float)(H - 1));
    const int i0 = min((int)floorf(gx), W - 2);
    const int j0 = min((int)floorf(gy), H - 2);
    const float fx = gx - (float)i0, fy = gy - (float)j0;
    const float* r0 = sdf + (size_t)j0 * W + i0;
    const float* r1 = r0 + W;
    const float top = fmaf(fx, r0[1] - r0[0], r0[0]);
    const float bot = fmaf(fx, r1[1] - r1[0], r1[0]);
    return fmaf(fy, bot - top, top);
}

// ---------------------------------------------------------------------------
// Models (explicit Euler, inputs saturated inside f).  sth/cth are the sine
// and cosine of the *old* heading.
// ---------------------------------------------------------------------------
template <int MODEL> struct Model;

template <> struct Model<MPPI_QUAD6> {
    static constexpr int NS = 6;
    // state (x, z, theta, vx, vz, omega); inputs: rotor thrust deviations.
    __device__ static __forceinline__ void step(const DevParams& p, float* x, float s0, float s1,
                                                float sth, float cth)
    {
        const float dt = p.dt;
        const float hover = 0.5f * p.mass * p.gravity;
        const float F1 = hover + s0, F2 = hover + s1;
        const float acc = (F1 + F2) / p.mass;
        const float x0 = x[0] + x[3] * dt;
        const float x1 = x[1] + x[4] * dt;
        const float x2 = x[2] + x[5] * dt;
        const float x3 = x[3] - acc * sth * dt;
        const float x4 = x[4] + (acc * cth - p.gravity) * dt;
        const float x5 = x[5] + (F2 - F1) * (p.arm / p.inertia) * dt;
        x[0] = x0; x[1] = x1; x[2] = x2; x[3] = x3; x[4] = x4; x[5] = x5;
    }
};

template <> struct Model<MPPI_QUAD5> {
    static constexpr int NS = 5;
    // Sec. V-A: state (x, z, theta, vx, vz); inputs (pitch rate, throttle).
    __device__ static __forceinline__ void step(const DevParams& p, float* x, float s0, float s1,
                                                float sth, float cth)
    {
        const float dt = p.dt;
        const float acc = (p.mass * p.gravity + s1) / p.mass;
        const float x0 = x[0] + x[3] * dt;
        const float x1 = x[1] + x[4] * dt;
        const float x2 = x[2] + s0 * dt;
        const float x3 = x[3] - acc * sth * dt;
        const float x4 = x[4] + (acc * cth - p.gravity) * dt;
        x[0] = x0; x[1] = x1; x[2] = x2; x[3] = x3; x[4] = x4;
    }
};

template <> struct Model<MPPI_CAR> {
    static constexpr int NS = 4;
    // Sec. V-B Ackermann model: state (x, y, theta, v); inputs (steer, accel).
    __device__ static __forceinline__ void step(const DevParams& p, float* x, float s0, float s1,
                                                float sth, float cth)
    {
        const float dt = p.dt;
        const float v = x[3];
        const float x0 = x[0] + v * cth * dt;
        const float x1 = x[1] + v * sth * dt;
        const float x2 = x[2] + v * tanf(s0) / p.wheelbase * dt;
        const float x3 = x[3] + s1 * dt;
        x[0] = x0; x[1] = x1; x[2] = x2; x[3] = x3;
    }
};

// LDS carve-up of one rollout tile.
struct TileLds {
    float4* obs;     // [J] (ox, oy, -r^2, 0), local frame
    float2* U;       // [T]
    float* ref;      // [(T+1) n], local frame
    double* e;       // [kBlock]
    double* slots;   // [16]
};

__device__ __forceinline__ TileLds carve(unsigned char* smem, int J, int T, int n)
{
    TileLds L;
    size_t off = 0;
    L.obs = reinterpret_cast<float4*>(smem + off);
    off += (size_t)(J > 0 ? J : 1) * 16;
    L.U = reinterpret_cast<float2*>(smem + off);
    off += (size_t)T * 8;
    L.ref = reinterpret_cast<float*>(smem + off);
    off += (size_t)(T + 1) * n * 4;
    off = (off + 15) & ~(size_t)15;
    L.e = reinterpret_cast<double*>(smem + off);
    off += (size_t)kBlock * 8;
    L.slots = reinterpret_cast<double*>(smem + off);
    return L;
}

struct X0 {
    float v[MPPI_NMAX + 2];
};

// Fused barrier of a (local-frame) pose, cooperatively over the block.
__device__ float fused_barrier_block(const DevParams& p, const TileLds& L, int P, float px0, float py0, float th,
                                     float inv_res, float offx, float offy)
{
    float sth, cth;
    sincosf(th, &sth, &cth);
    float acc = 0.0f;
    const int J = p.J;
    for (int idx = threadIdx.x; idx < P * J; idx += kBlock) {
        const int i = idx / J, j = idx - i * J;
        const float a = p.shape[i][0], b = p.shape[i][1];
        const float px = px0 + (a * cth - b * sth);
        const float py = py0 + (a * sth + b * cth);
        const float4 o = L.obs[j];
        const float dx = px - o.x, dy = py - o.y;
        acc += barrier_rcp(fmaf(dx, dx, fmaf(dy, dy, o.z)), p.h_eps);
    }
    if (p.sdf != nullptr && (int)threadIdx.x < P) {
        const int i = threadIdx.x;
        const float a = p.shape[i][0], b = p.shape[i][1];
        const float px = px0 + (a * cth - b * sth);
        const float py = py0 + (a * sth + b * cth);
        acc += barrier_rcp(sdf_sample(p.sdf, p.map_w, p.map_h, fmaf(px, inv_res, offx), fmaf(py, inv_res, offy)),
                           p.h_eps);
    }
    return block_sum_f(acc, L.slots);
}

// ---------------------------------------------------------------------------
// One sample tile: rollout, tile softmax partials, last-tile merge.
// PT = compile-time number of shape points (0: runtime P <= MPPI_PMAX).
// ---------------------------------------------------------------------------
template <int MODEL, int G, int PT>
__device__ void rollout_tile(const DevParams& p, const int tile, const X0& xs, unsigned char* smem)
{
    constexpr int NS = Model<MODEL>::NS;
    constexpr int PM = PT ? PT : MPPI_PMAX;
    const int tid = threadIdx.x;
    const int J = p.J, T = p.T, K = p.K, Kp = p.Kp;
    const int P = PT ? PT : p.P;
    const TileLds L = carve(smem, J, T, NS);

    const uint32_t iter = p.st->iter;
    const float* Uin = p.U + (size_t)(iter & 1u) * T * kM;

    // ---- staging: local frame centred on the start position ----
    const double ox = (double)xs.v[0], oy = (double)xs.v[1];
    for (int j = tid; j < J; j += kBlock) {
        const double cx = (double)p.obs[3 * j], cy = (double)p.obs[3 * j + 1], r = (double)p.obs[3 * j + 2];
        L.obs[j] = make_float4((float)(cx - ox), (float)(cy - oy), (float)(-(r * r)), 0.0f);
    }
    for (int t = tid; t < T; t += kBlock) L.U[t] = make_float2(Uin[2 * t], Uin[2 * t + 1]);
    for (int i = tid; i < (T + 1) * NS; i += kBlock) {
        const int a = i % NS;
        const float v = p.xref[i];
        L.ref[i] = a == 0 ? (float)((double)v - ox) : a == 1 ? (float)((double)v - oy) : v;
    }
    float inv_res = 0.0f, offx = 0.0f, offy = 0.0f;
    const bool has_map = p.sdf != nullptr;
    if (has_map) {
        inv_res = (float)(1.0 / (double)p.map_res);
        offx = (float)((ox - (double)p.map_x0) / (double)p.map_res - 0.5);
        offy = (float)((oy - (double)p.map_y0) / (double)p.map_res - 0.5);
    }
    __syncthreads();

    // beta_0 = fused B(h(x0)); beta_d = fused B(h(x_d)), x_d = x_ref[T].
    const float beta0 = fused_barrier_block(p, L, P, 0.0f, 0.0f, xs.v[2], inv_res, offx, offy);
    const float beta_d = fused_barrier_block(p, L, P, L.ref[T * NS], L.ref[T * NS + 1], L.ref[T * NS + 2],
                                             inv_res, offx, offy);

    // ---- per-lane setup ----
    const int lane = tid & (kWave - 1);
    const int g = tid & (G - 1);
    const int sidx = tid / G;
    const int k = tile * p.spt + sidx;
    const bool valid = k < K;
    const int gbase = lane & ~(G - 1);

    const float S_e = p.st->S_e;
    const float sqS = sqrtf(S_e);
    const float scale0 = sqS * p.sigma[0], scale1 = sqS * p.sigma[1];
    const float cw0 = p.sigma[0] > 0.0f ? p.gamma_u / (S_e * p.sigma[0] * p.sigma[0]) : 0.0f;
    const float cw1 = p.sigma[1] > 0.0f ? p.gamma_u / (S_e * p.sigma[1] * p.sigma[1]) : 0.0f;
    const uint64_t ctr = p.st->counter;
    const uint32_t c_lo = (uint32_t)ctr, c_hi = (uint32_t)(ctr >> 32);
    const float eps = p.h_eps;

    float x[NS];
    x[0] = 0.0f;
    x[1] = 0.0f;
#pragma unroll
    for (int a = 2; a < NS; ++a) x[a] = xs.v[a];
    float sth, cth;
    sincosf(x[2], &sth, &cth);
    // eq. barrier_update is linear in beta, so beta_t = bv_t + c_t with the
    // sample-dependent part bv_t = b_t + gamma_B bv_{t-1} (bv_0 = beta_0) and
    // the common part c_t = gamma_B (c_{t-1} - beta_d) (c_0 = 0).  The common
    // part's cost R_B sum_t c_t is the same for every sample and is added in
    // FP64 (cshift), so a large beta_d cannot swamp the FP32 running sum.
    float beta = beta0;
    double cshift = 0.0;
    {
        double c = 0.0;
        for (int t = 0; t < T; ++t) {
            c = (double)p.gamma_b * (c - (double)beta_d);
            cshift += (double)p.r_b * c;
        }
    }
    float S_hi = 0.0f, S_lo = 0.0f;
    float my_du0 = 0.0f, my_du1 = 0.0f;

    float sa[PM], sb[PM];
#pragma unroll
    for (int i = 0; i < PM; ++i) {
        sa[i] = (PT || i < P) ? p.shape[i][0] : 0.0f;
        sb[i] = (PT || i < P) ? p.shape[i][1] : 0.0f;
    }

    for (int t = 0; t < T; ++t) {
        // -- noise (Alg. 1 sampling; Sec. IV-C) --
        float du0, du1;
        if constexpr (G == 1) {
            const uint4 r = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)t, c_lo, c_hi), p.seed_lo, p.seed_hi);
            const float2 z = nln_pair(r, scale0, scale1, p.mu_ln, p.sigma_ln);
            du0 = z.x;
            du1 = z.y;
            if (valid) {
                p.du[(size_t)(2 * t) * Kp + k] = du0;
                p.du[(size_t)(2 * t + 1) * Kp + k] = du1;
            }
        } else {
            const int j = t & (G - 1);
            if (j == 0) {
                const int tt = t + g;
                const uint4 r = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)tt, c_lo, c_hi), p.seed_lo, p.seed_hi);
                const float2 z = nln_pair(r, scale0, scale1, p.mu_ln, p.sigma_ln);
                my_du0 = z.x;
                my_du1 = z.y;
                if (valid && tt < T) {
                    p.du[(size_t)(2 * tt) * Kp + k] = my_du0;
                    p.du[(size_t)(2 * tt + 1) * Kp + k] = my_du1;
                }
            }
            du0 = lane_read(my_du0, gbase + j);
            du1 = lane_read(my_du1, gbase + j);
        }

        // -- dynamics with saturated inputs --
        const float2 u = L.U[t];
        const float v0 = u.x + du0, v1 = u.y + du1;
        const float s0 = fminf(fmaxf(v0, p.u_min[0]), p.u_max[0]);
        const float s1 = fminf(fmaxf(v1, p.u_min[1]), p.u_max[1]);
        Model<MODEL>::step(p, x, s0, s1, sth, cth);
        sincosf(x[2], &sth, &cth);

        // -- shape points and this lane's share of the fused barrier --
        float px[PM], py[PM];
#pragma unroll
        for (int i = 0; i < PM; ++i) {
            px[i] = x[0] + (sa[i] * cth - sb[i] * sth);
            py[i] = x[1] + (sa[i] * sth + sb[i] * cth);
        }
        float acc = 0.0f;
        for (int j = g; j < J; j += G) {
            const float4 o = L.obs[j];
#pragma unroll
            for (int i = 0; i < PM; ++i) {
                if (PT || i < P) {
                    const float dx = px[i] - o.x, dy = py[i] - o.y;
                    acc += barrier_rcp(fmaf(dx, dx, fmaf(dy, dy, o.z)), eps);
                }
            }
        }
        if (has_map) {
#pragma unroll
            for (int i = 0; i < PM; ++i) {
                if ((PT || i < P) && (i & (G - 1)) == g) {
                    acc += barrier_rcp(sdf_sample(p.sdf, p.map_w, p.map_h, fmaf(px[i], inv_res, offx),
                                                  fmaf(py[i], inv_res, offy)),
                                       eps);
                }
            }
        }
        const float b = group_sum<G>(acc);

        // -- barrier state (eq. barrier_update, sample-dependent part) and running cost --
        beta = fmaf(p.gamma_b, beta, b);
        const float* rf = L.ref + (t + 1) * NS;
        float q = 0.0f;
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const float d = x[a] - rf[a];
            q = fmaf(p.Q[a], d * d, q);
        }
        const float ctrl = cw0 * u.x * v0 + cw1 * u.y * v1;
        two_sum_acc(S_hi, S_lo, q + ctrl + p.r_b * beta);
    }
    {
        const float* rf = L.ref + T * NS;
        float phi = 0.0f;
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            const float d = x[a] - rf[a];
            phi = fmaf(p.Qf[a], d * d, phi);
        }
        two_sum_acc(S_hi, S_lo, phi);
    }

    // ---- tile softmax partials ----
    if (g == 0 && valid) {
        p.S[k] = S_hi;
        p.S[Kp + k] = S_lo;
    }
    const double Sd = ((double)S_hi + (double)S_lo) + cshift;
    const bool ok = valid && isfinite(Sd);
    const double rho_b = block_min_d(ok ? Sd : INFINITY, L.slots);
    const bool any = isfinite(rho_b);
    const bool use64 = any && (p.normaliser == MPPI_NORM_ON ||
                               (p.normaliser == MPPI_NORM_AUTO && fabs(rho_b) >= 1024.0 * (double)p.lambda));
    double ek = 0.0;
    if (ok) {
        const double d = (Sd - rho_b) / (double)p.lambda;
        ek = use64 ? exp(-d) : (double)expf(-(float)d);
    }
    if (g == 0) L.e[sidx] = ek;
    if (g == 0 && valid) p.e[k] = (float)ek;
    __syncthreads();
    const int spt = p.spt;
    double eta_b;
    if (use64) eta_b = block_sum_d(tid < spt ? L.e[tid] : 0.0, L.slots);
    else eta_b = (double)block_sum_f(tid < spt ? (float)L.e[tid] : 0.0f, L.slots);

    // N_b[r] = sum over the tile's samples of e_k du[r][k]; one wave per row.
    const int wave = tid >> 6;
    const int k0 = tile * spt;
    const int nk = min(spt, K - k0);
    for (int r = wave; r < 2 * T; r += kBlock / kWave) {
        const float* row = p.du + (size_t)r * Kp + k0;
        double out;
        if (use64) {
            double a = 0.0;
            for (int s = lane; s < nk; s += kWave) a += L.e[s] * (double)row[s];
            out = wave_sum_d(a);
        } else {
            float a = 0.0f;
            for (int s = lane; s < nk; s += kWave) a = fmaf((float)L.e[s], row[s], a);
            out = (double)wave_sum_f(a);
        }
        if (lane == 0) p.partN[(size_t)r * p.tiles + tile] = any ? out : 0.0;
    }
    if (tid == 0) {
        p.rho_b[tile] = rho_b;
        p.eta_b[tile] = any ? eta_b : 0.0;
        p.flag_b[tile] = use64 ? 1 : 0;
    }

    // ---- completion ticket; the last tile merges the tile scalars ----
    __threadfence();
    __syncthreads();
    __shared__ uint32_t s_last;
    if (tid == 0) s_last = atomicAdd(&p.st->tiles_done, 1u) == (uint32_t)(p.tiles - 1) ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    const int nt = p.tiles;
    double m = INFINITY;
    for (int b = tid; b < nt; b += kBlock) m = fmin(m, __builtin_nontemporal_load(&p.rho_b[b]));
    const double rho = block_min_d(m, L.slots);
    double es = 0.0;
    int n64 = 0;
    if (isfinite(rho)) {
        for (int b = tid; b < nt; b += kBlock) {
            const double rb = __builtin_nontemporal_load(&p.rho_b[b]);
            const double f = isfinite(rb) ? exp(-(rb - rho) / (double)p.lambda) : 0.0;
            p.f_b[b] = f;
            es += f * __builtin_nontemporal_load(&p.eta_b[b]);
            n64 += __builtin_nontemporal_load(&p.flag_b[b]);
        }
    }
    const double eta = block_sum_d(es, L.slots);
    const double n64s = block_sum_d((double)n64, L.slots);
    if (tid == 0) {
        CtrlState* st = p.st;
        st->rho = rho;
        st->eta = eta;
        st->status = (isfinite(rho) && eta > 0.0 && isfinite(eta)) ? MPPI_OK : MPPI_E_NUMERIC;
        st->beta0 = beta0;
        st->beta_d = beta_d;
        st->cshift = cshift;
        st->fp64_tiles = (int32_t)n64s;
        st->tiles_done = 0u;
        st->iter = iter + 1u;
    }
}

// ---------------------------------------------------------------------------
// Update rows [row0, row0 + 4) of one controller (one wave per row).
// ---------------------------------------------------------------------------
__device__ void update_rows(const DevParams& p, int row0, float* u0_dev)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int r = row0 + (threadIdx.x >> 6);
    const int T = p.T;
    const CtrlState* st = p.st;
    const uint32_t iter = st->iter;                 // already advanced by the rollout
    const float* Uin = p.U + (size_t)((iter - 1u) & 1u) * T * kM;
    float* Uout = p.U + (size_t)(iter & 1u) * T * kM;
    const bool ok = st->status == MPPI_OK;
    if (r >= 2 * T) return;

    float us;
    if (ok) {
        const int nt = p.tiles;
        const double* row = p.partN + (size_t)r * nt;
        double a = 0.0;
        for (int b = lane; b < nt; b += kWave) a += p.f_b[b] * row[b];
        a = wave_sum_d(a);
        us = (float)((double)Uin[r] + a / st->eta);
    } else {
        us = Uin[r];
    }
    if (lane != 0) return;
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
        if (p.res) p.res->u0[r] = us;
        if (r == 0) {
            CtrlState* sw = p.st;
            const uint64_t c = sw->counter;
            sw->last_counter = c;
            if (ok) sw->counter = c + 1u;
            if (p.res) {
                p.res->status = st->status;
                p.res->counter = c;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <int MODEL, int G, int PT>
__global__ __launch_bounds__(kBlock) void k_rollout(DevParams p, StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    X0 xs;
#pragma unroll
    for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = a.x0_ptr ? (i < p.n ? a.x0_ptr[i] : 0.0f) : a.x0[i];
    rollout_tile<MODEL, G, PT>(p, blockIdx.x, xs, smem);
}

__global__ __launch_bounds__(kBlock) void k_update(DevParams p, StepArgs a)
{
    update_rows(p, blockIdx.x * kRowsPerBlock, a.u0_dev);
}

template <int MODEL, int G>
__device__ __forceinline__ void dispatch_p(const DevParams& p, int tile, const X0& xs, unsigned char* smem)
{
    constexpr int PD = MODEL == MPPI_CAR ? 8 : 7;
    if (p.P == PD) rollout_tile<MODEL, G, PD>(p, tile, xs, smem);
    else rollout_tile<MODEL, G, 0>(p, tile, xs, smem);
}

template <int MODEL>
__device__ __forceinline__ void dispatch_g(const DevParams& p, int tile, const X0& xs, unsigned char* smem)
{
    switch (p.G) {
    case 1: dispatch_p<MODEL, 1>(p, tile, xs, smem); break;
    case 2: dispatch_p<MODEL, 2>(p, tile, xs, smem); break;
    case 4: dispatch_p<MODEL, 4>(p, tile, xs, smem); break;
    case 8: dispatch_p<MODEL, 8>(p, tile, xs, smem); break;
    default: dispatch_p<MODEL, 16>(p, tile, xs, smem); break;
    }
}

// Persistent rollout over a work list of (controller, tile) units, taken in
// list order (the host sorts it longest-first).  Every block leaves the loop
// once the list is exhausted; the last block to leave resets the queue.
__global__ __launch_bounds__(kBlock) void k_batch_rollout(const DevParams* __restrict__ ps,
                                                          const BatchUnit* __restrict__ units, int nunits,
                                                          const float* __restrict__ x0s, uint32_t* queue)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_unit;
    for (;;) {
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(&queue[0], 1u);
        __syncthreads();
        const int u = s_unit;
        __syncthreads();
        if (u >= nunits) break;
        const BatchUnit bu = units[u];
        const DevParams& p = ps[bu.ctrl];
        X0 xs;
#pragma unroll
        for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = x0s[(size_t)bu.ctrl * (MPPI_NMAX + 2) + i];
        switch (p.model) {
        case MPPI_QUAD6: dispatch_g<MPPI_QUAD6>(p, bu.tile, xs, smem); break;
        case MPPI_QUAD5: dispatch_g<MPPI_QUAD5>(p, bu.tile, xs, smem); break;
        default: dispatch_g<MPPI_CAR>(p, bu.tile, xs, smem); break;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[1], 1u) == gridDim.x - 1u) {
            queue[0] = 0u;
            queue[1] = 0u;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_update(const DevParams* __restrict__ ps,
                                                         const RowUnit* __restrict__ units, float* u0s)
{
    const RowUnit ru = units[blockIdx.x];
    update_rows(ps[ru.ctrl], ru.row0, u0s ? u0s + (size_t)ru.ctrl * kM : nullptr);
}

// w_k = e_k f_b(k) / eta: the weights the update used.
__global__ __launch_bounds__(kBlock) void k_weights(DevParams p, double* w)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= p.K) return;
    const CtrlState* st = p.st;
    w[k] = st->status == MPPI_OK ? (double)p.e[k] * p.f_b[k / p.spt] / st->eta : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_philox_words(DevParams p, uint64_t counter, uint32_t* out)
{
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= p.K * p.T) return;
    const int k = idx / p.T, t = idx - k * p.T;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)t, (uint32_t)counter, (uint32_t)(counter >> 32)),
                                  p.seed_lo, p.seed_hi);
    uint4* o = reinterpret_cast<uint4*>(out) + idx;
    *o = r;
}

template <int MODEL, int G>
hipError_t launch_rollout_mg(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    constexpr int PD = MODEL == MPPI_CAR ? 8 : 7;
    if (p.P == PD) hipLaunchKernelGGL((k_rollout<MODEL, G, PD>), dim3(p.tiles), dim3(kBlock), lds, s, p, a);
    else hipLaunchKernelGGL((k_rollout<MODEL, G, 0>), dim3(p.tiles), dim3(kBlock), lds, s, p, a);
    return hipGetLastError();
}

template <int MODEL>
hipError_t launch_rollout_m(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    switch (p.G) {
    case 1: return launch_rollout_mg<MODEL, 1>(p, a, lds, s);
    case 2: return launch_rollout_mg<MODEL, 2>(p, a, lds, s);
    case 4: return launch_rollout_mg<MODEL, 4>(p, a, lds, s);
    case 8: return launch_rollout_mg<MODEL, 8>(p, a, lds, s);
    case 16: return launch_rollout_mg<MODEL, 16>(p, a, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool tile_lanes_supported(int G) { return G == 1 || G == 2 || G == 4 || G == 8 || G == 16; }

hipError_t launch_rollout(const DevParams& p, const StepArgs& a, hipStream_t s)
{
    const size_t lds = tile_lds_bytes(p.J, p.T, p.n);
    switch (p.model) {
    case MPPI_QUAD6: return launch_rollout_m<MPPI_QUAD6>(p, a, lds, s);
    case MPPI_QUAD5: return launch_rollout_m<MPPI_QUAD5>(p, a, lds, s);
    case MPPI_CAR: return launch_rollout_m<MPPI_CAR>(p, a, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_update(const DevParams& p, const StepArgs& a, hipStream_t s)
{
    const int rows = 2 * p.T;
    hipLaunchKernelGGL(k_update, dim3((rows + kRowsPerBlock - 1) / kRowsPerBlock), dim3(kBlock), 0, s, p, a);
    return hipGetLastError();
}

hipError_t launch_batch_rollout(const DevParams* d_params, const BatchUnit* d_units, int nunits,
                                const float* d_x0s, uint32_t* d_queue, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_rollout, dim3(grid), dim3(kBlock), lds, s, d_params, d_units, nunits, d_x0s, d_queue);
    return hipGetLastError();
}

hipError_t launch_batch_update(const DevParams* d_params, const RowUnit* d_units, int nunits, float* d_u0s,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_update, dim3(nunits), dim3(kBlock), 0, s, d_params, d_units, d_u0s);
    return hipGetLastError();
}

hipError_t launch_weights(const DevParams& p, double* d_w, hipStream_t s)
{
    hipLaunchKernelGGL(k_weights, dim3((p.K + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, d_w);
    return hipGetLastError();
}

hipError_t launch_philox_words(const DevParams& p, uint64_t counter, uint32_t* d_words, hipStream_t s)
{
    const int n = p.K * p.T;
    hipLaunchKernelGGL(k_philox_words, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, counter, d_words);
    return hipGetLastError();
}

int batch_rollout_blocks_per_cu(size_t lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_rollout, kBlock, lds) != hipSuccess) return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace dbas
