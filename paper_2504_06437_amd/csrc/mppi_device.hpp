// Device code of the DBaS-Log-MPPI rollout (gfx950), shared by the kernel
// translation units: helpers, the models, the rollout tile and the rollout
// kernel templates (standalone and batched).  Everything has internal
// linkage; each unit instantiates what it launches.
//
//   rollout kernel  -- one workgroup per tile of S samples.  The horizon is
//                      cut into chunks that flow through a pipeline of
//                      workgroup-wide stages; per chunk:
//                       - inputs: Philox4x32-10 normal x log-normal noise
//                         (Sec. IV-C) for every (step, sample), turned into the
//                         state-independent terms (saturated inputs, their
//                         model terms, the control cost of Alg. 1), in LDS;
//                       - dynamics: one lane per sample integrates the state
//                         (eq. veh_dyn), storing the pose of every step and
//                         adding the tracking and control costs;
//                       - barrier: every (step, sample) is split over lanes
//                         that each take a range of obstacles (LDS) and the
//                         costmap -- the bulk of the work, no dependence
//                         between items;
//                       - barrier state: one lane per sample runs the
//                         recursion of eq. barrier_update and adds R_B beta
//                         (Alg. 1, eq. cost-to-go_bas) to its compensated
//                         FP32 cost.
//                      The sequential parts (dynamics, barrier state) of one
//                      chunk overlap the parallel parts of its neighbours.
//                      The tile then forms its own min-shifted exponentials
//                      and the tile sums eta_b = sum e_k and N_b[t][c] =
//                      sum e_k du_k.  Tiles never wait for one another.
// Positions are handled in a frame centred on the iteration's start position
// (obstacles, reference and costmap offset are translated once in FP64), so
// FP32 rounding is relative to the rollout's extent, not the world's.
#pragma once

#include "mppi_internal.hpp"

#include <math.h>

#include <algorithm>
#include <type_traits>

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
// du_c = sqrt(S_e) sigma_c n_c exp(mu_ln + sigma_ln z_c), or with `normal`
// (Vanilla MPPI's law) the normal part sqrt(S_e) sigma_c n_c alone.
__device__ __forceinline__ float2 nln_pair(uint4 r, float scale0, float scale1, float mu_ln, float sigma_ln,
                                           bool normal)
{
    const float u0 = word_to_uniform(r.x), u1 = word_to_uniform(r.y);
    const float rn = sqrtf(-2.0f * logf(u0));
    float sn, cn;
    sincospif(2.0f * u1, &sn, &cn);
    float2 o;
    o.x = scale0 * (rn * cn);
    o.y = scale1 * (rn * sn);
    if (!normal) {
        const float u2 = word_to_uniform(r.z), u3 = word_to_uniform(r.w);
        const float rz = sqrtf(-2.0f * logf(u2));
        float sz, cz;
        sincospif(2.0f * u3, &sz, &cz);
        o.x *= expf(fmaf(sigma_ln, rz * cz, mu_ln));
        o.y *= expf(fmaf(sigma_ln, rz * sz, mu_ln));
    }
    return o;
}

// sin and cos of an angle (a heading, a steering angle).  Cody-Waite
// reduction by pi/2 (three-part split of pi/2, each product exact inside an
// FMA) to |r| <= pi/4, then the Taylor series of sin to r^9 and of cos to
// r^10 (truncation < 3e-9 on |r| <= pi/4, below half an FP32 ulp), and the
// quadrant's swap and signs.  Angles beyond 4096 quarter turns fall back to
// the library routine.
__device__ __forceinline__ void heading_sincos(float x, float& s, float& c)
{
    const float k = rintf(x * 0.63661975f);
    if (fabsf(k) > 4096.0f) {
        sincosf(x, &s, &c);
        return;
    }
    float r = fmaf(-k, 1.5707963705062866f, x);
    r = fmaf(-k, -4.371138828673793e-08f, r);
    r = fmaf(-k, -1.7151245100058819e-15f, r);
    const float r2 = r * r;
    const float ps = r2 * fmaf(r2, fmaf(r2, fmaf(r2, 2.7557319e-06f, -1.9841270e-04f), 8.3333333e-03f),
                               -1.6666667e-01f);
    const float sr = fmaf(r, ps, r);
    const float pc = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -2.7557319e-07f, 2.4801587e-05f), -1.3888889e-03f),
                                             4.1666667e-02f), -0.5f), 1.0f);
    const int q = (int)k & 3;
    const float a = (q & 1) ? pc : sr;
    const float b = (q & 1) ? sr : pc;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// ---------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------
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

// Block reductions over NW waves; every thread gets the result.  slots
// holds at least NW doubles.
template <int NW>
__device__ __forceinline__ double block_min_d(double v, double* slots)
{
    v = wave_min_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = slots[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r = fmin(r, slots[i]);
    return r;
}

template <int NW>
__device__ __forceinline__ double block_sum_d(double v, double* slots)
{
    v = wave_sum_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = slots[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r += slots[i];
    return r;
}

// two sums with one pair of barriers; slots holds at least 2 NW doubles
template <int NW>
__device__ __forceinline__ double2 block_sum_d2(double a, double b, double* slots)
{
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        slots[threadIdx.x >> 6] = a;
        slots[NW + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    double ra = slots[0], rb = slots[NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
        ra += slots[i];
        rb += slots[NW + i];
    }
    return make_double2(ra, rb);
}

template <int NW>
__device__ __forceinline__ float block_sum_f(float v, double* slots)
{
    v = wave_sum_f(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = (double)v;
    __syncthreads();
    float r = (float)slots[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r += (float)slots[i];
    return r;
}

// Workgroup barrier that orders LDS accesses only: global stores issued
// before it may still be in flight after it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// ---------------------------------------------------------------------------
// Barrier terms.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float barrier_rcp(float h, float eps)
{
    return __builtin_amdgcn_rcpf(fmaxf(h, eps));
}

// h clamped to [eps, kHMax]: the lower end is the barrier's own cap
// B = 1/max(h, eps); the upper end (h = 1e9 m^2, 31 km) keeps the products of
// four clamped values below the FP32 range while changing B by < 1e-9.
constexpr float kHMax = 1e9f;

__device__ __forceinline__ float clamp_h(float h, float eps)
{
    return __builtin_amdgcn_fmed3f(h, eps, kHMax);
}

// sum_i 1/h_i for N clamped values, taken four at a time as one fraction
// ((a+b)cd + (c+d)ab) / (abcd) -- exact up to rounding, all terms positive,
// one reciprocal per four -- alternating between two accumulators.
template <int N>
__device__ __forceinline__ void reciprocal_sum(const float* h, float& acc, float& acc2)
{
    int k = 0;
#pragma unroll
    for (int i = 0; i + 4 <= N; i += 4, ++k) {
        const float ab = h[i] * h[i + 1], cd = h[i + 2] * h[i + 3];
        const float num = fmaf(h[i] + h[i + 1], cd, (h[i + 2] + h[i + 3]) * ab);
        float& a = (k & 1) ? acc2 : acc;
        a = fmaf(num, __builtin_amdgcn_rcpf(ab * cd), a);
    }
    constexpr int r = N % 4;
    constexpr int i = N - r;
    float& a = (k & 1) ? acc2 : acc;
    if constexpr (r == 3) {
        const float ab = h[i] * h[i + 1];
        a = fmaf(fmaf(h[i] + h[i + 1], h[i + 2], ab), __builtin_amdgcn_rcpf(ab * h[i + 2]), a);
    } else if constexpr (r == 2) {
        a = fmaf(h[i] + h[i + 1], __builtin_amdgcn_rcpf(h[i] * h[i + 1]), a);
    } else if constexpr (r == 1) {
        a += __builtin_amdgcn_rcpf(h[i]);
    }
}

// sum_i 1/h_i of N clamped values as a value (the clamped form of the layout
// bodies' obstacles that leave the pair-fraction form).
template <int N>
__device__ __forceinline__ float reciprocal_total(const float* h)
{
    float a = 0.0f, b = 0.0f;
    reciprocal_sum<N>(h, a, b);
    return a + b;
}

// Bilinear costmap sample between cell centres, clamped to the edge cells.
// (gx, gy) are continuous cell coordinates; any float input stays in bounds.
// With the four-texel layout (sdf4: for every square between four cell
// centres, its four values in one 16-byte record) a sample is one load
// instead of four scattered ones; the arithmetic, and so the result, is the
// same.
__device__ __forceinline__ float sdf_sample(const DevParams& p, float gx, float gy)
{
    const int W = p.map_w, H = p.map_h;
    gx = fminf(fmaxf(gx, 0.0f), (float)(W - 1));
    gy = fminf(fmaxf(gy, 0.0f), (float)(H - 1));
    const int i0 = min((int)floorf(gx), W - 2);
    const int j0 = min((int)floorf(gy), H - 2);
    const float fx = gx - (float)i0, fy = gy - (float)j0;
    float s00, s01, s10, s11;
    if (p.sdf4) {
        const float4 c = p.sdf4[(size_t)j0 * (W - 1) + i0];
        s00 = c.x;
        s01 = c.y;
        s10 = c.z;
        s11 = c.w;
    } else {
        const float* r0 = p.sdf + (size_t)j0 * W + i0;
        const float* r1 = r0 + W;
        s00 = r0[0];
        s01 = r0[1];
        s10 = r1[0];
        s11 = r1[1];
    }
    const float top = fmaf(fx, s01 - s00, s00);
    const float bot = fmaf(fx, s11 - s10, s10);
    return fmaf(fy, bot - top, top);
}

// ---------------------------------------------------------------------------
// Models (explicit Euler, inputs saturated inside f).  inputs() turns the
// saturated controls into the model's state-independent terms (f0, f1);
// step() advances the state with them, using the sine and cosine of the *old*
// heading.
// ---------------------------------------------------------------------------
template <int MODEL> struct Model;

template <> struct Model<MPPI_QUAD6> {
    static constexpr int NS = 6;
    // state (x, z, theta, vx, vz, omega); inputs: rotor thrust deviations from
    // hover.  f0 = (F1 + F2)/m, f1 = (F2 - F1) arm / I.
    __device__ static __forceinline__ void inputs(const DevParams& p, float s0, float s1, float& f0, float& f1)
    {
        const float hover = 0.5f * p.mass * p.gravity;
        const float F1 = hover + s0, F2 = hover + s1;
        f0 = (F1 + F2) / p.mass;
        f1 = (F2 - F1) * (p.arm / p.inertia);
    }
    __device__ static __forceinline__ void step(const DevParams& p, float* x, float f0, float f1, float sth, float cth)
    {
        const float dt = p.dt;
        const float x0 = x[0] + x[3] * dt;
        const float x1 = x[1] + x[4] * dt;
        const float x2 = x[2] + x[5] * dt;
        const float x3 = x[3] - f0 * sth * dt;
        const float x4 = x[4] + (f0 * cth - p.gravity) * dt;
        const float x5 = x[5] + f1 * dt;
        x[0] = x0; x[1] = x1; x[2] = x2; x[3] = x3; x[4] = x4; x[5] = x5;
    }
};

template <> struct Model<MPPI_QUAD5> {
    static constexpr int NS = 5;
    // Sec. V-A: state (x, z, theta, vx, vz); inputs (pitch rate, throttle).
    // f0 = pitch rate, f1 = (m g + u_t)/m.
    __device__ static __forceinline__ void inputs(const DevParams& p, float s0, float s1, float& f0, float& f1)
    {
        f0 = s0;
        f1 = (p.mass * p.gravity + s1) / p.mass;
    }
    __device__ static __forceinline__ void step(const DevParams& p, float* x, float f0, float f1, float sth, float cth)
    {
        const float dt = p.dt;
        const float x0 = x[0] + x[3] * dt;
        const float x1 = x[1] + x[4] * dt;
        const float x2 = x[2] + f0 * dt;
        const float x3 = x[3] - f1 * sth * dt;
        const float x4 = x[4] + (f1 * cth - p.gravity) * dt;
        x[0] = x0; x[1] = x1; x[2] = x2; x[3] = x3; x[4] = x4;
    }
};

template <> struct Model<MPPI_CAR> {
    static constexpr int NS = 4;
    // Sec. V-B Ackermann model: state (x, y, theta, v); inputs (steer, accel).
    // f0 = tan(phi)/L = sin(phi) / (cos(phi) L), f1 = a.
    __device__ static __forceinline__ void inputs(const DevParams& p, float s0, float s1, float& f0, float& f1)
    {
        float sp, cp;
        heading_sincos(s0, sp, cp);
        f0 = sp / (cp * p.wheelbase);
        f1 = s1;
    }
    __device__ static __forceinline__ void step(const DevParams& p, float* x, float f0, float f1, float sth, float cth)
    {
        const float dt = p.dt;
        const float v = x[3];
        const float x0 = x[0] + v * cth * dt;
        const float x1 = x[1] + v * sth * dt;
        const float x2 = x[2] + v * f0 * dt;
        const float x3 = x[3] + f1 * dt;
        x[0] = x0; x[1] = x1; x[2] = x2; x[3] = x3;
    }
};

// LDS carve-up of one rollout tile (sizes: tile_fixed_lds, then two chunks of
// per-(step, sample) slots).
struct TileLds {
    float4* obs;      // [J] (ox, oy, -r^2 + d, -r^2), local frame; d = |s_0|^2 on the
                      // vehicle's layout-form and the quadrotor's mirrored-axis tiles, else 0
    float2* U;        // [T]
    float* ref;       // [(T+1) n], local frame
    double* e;        // [kMaxTile] tile exponentials
    double* slots;    // [16] block-reduction slots
    int* work;        // [4] pool waves per SIMD, [4] the owner wave's SIMD,
                      // [5], [6] unused, [7] the bits of
                      // the largest |o|^2 over the obstacles
    // chunk slots, two buffers each (buffer b at offset b * cb, cb = cs + kXSlots):
    float4* in;       // [2][cs] per (step, sample): (f0, f1, control cost, costmap terms of the
                      // chunk two behind: sum B(sdf) or, with the indicator, the smallest sdf)
    float4* pose;     // [2][cs] per (step, sample): (x, y, cos theta, sin theta)
    float* bval;      // [2][cs] per (step, sample): fused barrier
    float2* nz;       // [T][S] the tile's noise, when it fits (else null)
    int cs;           // (step, sample) items of a full chunk
    int cb;           // buffer stride: cs + kXSlots
};

__device__ __forceinline__ TileLds carve(unsigned char* smem, int J, int T, int n, int cs, bool keep_noise)
{
    TileLds L;
    size_t off = 0;
    L.obs = reinterpret_cast<float4*>(smem + off);
    off += (size_t)obstacle_slots(J) * 16;
    L.U = reinterpret_cast<float2*>(smem + off);
    off += (size_t)T * 8;
    L.ref = reinterpret_cast<float*>(smem + off);
    off += (size_t)(T + 1) * n * 4;
    off = (off + 15) & ~(size_t)15;
    L.e = reinterpret_cast<double*>(smem + off);
    off += (size_t)kMaxTile * 8;
    L.slots = reinterpret_cast<double*>(smem + off);
    off += 16 * 8;
    L.work = reinterpret_cast<int*>(smem + off);
    off += 64;
    L.cs = cs;
    L.cb = cs + kXSlots;
    L.in = reinterpret_cast<float4*>(smem + off);
    off += (size_t)2 * L.cb * 16;
    L.pose = reinterpret_cast<float4*>(smem + off);
    off += (size_t)2 * L.cb * 16;
    L.bval = reinterpret_cast<float*>(smem + off);
    off += (size_t)2 * L.cb * 4;
    L.nz = keep_noise ? reinterpret_cast<float2*>(smem + off) : nullptr;
    return L;
}

struct X0 {
    float v[MPPI_NMAX + 2];
    uint32_t parity;     // which half of the warm-start double buffer holds U
};

constexpr int kRollWaves = kRollBlock / kWave;
constexpr int kSimdsPerCU = 4;
// s_getreg operand for the SIMD of the issuing wave: HW_ID bits [5:4].
constexpr int kHwIdSimd = (1 << 11) | (4 << 6) | 4;
constexpr int kUpdWaves = kUpdBlock / kWave;

// Sum of a float pair over the block (NW waves); every thread gets it.
template <int NW>
__device__ __forceinline__ float2 block_sum_f2(float2 v, double* slots)
{
    v.x = wave_sum_f(v.x);
    v.y = wave_sum_f(v.y);
    float* s = reinterpret_cast<float*>(slots);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        s[2 * (threadIdx.x >> 6)] = v.x;
        s[2 * (threadIdx.x >> 6) + 1] = v.y;
    }
    __syncthreads();
    float2 r = make_float2(s[0], s[1]);
#pragma unroll
    for (int i = 1; i < NW; ++i) {
        r.x += s[2 * i];
        r.y += s[2 * i + 1];
    }
    return r;
}

// Part of the fused barrier of one pose, lane sp of a group of js = 2^lg
// lanes: every shape point against obstacles sp, sp + js, sp + 2 js, ...
// below J (read from LDS).  The costmap terms are formed apart (map_terms).
//
// With e = pose - o, the heading u = (cos, sin) and its normal v, a shape
// point with body offset (a, b) gives
//   h = |e + a u + b v|^2 - r^2 = (|e|^2 - r^2) + (a^2 + 2a e.u) + (b^2 + 2b e.v).
// The fixed-P tiles use the layout of the paper's bodies (the host checks it):
// * vehicle, the corners and side midpoints of a rectangle: the two terms
//   take only the values for a = +-alpha, 0 and b = +-beta, 0, so one
//   obstacle costs 20 operations for its 8 pairs;
// * quadrotors, every point on the body axis (b = 0): h = |e|^2 - r^2 +
//   fma(2a, e.u, a^2), two operations a pair; when the points mirror about
//   the centre (the paper's frame), a mirrored pair takes three operations.
// The runtime-P tile takes any shape: h = (|e|^2 - r^2) + 2 e.d_i + |d_i|^2
// with d_i the rotated offset, one add and two FMAs a pair.
// (sa2, sb2) = 2 (a_i, b_i), ss = a_i^2 + b_i^2.
template <int MODEL, int PT>
__device__ __forceinline__ float fused_barrier_pose(const DevParams& p, const TileLds& L, int P, const float* sa2,
                                                    const float* sb2, const float* ss, float4 pose, int sp, int lg,
                                                    float omax2)
{
    constexpr int PM = PT ? PT : MPPI_PMAX;
    const float eps = p.h_eps;
    const float cs = pose.z, sn = pose.w;
    float acc = 0.0f, acc2 = 0.0f;
    const int J = p.J, js = 1 << lg;
    // Lane sp of its group of js takes obstacles sp, sp + js, ...: q of them
    // on every lane, and one more when sp < rem.  The loop count q is the
    // same on every lane, so the loop is counted in scalar registers; both
    // reads of a pair are issued before either obstacle is used.
    const int q = J >> lg, rem = J & (js - 1);
    auto run = [&](auto&& body) __attribute__((always_inline)) {
        const float4* ob = L.obs + sp;
        for (int i = 0; i + 2 <= q; i += 2) {
            const float4 o0 = ob[0], o1 = ob[js];
            ob += 2 * js;
            body(o0);
            body(o1);
        }
        if (q & 1) {
            body(ob[0]);
            ob += js;
        }
        if (sp < rem) body(ob[0]);
    };
    // The same walk for a guarded fast form: fast(o, m) gives an obstacle's
    // sum f and the smallest of the terms whose signs the guard tests, and
    // the form is exact there when m > 0 and f <= fmax; slow(o) gives the
    // clamped per-point sum.  Four obstacles an iteration share one
    // wave-uniform test (the smallest m and the largest f of the four), so
    // the loop takes no branch per obstacle; the sums are added in obstacle
    // order either way.
    auto run_guarded = [&](auto&& fast, auto&& slow, float fmax, float& sum) __attribute__((always_inline)) {
        auto one = [&](const float4 o) __attribute__((always_inline)) {
            float m;
            float f = fast(o, m);
            const bool ok = (m > 0.0f) & (f <= fmax);
            if (__builtin_expect(__ballot(!ok) != 0, 0)) {
                const float s = slow(o);
                f = ok ? f : s;
            }
            sum += f;
        };
        const float4* ob = L.obs + sp;
        int i = 0;
        for (; i + 4 <= q; i += 4) {
            const float4 o0 = ob[0], o1 = ob[js], o2 = ob[2 * js], o3 = ob[3 * js];
            ob += 4 * js;
            float m0, m1, m2, m3;
            float f0 = fast(o0, m0), f1 = fast(o1, m1), f2 = fast(o2, m2), f3 = fast(o3, m3);
            const bool ok = (fminf(fminf(m0, m1), fminf(m2, m3)) > 0.0f) & (fmaxf(fmaxf(f0, f1), fmaxf(f2, f3)) <= fmax);
            if (__builtin_expect(__ballot(!ok) != 0, 0)) {
                const bool k0 = (m0 > 0.0f) & (f0 <= fmax), k1 = (m1 > 0.0f) & (f1 <= fmax);
                const bool k2 = (m2 > 0.0f) & (f2 <= fmax), k3 = (m3 > 0.0f) & (f3 <= fmax);
                if (__ballot(!k0)) { const float s = slow(o0); f0 = k0 ? f0 : s; }
                if (__ballot(!k1)) { const float s = slow(o1); f1 = k1 ? f1 : s; }
                if (__ballot(!k2)) { const float s = slow(o2); f2 = k2 ? f2 : s; }
                if (__ballot(!k3)) { const float s = slow(o3); f3 = k3 ? f3 : s; }
            }
            sum += f0;
            sum += f1;
            sum += f2;
            sum += f3;
        }
        for (; i < q; ++i) {
            one(ob[0]);
            ob += js;
        }
        if (sp < rem) one(ob[0]);
    };
    // Pair fractions (the layout forms' fast path).  Two points whose h are
    // c + d and c - d give 1/(c+d) + 1/(c-d) = 2c/(c^2 - d^2); the bodies of
    // Sec. V split into such pairs (the vehicle's four, the quadrotor's three
    // mirrored ones plus its middle point), and their fractions meet in one:
    // one reciprocal per obstacle, no clamp.  It holds when every h of the
    // obstacle is at least gmin = max(h_eps, 1e-4) -- then B(h) = 1/h, and
    // every h lies in [gmin, 2c] -- and c is at most the form's cap, so the
    // products of all the h stay inside the FP32 range.  Any other obstacle
    // takes the clamped per-point form.  `half` sums c/q, half of each
    // fraction.
    const float gmin = fmaxf(eps, 1e-4f);
    float half = 0.0f;
    if constexpr (PT != 0 && MODEL == MPPI_CAR) {
        static_assert(PT == 8, "vehicle layout: 8 points");
        // point 0 is (a, b); o.z = -r^2 + a^2 + b^2, so C = |e|^2 - r^2 + a^2 +
        // b^2 takes two operations, and with P = 2a e.u, Q = 2b e.v the
        // corners are (C +- P) +- Q, the side midpoints C +- P - b^2 and
        // C - a^2 +- Q.  Pairs: (C+P) +- Q, (C-P) +- Q, (C-b^2) +- P and
        // (C-a^2) +- Q; the smallest h is C - |P| - |Q| (a corner),
        // C - b^2 - |P| or C - a^2 - |Q|, the largest at most 2C.
        // Cap: C <= 2e4, so 8 values of h <= 4e4 multiply below 7e36.
        constexpr float kCap = 2.0e4f;
        const float AA = ss[4], BB = ss[6];
        const float cu = sa2[0] * cs, su = sa2[0] * sn, cv = sb2[0] * cs, sv = sb2[0] * sn;
        // NOCAP: C <= |pose - o|^2 + a^2 + b^2 <= 2 |pose|^2 + 2 max_j |o_j|^2 +
        // a^2 + b^2 is below the cap on every lane of the unit, so no obstacle
        // needs the cap term in the guard
        auto body = [&](auto nocap_tag) __attribute__((always_inline)) {
            constexpr bool NOCAP = decltype(nocap_tag)::value;
            run([&](const float4 o) __attribute__((always_inline)) {
                const float ex = pose.x - o.x, ey = pose.y - o.y;
                const float C = fmaf(ex, ex, fmaf(ey, ey, o.z));
                const float Pu = fmaf(ex, cu, ey * su), Qv = fmaf(ey, cv, -ex * sv);
                const float X1 = C + Pu, X2 = C - Pu, X3 = C - BB, X4 = C - AA;
                const float aP = fabsf(Pu), aQ = fabsf(Qv);
                const float g = NOCAP ? fminf(fminf(C - aP - aQ, X3 - aP), X4 - aQ)
                                      : fminf(fminf(C - aP - aQ, X3 - aP), fminf(X4 - aQ, (kCap + gmin) - C));
                const float P2 = Pu * Pu, Q2 = Qv * Qv;
                const float q1 = fmaf(X1, X1, -Q2), q2 = fmaf(X2, X2, -Q2);
                const float q3 = fmaf(X3, X3, -P2), q4 = fmaf(X4, X4, -Q2);
                const float n12 = fmaf(X1, q2, X2 * q1), d12 = q1 * q2;
                const float n34 = fmaf(X3, q4, X4 * q3), d34 = q3 * q4;
                float f = fmaf(n12, d34, n34 * d12) * __builtin_amdgcn_rcpf(d12 * d34);
                // (a wave-uniform branch: the clamped form only when a lane needs it)
                if (__builtin_expect(__ballot(g < gmin) != 0, 0)) {
                    float h[8] = {X1 + Qv, X1 - Qv, X2 + Qv, X2 - Qv, X1 - BB, X2 - BB, X4 + Qv, X4 - Qv};
#pragma unroll
                    for (int i = 0; i < 8; ++i) h[i] = clamp_h(h[i], eps);
                    const float slow = 0.5f * reciprocal_total<8>(h);
                    f = g >= gmin ? f : slow;
                }
                half += f;
            });
        };
        const float bound = fmaf(2.0f, fmaf(pose.x, pose.x, pose.y * pose.y), omax2) + ss[0];
        if (__ballot(!(bound <= kCap)) == 0) body(std::true_type{});
        else body(std::false_type{});
    } else if constexpr (PT != 0) {
        static_assert(PT == 7, "quadrotor layout: 7 points");
        // The mirrored-axis form: a_{6-i} = -a_i, and |a_0| is the largest
        // |a_i| (the host checks both): pair i shares c_i = |e|^2 - r^2 + a_i^2
        // and its two points differ in the sign of d_i = 2 a_i e.u.  o.z =
        // -r^2 + a_0^2, so c_0 = b0 = |e|^2 + o.z itself and c_i = b0 + (a_i^2 -
        // a_0^2) <= b0.  It runs when the middle point is the centre (a_3 = 0,
        // the paper's body: h_m = b0 - a_0^2 <= b0) and no obstacle of this unit
        // can pass the cap: every h is then at most 2 b0 <= 2e5, and 7 of them
        // multiply below 1.3e37.  The cap holds for the whole unit when
        // 2 |pose|^2 + 2 max_j |o_j|^2 + a_0^2 <= 1e5 on every lane, since
        // b0 <= |pose - o|^2 + a_0^2.  Any other unit, or body, runs the
        // clamped per-point form below.
        constexpr float kCap = 1.0e5f;
        const bool mirrored = p.shape_kind == kShapeMirroredAxis;
        bool fast = false;
        if (mirrored && sa2[3] == 0.0f) {
            const float bound = fmaf(2.0f, fmaf(pose.x, pose.x, pose.y * pose.y), omax2) + ss[0];
            fast = __ballot(!(bound <= kCap)) == 0;
        }
        if (fast) {
            const float A0 = sa2[0], D1 = ss[1] - ss[0], D2 = ss[2] - ss[0];
            const float DM = -ss[0];
            // The heading projection enters scaled by A0 = 2 a_0: w = A0 e.u,
            // so pair 0's q is b0^2 - w^2 with no coefficient, and pair i's
            // is b_i^2 - (A_i / A0)^2 w^2.  (A0 = 0 only for a body whose
            // points all sit at its centre: then every A_i is 0.)
            const float R1 = A0 != 0.0f ? sa2[1] / A0 : 0.0f, R2 = A0 != 0.0f ? sa2[2] / A0 : 0.0f;
            const float nK1 = -(R1 * R1), nK2 = -(R2 * R2);
            const float csw = A0 * cs, snw = A0 * sn;
            // The guard reads the fraction itself: h_m = b0 - a_0^2 is the
            // smallest c_i, so h_m > 0 and q_i = (c_i - d_i)(c_i + d_i) > 0 put
            // every h above 0; then f = (1/2) sum 1/h <= 1/(2 gmin) puts every
            // h at or above gmin.  (A NaN f fails the comparison.)
            // (the middle point enters as hd = 2 h_m, so that pair 2 and the
            // middle point meet as b2/q2 + 1/hd = (b2 hd + q2)/(q2 hd))
            const float fcap = 0.5f / gmin, DM2 = 2.0f * DM;
            auto fast_sum = [&](const float4 o, float& m) __attribute__((always_inline)) {
                const float ex = pose.x - o.x, ey = pose.y - o.y;
                const float b0 = fmaf(ex, ex, fmaf(ey, ey, o.z));
                const float w = fmaf(ex, csw, ey * snw);
                const float b1 = b0 + D1, b2 = b0 + D2;
                const float hd = fmaf(2.0f, b0, DM2);
                const float w2 = w * w;
                const float q0 = fmaf(b0, b0, -w2), q1 = fmaf(b1, b1, nK1 * w2);
                const float q2 = fmaf(b2, b2, nK2 * w2);
                const float n01 = fmaf(b0, q1, b1 * q0), d01 = q0 * q1;
                const float n2m = fmaf(b2, hd, q2), d2m = q2 * hd;
                m = fminf(fminf(q0, q1), fminf(q2, hd));
                return fmaf(n01, d2m, n2m * d01) * __builtin_amdgcn_rcpf(d01 * d2m);
            };
            auto clamped_sum = [&](const float4 o) __attribute__((always_inline)) {
                const float ex = pose.x - o.x, ey = pose.y - o.y;
                const float b0 = fmaf(ex, ex, fmaf(ey, ey, o.z));
                const float w = fmaf(ex, csw, ey * snw);
                const float b1 = b0 + D1, b2 = b0 + D2, hm = b0 + DM;
                float h[7] = {b0 + w, fmaf(R1, w, b1), fmaf(R2, w, b2), hm, fmaf(-R2, w, b2), fmaf(-R1, w, b1), b0 - w};
#pragma unroll
                for (int i = 0; i < 7; ++i) h[i] = clamp_h(h[i], eps);
                return 0.5f * reciprocal_total<7>(h);
            };
            run_guarded(fast_sum, clamped_sum, fcap, half);
        } else {
            // (on the mirrored-axis tile o.z carries the a_0^2 offset)
            float ssx[PM];
#pragma unroll
            for (int i = 0; i < PM; ++i) ssx[i] = mirrored ? ss[i] - ss[0] : ss[i];
            run([&](const float4 o) __attribute__((always_inline)) {
                const float ex = pose.x - o.x, ey = pose.y - o.y;
                const float ee = fmaf(ex, ex, fmaf(ey, ey, o.z));
                const float pu = fmaf(ex, cs, ey * sn);
                float h[PM];
#pragma unroll
                for (int i = 0; i < PM; ++i) h[i] = clamp_h(ee + fmaf(sa2[i], pu, ssx[i]), eps);
                reciprocal_sum<PM>(h, acc, acc2);
            });
        }
    } else {
        float tx[PM], ty[PM];       // 2 d_i
#pragma unroll
        for (int i = 0; i < PM; ++i) {
            tx[i] = fmaf(sa2[i], cs, -sb2[i] * sn);
            ty[i] = fmaf(sa2[i], sn, sb2[i] * cs);
        }
        run([&](const float4 o) __attribute__((always_inline)) {
            const float ex = pose.x - o.x, ey = pose.y - o.y;
            const float ee = fmaf(ex, ex, fmaf(ey, ey, o.z));
#pragma unroll
            for (int i = 0; i < PM; ++i) {
                if (i < P) acc += __builtin_amdgcn_rcpf(clamp_h(fmaf(ex, tx[i], fmaf(ey, ty[i], ee + ss[i])), eps));
            }
        });
    }
    acc += acc2;
    acc = fmaf(2.0f, half, acc);
    return acc;
}

// The costmap terms of one pose (every shape point): sum_i B(sdf(p_i)), or
// with the indicator the smallest sdf(p_i).  Four shape points' reads are in
// flight at a time; the body offsets come from the parameter block (uniform
// scalar loads), so the loop holds no per-point registers.
template <int PT, bool IND>
__device__ __forceinline__ float map_terms(const DevParams& p, int P, float4 pose, float inv_res, float offx,
                                           float offy)
{
    constexpr int G = 4;
    const int np = PT ? PT : P;
    const float cs = pose.z, sn = pose.w;
    float acc = IND ? INFINITY : 0.0f;
#pragma unroll 1
    for (int i0 = 0; i0 < np; i0 += G) {
        float v[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int i = min(i0 + j, np - 1);
            const float a = p.shape[i][0], b = p.shape[i][1];
            const float px = pose.x + fmaf(a, cs, -b * sn);
            const float py = pose.y + fmaf(a, sn, b * cs);
            v[j] = sdf_sample(p, fmaf(px, inv_res, offx), fmaf(py, inv_res, offy));
        }
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (i0 + j < np) acc = IND ? fminf(acc, v[j]) : acc + barrier_rcp(v[j], p.h_eps);
    }
    return acc;
}

// The comparison controllers' constraint test of one pose (Sec. IV-A's
// weighted indicator): lane sp of a group of js = 2^lg lanes returns the
// smallest h of every shape point against obstacles sp, sp + js, ... (+inf
// when it has none); with the costmap's smallest value (map_terms), the
// group's minimum decides whether the pose violates a constraint (h < 0).
// General form h = (|e|^2 - r^2) + 2 e.d_i + |d_i|^2, as the runtime-P
// barrier takes it.
__device__ __forceinline__ float clearance_pose(const DevParams& p, const TileLds& L, int P, const float* sa2,
                                                const float* sb2, const float* ss, float4 pose, int sp, int lg)
{
    constexpr int PM = MPPI_PMAX;
    const float cs = pose.z, sn = pose.w;
    const int J = p.J, js = 1 << lg;
    float lo = INFINITY, lo2 = INFINITY;
    float tx[PM], ty[PM];       // 2 d_i
#pragma unroll
    for (int i = 0; i < PM; ++i) {
        tx[i] = fmaf(sa2[i], cs, -sb2[i] * sn);
        ty[i] = fmaf(sa2[i], sn, sb2[i] * cs);
    }
    for (int j = sp; j < J; j += js) {
        const float4 o = L.obs[j];
        const float ex = pose.x - o.x, ey = pose.y - o.y;
        const float ee = fmaf(ex, ex, fmaf(ey, ey, o.z));
#pragma unroll
        for (int i = 0; i < PM; i += 2) {
            if (i < P) lo = fminf(lo, fmaf(ex, tx[i], fmaf(ey, ty[i], ee + ss[i])));
            if (i + 1 < P) lo2 = fminf(lo2, fmaf(ex, tx[i + 1], fmaf(ey, ty[i + 1], ee + ss[i + 1])));
        }
    }
    lo = fminf(lo, lo2);
    return lo;
}

// ---------------------------------------------------------------------------
// One tile of S samples: rollout and the tile's softmax partials.
// PT = compile-time number of shape points (0: runtime P <= MPPI_PMAX; the
// fixed-P tiles use the layout form of the paper's bodies).  The standalone
// and the batched kernels run the same tile.
//
// The horizon is cut into chunks of tc steps that flow through a pipeline of
// workgroup-wide stages.  In stage k:
//   * the waves that own samples (lane tid < S) first run the barrier-state
//     recursion over chunk k-2 and then integrate the dynamics of chunk k --
//     the two sequential parts, one lane per sample;
//   * the other waves draw the noise and inputs of chunk k+1;
//   * then the pool waves take units of the fused-barrier work of chunk k-1,
//     shared out by SIMD (see barrier_chunk).
// Every (step, sample) of a chunk is split over nsp adjacent lanes; lane sp
// of the group takes obstacles sp, sp + nsp, ..., so a wave's lanes read one
// contiguous run of obstacles at a time; the nsp partial sums meet by wave
// shuffles.
// Inputs, poses and barrier values are double-buffered by chunk parity.
// ---------------------------------------------------------------------------
template <int MODEL, int S, int PT, bool IND, bool MAP>
__device__ void rollout_tile(const DevParams& p, const int tile, const X0& xs, unsigned char* smem)
{
    static_assert(!IND || PT == 0, "the indicator runs on the runtime-P tile");
    constexpr int NS = Model<MODEL>::NS;
    constexpr int PM = PT ? PT : MPPI_PMAX;
    constexpr int DW = (S + kWave - 1) / kWave;     // waves that own samples
    constexpr int POOL0 = DW * kWave;               // first thread of the noise pool
    static_assert(S >= 16 && S <= kMaxTile && (S & (S - 1)) == 0, "tile size");
    static_assert(POOL0 < kRollBlock, "the noise pool needs a wave");
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const int J = p.J, T = p.T, K = p.K, Kp = p.Kp;
    const int P = PT ? PT : p.P;
    // the host only configures tiles whose chunk holds at least one step
    const int tc = tile_chunk_steps(J, T, NS, S);
    // chunk 0 is shorter: its dynamics run while the barrier pool has no
    // poses yet
    const int tc0 = min(tile_first_chunk(T), tc);
    const int nch = 1 + (T - tc0 + tc - 1) / tc;
    const bool keep_noise = tile_keeps_noise(J, T, NS, S);
    const TileLds L = carve(smem, J, T, NS, tc * S, keep_noise);
    const CtrlState* cs_in = p.st;
    const float S_e = cs_in->S_e;
    const uint64_t ctr = cs_in->counter;
    const uint32_t c_lo = (uint32_t)ctr, c_hi = (uint32_t)(ctr >> 32);

    // the Philox words of sample kk at step t (Sec. IV-C: counter (k, t, iteration))
    // (the key words, uniform over the tile, pass through an empty asm
    // statement, so that the twenty round keys are formed per item by scalar
    // adds instead of being held in scalar registers across the whole stage
    // loop, where they crowded out other values into reloads)
    auto philox_at = [&](int kk, int t) __attribute__((always_inline)) {
        uint32_t k0 = __builtin_amdgcn_readfirstlane(p.seed_lo), k1 = __builtin_amdgcn_readfirstlane(p.seed_hi);
        asm volatile("" : "+s"(k0), "+s"(k1));
        return philox4x32_10(make_uint4((uint32_t)kk, (uint32_t)t, c_lo, c_hi), k0, k1);
    };
    // Chunk 0's words are drawn first, on the upper half of the workgroup (two
    // items per thread), while the staging below waits on memory.
    const int items0 = tc0 * S;
    const int j0 = tid - kRollBlock / 2;
    uint4 w0 = make_uint4(0u, 0u, 0u, 0u), w1 = w0;
    if (j0 >= 0 && j0 < items0) w0 = philox_at(tile * S + (j0 & (S - 1)), j0 / S);
    if (j0 >= 0 && j0 + kRollBlock / 2 < items0)
        w1 = philox_at(tile * S + ((j0 + kRollBlock / 2) & (S - 1)), (j0 + kRollBlock / 2) / S);

    const float* Uin = p.U + (size_t)(xs.parity & 1u) * T * kM;

    // ---- staging: local frame centred on the start position ----
    const double ox = (double)xs.v[0], oy = (double)xs.v[1];
    float omax_mine = 0.0f;     // this thread's largest |o|^2 (local frame), for the barrier's cap bound
    float omax2 = 0.0f;         // 2 max_j |o_j|^2, known from the first stage on
    {
        // the vehicle's layout form and the quadrotor's mirrored-axis form
        // offset |e|^2 - r^2 by |s_0|^2 (third word); the fourth word keeps
        // -r^2
        const bool offset = PT != 0 && (MODEL == MPPI_CAR || p.shape_kind == kShapeMirroredAxis);
        const double s00 = (double)p.shape[0][0], s01 = (double)p.shape[0][1];
        const double d0 = offset ? s00 * s00 + s01 * s01 : 0.0;
        for (int j = tid; j < J; j += kRollBlock) {
            const double cx = (double)p.obs[3 * j], cy = (double)p.obs[3 * j + 1], r = (double)p.obs[3 * j + 2];
            const float4 o = make_float4((float)(cx - ox), (float)(cy - oy), (float)(d0 - r * r), (float)(-(r * r)));
            L.obs[j] = o;
            if constexpr (PT != 0) omax_mine = fmaxf(omax_mine, fmaf(o.x, o.x, o.y * o.y));
        }
    }
    if (tid < 8) L.work[tid] = 0;
    for (int t = tid; t < T; t += kRollBlock) L.U[t] = make_float2(Uin[2 * t], Uin[2 * t + 1]);
    for (int i = tid; i < (T + 1) * NS; i += kRollBlock) {
        const int a = i % NS;
        const float v = p.xref[i];
        L.ref[i] = a == 0 ? (float)((double)v - ox) : a == 1 ? (float)((double)v - oy) : v;
    }
    float inv_res = 0.0f, offx = 0.0f, offy = 0.0f;
    // MAP: the controller has a costmap (p.sdf set); the tiles without one
    // carry none of its code
    if constexpr (MAP) {
        inv_res = (float)(1.0 / (double)p.map_res);
        offx = (float)((ox - (double)p.map_x0) / (double)p.map_res - 0.5);
        offy = (float)((oy - (double)p.map_y0) / (double)p.map_res - 0.5);
    }
    lds_barrier();

    // The barrier units of a stage are shared out by SIMD (see
    // barrier_chunk): each wave learns its SIMD and, outside the owner waves,
    // its slot among the pool waves of that SIMD.
    const int simd = __builtin_amdgcn_s_getreg(kHwIdSimd);
    int pslot = 0;
    if (lane == 0) {
        if (wave >= DW) pslot = atomicAdd(&L.work[simd], 1);
        else if (wave == 0) L.work[4] = simd;
    }
    pslot = __builtin_amdgcn_readfirstlane(pslot);
    int my_pool = 1;                    // pool waves on this wave's SIMD
    int my_classes = 0;                 // bit cl: this wave's SIMD serves unit class cl

    float beta0 = 0.0f, beta_d = 0.0f;      // fused B(h(x0)), fused B(h(x_d)), formed in stage 1

    // ---- setup: lanes 0..S-1 own one sample each ----
    const bool owner = tid < S;
    const int k = tile * S + tid;
    const bool valid = owner && k < K;

    const float sqS = sqrtf(S_e);
    const float scale0 = sqS * p.sigma[0], scale1 = sqS * p.sigma[1];
    const bool normal_law = p.sampling == MPPI_SAMPLE_NORMAL;
    const float cw0 = p.sigma[0] > 0.0f ? p.gamma_u / (S_e * p.sigma[0] * p.sigma[0]) : 0.0f;
    const float cw1 = p.sigma[1] > 0.0f ? p.gamma_u / (S_e * p.sigma[1] * p.sigma[1]) : 0.0f;

    float x[NS];
    x[0] = 0.0f;
    x[1] = 0.0f;
#pragma unroll
    for (int a = 2; a < NS; ++a) x[a] = xs.v[a];
    float sth, cth;
    heading_sincos(x[2], sth, cth);
    // eq. barrier_update is linear in beta, so beta_t = bv_t + c_t with the
    // sample-dependent part bv_t = b_t + gamma_B bv_{t-1} (bv_0 = beta_0) and
    // the common part c_t = gamma_B (c_{t-1} - beta_d) (c_0 = 0), whose sum is
    // -beta_d gamma_B/(1-gamma_B) (T - gamma_B (1-gamma_B^T)/(1-gamma_B)).
    // The common part's cost R_B sum_t c_t is the same for every sample and is
    // added in FP64 (cshift), so a large beta_d cannot swamp the FP32 sums;
    // the host forms its factor R_B sum_t c_t / beta_d once per controller.
    float beta = 0.0f;
    float S_hi = 0.0f, S_lo = 0.0f;

    float sa2[PM], sb2[PM], ss[PM];       // 2 s_i and |s_i|^2
#pragma unroll
    for (int i = 0; i < PM; ++i) {
        const float a = (PT || i < P) ? p.shape[i][0] : 0.0f;
        const float b = (PT || i < P) ? p.shape[i][1] : 0.0f;
        sa2[i] = 2.0f * a;
        sb2[i] = 2.0f * b;
        ss[i] = fmaf(a, a, b * b);
    }

    auto chunk_t0 = [&](int c) { return c == 0 ? 0 : tc0 + (c - 1) * tc; };
    auto chunk_len = [&](int c) { return c == 0 ? tc0 : min(tc, T - chunk_t0(c)); };

    // the noise of sample kk at step t (Sec. IV-C mixture, scaled per Alg. 1)
    auto noise_of = [&](uint4 r) __attribute__((always_inline)) {
        return nln_pair(r, scale0, scale1, p.mu_ln, p.sigma_ln, normal_law);
    };
    auto noise_at = [&](int kk, int t) __attribute__((always_inline)) { return noise_of(philox_at(kk, t)); };

    // the inputs of item idx = (t - t0) S + s of a chunk from its noise z
    auto store_input = [&](float4* dst, int idx, int t, int s, float2 z) __attribute__((always_inline)) {
        const float2 u = L.U[t];
        const float v0 = u.x + z.x, v1 = u.y + z.y;
        const float s0 = fminf(fmaxf(v0, p.u_min[0]), p.u_max[0]);
        const float s1 = fminf(fmaxf(v1, p.u_min[1]), p.u_max[1]);
        float f0, f1;
        Model<MODEL>::inputs(p, s0, s1, f0, f1);
        const float ccost = cw0 * u.x * v0 + cw1 * u.y * v1;
        if constexpr (MAP) {
            // (.w is left alone: it carries the costmap terms of the chunk
            // two behind, from the pool's map units to the barrier-state
            // stage)
            float* d = reinterpret_cast<float*>(dst + idx);
            d[0] = f0;
            d[1] = f1;
            d[2] = ccost;
        } else {
            dst[idx] = make_float4(f0, f1, ccost, 0.0f);
        }
        if (keep_noise) L.nz[t * S + s] = z;
    };

    // inputs of every (step, sample) of chunk c, over threads [first, block)
    auto inputs_chunk = [&](int c, int first) __attribute__((always_inline)) {
        const int t0 = chunk_t0(c), items = chunk_len(c) * S;
        float4* dst = L.in + (c & 1) * L.cb;
        for (int idx = tid - first; idx < items; idx += kRollBlock - first) {
            const int s = idx & (S - 1), t = t0 + idx / S;
            store_input(dst, idx, t, s, noise_at(tile * S + s, t));
        }
    };

    // dynamics of chunk c (owner lanes): poses to LDS, tracking + control cost
    auto dynamics_chunk = [&](int c) __attribute__((always_inline)) {
        const int t0 = chunk_t0(c), n = chunk_len(c);
        const float4* src = L.in + (c & 1) * L.cb;
        float4* pz = L.pose + (c & 1) * L.cb;
        float4 nin = src[tid];
        for (int tt = 0; tt < n; ++tt) {
            const float4 in = nin;
            if (tt + 1 < n) nin = src[(tt + 1) * S + tid];
            const float* rf = L.ref + (t0 + tt + 1) * NS;
            float ref[NS];
#pragma unroll
            for (int a = 0; a < NS; ++a) ref[a] = rf[a];
            Model<MODEL>::step(p, x, in.x, in.y, sth, cth);
            heading_sincos(x[2], sth, cth);
            pz[tt * S + tid] = make_float4(x[0], x[1], cth, sth);
            float q = 0.0f;
#pragma unroll
            for (int a = 0; a < NS; ++a) {
                const float d = x[a] - ref[a];
                q = fmaf(p.Q[a], d * d, q);
            }
            two_sum_acc(S_hi, S_lo, q + in.z);
        }
    };

    // barrier-state recursion over chunk c (owner lanes) and its cost; with
    // the indicator, the weighted count of its steps that violate a
    // constraint (the pool left each step's smallest h in bval)
    auto beta_chunk = [&](int c) __attribute__((always_inline)) {
        const int n = chunk_len(c);
        const float* bv = L.bval + (c & 1) * L.cb;
        [[maybe_unused]] const float4* mv = L.in + (c & 1) * L.cb;
        float nb = bv[tid];
        for (int tt = 0; tt < n; ++tt) {
            float b = nb;
            if constexpr (MAP) b = IND ? fminf(b, mv[tt * S + tid].w) : b + mv[tt * S + tid].w;
            if (tt + 1 < n) nb = bv[(tt + 1) * S + tid];
            if constexpr (IND) {
                if (b < 0.0f) two_sum_acc(S_hi, S_lo, p.collision_weight);
            } else {
                beta = fmaf(p.gamma_b, beta, b);
                two_sum_acc(S_hi, S_lo, p.r_b * beta);
            }
        }
    };

    // The barrier splits of the tile's chunks (tile_lg_pack): set by the host
    // in the parameter block, else formed here.
    const int lg_pack = (p.lg_pack & kLgPackSet) ? p.lg_pack : tile_lg_pack(J, T, NS, S, P);

    // Fused barrier of every (step, sample) of chunk c, in units of one wave.
    // The units are shared out by SIMD, not taken first come first served: a SIMD's older waves win the issue arbitration, so under a
    // shared counter they took the most units and the SIMD of the owner wave
    // finished last.  Unit u belongs to class u mod 4; class cl is served by
    // the SIMD of rank 3 - cl from the owner wave's SIMD (the class that is
    // one unit short, when there is one, goes to the owner's SIMD), or,
    // should that SIMD have no pool wave, by the next one that has.  Within a
    // SIMD the pool waves take the class's units round-robin by slot; the
    // owner waves take none.  Which wave computes a unit never changes its
    // arithmetic.
    auto barrier_chunk = [&](int c) __attribute__((always_inline)) {
        const int items = chunk_len(c) * S;
        // with the barrier state, chunk 0 also takes the poses of x0 and x_d
        // (its extra slots)
        const int xitems = (!IND && c == 0) ? kXSlots : 0;
        const int all = items + xitems;
        const int lg = (lg_pack >> (c == 0 ? 0 : c == nch - 1 ? 8 : 4)) & 15;
        const int nsp = 1 << lg;
        // obstacle units (nsp lanes per item), then, with a costmap, map units
        // (one item per lane, every shape point: their reads all in flight at
        // once, away from the long obstacle units)
        const int ounits = ((all << lg) + kWave - 1) / kWave;
        const int units = ounits + (MAP ? (all + kWave - 1) / kWave : 0);
        const float4* pz = L.pose + (c & 1) * L.cb;
        float* bv = L.bval + (c & 1) * L.cb;
        [[maybe_unused]] float4* mv = L.in + (c & 1) * L.cb;
        auto unit = [&](int u) __attribute__((always_inline)) {
            if constexpr (MAP) {
                if (u >= ounits) {
                    const int item = (u - ounits) * kWave + lane;
                    if (item < all) mv[item].w = map_terms<PT, IND>(p, P, pz[item], inv_res, offx, offy);
                    return;
                }
            }
            const int g = u * kWave + lane;
            const int item = g >> lg, sp = g & (nsp - 1);
            float part = IND ? INFINITY : 0.0f;
            if constexpr (IND) {
                if (item < items) part = clearance_pose(p, L, P, sa2, sb2, ss, pz[item], sp, lg);
                for (int m = 1; m < nsp; m <<= 1) part = fminf(part, __shfl_xor(part, m));
                if (sp == 0 && item < items) bv[item] = part;
            } else {
                if (item < all) part = fused_barrier_pose<MODEL, PT>(p, L, P, sa2, sb2, ss, pz[item], sp, lg, omax2);
                for (int m = 1; m < nsp; m <<= 1) part += __shfl_xor(part, m);
                if (sp == 0 && item < all) bv[item] = part;
            }
        };
        if (wave < DW) return;
        // the classes this SIMD serves, in turn (one copy of the unit code)
        for (int cls = my_classes; cls != 0; cls &= cls - 1) {
            const int cl = __builtin_ctz(cls);
            for (int u = cl + kSimdsPerCU * pslot; u < units; u += kSimdsPerCU * my_pool) unit(u);
        }
    };

    // the largest |o|^2 over the obstacles (work[7] was cleared before the
    // staging barrier; non-negative floats order as their bit patterns)
    if constexpr (PT != 0) {
        if (omax_mine > 0.0f) atomicMax(&L.work[7], __float_as_int(omax_mine));
    }
    // The first chunk's inputs, on the upper half of the workgroup, from the
    // words drawn at entry (and drawn here for any item beyond two per thread).
    if (j0 >= 0) {
        constexpr int H = kRollBlock / 2;
        if (j0 < items0) store_input(L.in, j0, j0 / S, j0 & (S - 1), noise_of(w0));
        if (j0 + H < items0) store_input(L.in, j0 + H, (j0 + H) / S, (j0 + H) & (S - 1), noise_of(w1));
        for (int idx = j0 + 2 * H; idx < items0; idx += H)
            store_input(L.in, idx, idx / S, idx & (S - 1), noise_at(tile * S + (idx & (S - 1)), idx / S));
    }
    lds_barrier();
    if constexpr (PT != 0) omax2 = 2.0f * __int_as_float(L.work[7]);
    // (the SIMD counts are final: the barriers since have synchronised)
    {
        my_pool = __builtin_amdgcn_readfirstlane(max(L.work[simd], 1));
        const int osimd = __builtin_amdgcn_readfirstlane(L.work[4]);
        int mine = 0;
#pragma unroll
        for (int cl = 0; cl < kSimdsPerCU; ++cl) {
            int sv = (osimd + kSimdsPerCU - 1 - cl) & (kSimdsPerCU - 1);
            for (int t = 0; t < kSimdsPerCU && L.work[sv] == 0; ++t) sv = (sv + 1) & (kSimdsPerCU - 1);
            if (sv == simd) mine |= 1 << cl;
        }
        my_classes = __builtin_amdgcn_readfirstlane(mine);
    }
    for (int st_k = 0; st_k <= nch + 1; ++st_k) {
        if (wave < DW) {
            if (!IND && owner && st_k == 2) {
                // beta_0 and beta_d, formed in stage 1 in chunk 0's extra
                // slots (buffer 0 is next written in stage 3)
                const int i0 = tc0 * S;
                beta0 = L.bval[i0] + (MAP ? L.in[i0].w : 0.0f);
                beta_d = L.bval[i0 + 1] + (MAP ? L.in[i0 + 1].w : 0.0f);
                beta = beta0;
            }
            if (owner && st_k >= 2) beta_chunk(st_k - 2);
            if (owner && st_k < nch) dynamics_chunk(st_k);
        } else {
            if (!IND && st_k == 0 && wave == kRollWaves - 1 && lane < kXSlots) {
                // beta_0 and beta_d are the fused barriers of the poses of x0
                // and x_d = x_ref[T]: chunk 0 carries them in its two extra
                // slots, so the barrier units of stage 1 form them (this wave
                // has no noise to draw in stage 0)
                const float* xd = L.ref + T * NS;
                float sn, cn;
                heading_sincos(lane == 0 ? xs.v[2] : xd[2], sn, cn);
                L.pose[tc0 * S + lane] = lane == 0 ? make_float4(0.0f, 0.0f, cn, sn) : make_float4(xd[0], xd[1], cn, sn);
            }
            if (st_k + 1 < nch) inputs_chunk(st_k + 1, POOL0);
        }
        if (st_k >= 1 && st_k <= nch) barrier_chunk(st_k - 1);
        lds_barrier();
    }
    const double cshift = (double)beta_d * p.beta_d_weight;
    if (owner) {
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
    // (global stores come after the block reductions, whose barriers would
    // otherwise wait for them)
    const double Sd = ((double)S_hi + (double)S_lo) + cshift;
    const bool ok = valid && isfinite(Sd);
    auto wants64 = [&](double rho) {
        return isfinite(rho) && (p.normaliser == MPPI_NORM_ON ||
                                 (p.normaliser == MPPI_NORM_AUTO && fabs(rho) >= 1024.0 * (double)p.lambda));
    };
    auto weight = [&](double rho, bool u64) {
        double ek = 0.0;
        if (ok) {
            const double d = (Sd - rho) / (double)p.lambda;
            ek = u64 ? exp(-d) : (double)expf(-(float)d);
        }
        return ek;
    };
    double rho_b, eta_b, ek = 0.0;
    if constexpr (DW == 1) {
        // every sample is on wave 0: reduce over its first S lanes and
        // publish through LDS behind one barrier
        if (wave == 0) {
            double m = ok ? Sd : INFINITY;
#pragma unroll
            for (int o = S / 2; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o));
            m = __shfl(m, 0);
            const bool u64 = wants64(m);
            ek = weight(m, u64);
            if (owner) L.e[tid] = ek;
            double es;
            if (u64) {
                es = ek;
#pragma unroll
                for (int o = S / 2; o >= 1; o >>= 1) es += __shfl_xor(es, o);
            } else {
                float ef = (float)ek;
#pragma unroll
                for (int o = S / 2; o >= 1; o >>= 1) ef += __shfl_xor(ef, o);
                es = (double)ef;
            }
            if (tid == 0) {
                L.slots[0] = m;
                L.slots[1] = es;
            }
        }
        lds_barrier();
        rho_b = L.slots[0];
        eta_b = L.slots[1];
    } else {
        rho_b = block_min_d<kRollWaves>(ok ? Sd : INFINITY, L.slots);
        ek = weight(rho_b, wants64(rho_b));
        if (owner) L.e[tid] = ek;
        if (wants64(rho_b)) eta_b = block_sum_d<kRollWaves>(ek, L.slots);
        else eta_b = (double)block_sum_f<kRollWaves>((float)ek, L.slots);
    }
    const bool any = isfinite(rho_b);
    const bool use64 = wants64(rho_b);

    // N_b[2t + c] = sum over the tile's samples of e_k du[t][c][k].  The
    // noise is never stored in device memory on the way: it is kept in LDS
    // when it fits and otherwise drawn again from its counter, bit-identical
    // to the inputs phase (and written out here only when the controller
    // exports it).  TPT consecutive threads share a step t, each
    // summing every TPT-th sample in order, then combining across the TPT
    // threads.
    // (at least eight samples per thread: fewer shuffle rounds)
    int tpt = 1;
    while (tpt < 64 && (tpt << 1) * T <= kRollBlock && (tpt << 1) * 8 <= S) tpt <<= 1;
    const int steps_per_pass = kRollBlock / tpt;
    const int part = tid & (tpt - 1);
    const int k0 = tile * S;
    const int nk = min(S, K - k0);
    const bool store_du = p.export_noise != 0;
    // with smoothing, the unsmoothed sums gather in the (spent) chunk inputs
    const bool smooth = p.sgf_m > 0;
    double* nb = reinterpret_cast<double*>(L.in);
    for (int q0 = 0; q0 < T; q0 += steps_per_pass) {
        const int t = q0 + tid / tpt;
        double o0, o1;
        if (use64) {
            double a0 = 0.0, a1 = 0.0;
            if (t < T) {
                for (int s = part; s < nk; s += tpt) {
                    const float2 z = keep_noise ? L.nz[t * S + s] : noise_at(k0 + s, t);
                    if (store_du) {
                        p.du[(size_t)(2 * t) * Kp + k0 + s] = z.x;
                        p.du[(size_t)(2 * t + 1) * Kp + k0 + s] = z.y;
                    }
                    a0 += L.e[s] * (double)z.x;
                    a1 += L.e[s] * (double)z.y;
                }
            }
            for (int m = 1; m < tpt; m <<= 1) {
                a0 += __shfl_xor(a0, m);
                a1 += __shfl_xor(a1, m);
            }
            o0 = a0;
            o1 = a1;
        } else {
            float a0 = 0.0f, a1 = 0.0f;
            if (t < T) {
                for (int s = part; s < nk; s += tpt) {
                    const float2 z = keep_noise ? L.nz[t * S + s] : noise_at(k0 + s, t);
                    if (store_du) {
                        p.du[(size_t)(2 * t) * Kp + k0 + s] = z.x;
                        p.du[(size_t)(2 * t + 1) * Kp + k0 + s] = z.y;
                    }
                    a0 = fmaf((float)L.e[s], z.x, a0);
                    a1 = fmaf((float)L.e[s], z.y, a1);
                }
            }
            for (int m = 1; m < tpt; m <<= 1) {
                a0 += __shfl_xor(a0, m);
                a1 += __shfl_xor(a1, m);
            }
            o0 = (double)a0;
            o1 = (double)a1;
        }
        if (part == 0 && t < T) {
            if (smooth) {
                nb[2 * t] = o0;
                nb[2 * t + 1] = o1;
            } else {
                p.partN[(size_t)(2 * t) * p.tiles + tile] = any ? o0 : 0.0;
                p.partN[(size_t)(2 * t + 1) * p.tiles + tile] = any ? o1 : 0.0;
            }
        }
    }
    // Algorithm 1's Savitzky-Golay smoothing of the weighted increment is
    // linear along the horizon, so it is applied to the tile's own sums:
    // N_b[t][c] <- sum_j a_tj N_b[s_t + j][c] over the window of step t.
    if (smooth) {
        __syncthreads();
        const int m = p.sgf_m, Wn = 2 * m + 1;
        for (int r = tid; r < 2 * T; r += kRollBlock) {
            const int t = r >> 1, c = r & 1;
            const int s0 = min(max(t - m, 0), T - Wn);
            const float* a = p.sgf_coef + (size_t)t * Wn;
            double v = 0.0;
            for (int j = 0; j < Wn; ++j) v += (double)a[j] * nb[2 * (s0 + j) + c];
            p.partN[(size_t)r * p.tiles + tile] = any ? v : 0.0;
        }
    }
    if (valid) {
        p.S[k] = S_hi;
        p.S[Kp + k] = S_lo;
        p.e[k] = (float)ek;
    }
    if (tid == 0) {
        p.rho_b[tile] = rho_b;
        p.eta_b[tile] = any ? eta_b : 0.0;
        p.flag_b[tile] = use64 ? 1 : 0;
        if (tile == 0) {
            // identical in every tile; the update kernel reports them
            CtrlState* st = p.st;
            st->beta0 = beta0;
            st->beta_d = beta_d;
            st->cshift = cshift;
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Workgroups are handed to the chip's 8 XCDs in turn (workgroup i to XCD
// i mod 8).  The tile of workgroup i makes each XCD take a contiguous run of
// tiles, so the tiles whose partial sums share a line of the [2T][tiles]
// layout write it from one L2 (a bijection on [0, tiles) for any count).
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int i, int tiles)
{
    const int x = i % kXcds, j = i / kXcds;
    const int q = tiles / kXcds, r = tiles % kXcds;
    return x * q + min(x, r) + j;
}

// The kernel's arguments (the parameter block, then the step's arguments)
// are read field by field through the prologue, and each first touch of one
// of their lines would wait on memory in turn.  One word of every 64-byte
// line of the first Bytes bytes is loaded here, all in one batch, so the
// later loads hit the scalar cache.
template <int Bytes>
__device__ __forceinline__ void touch_kernargs()
{
    using KWord = const __attribute__((address_space(4))) uint32_t;
    KWord* kp = (KWord*)__builtin_amdgcn_kernarg_segment_ptr();
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < Bytes / 4; i += 16) t ^= kp[i];
    asm volatile("" ::"s"(t));
}

template <int MODEL, int S, int PT, bool IND, bool MAP>
__global__ __launch_bounds__(kRollBlock) void k_rollout(DevParams p, StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NS = Model<MODEL>::NS;
    touch_kernargs<(int)(sizeof(DevParams) + sizeof(StepArgs))>();
    X0 xs;
    if (a.x0_ptr) {
        // the state's NS words, unconditionally, so the loads issue together
#pragma unroll
        for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = i < NS ? a.x0_ptr[i] : 0.0f;
    } else {
#pragma unroll
        for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = a.x0[i];
    }
    xs.parity = a.parity;
    rollout_tile<MODEL, S, PT, IND, MAP>(p, xcd_tile((int)blockIdx.x, p.tiles), xs, smem);
}

// Persistent rollout over a work list of (controller, tile) units of one
// tile shape, taken in list order (the host sorts it longest-first): the
// tile of the standalone kernel of that shape.  Every block leaves the loop
// once the list is exhausted; the last block to leave resets the queue.
template <int MODEL, int S, int PT, bool IND, bool MAP>
__global__ __launch_bounds__(kRollBlock) void k_batch_rollout(const DevParams* __restrict__ ps,
                                                              const BatchUnit* __restrict__ units, int nunits,
                                                              const BatchIn* __restrict__ in, uint32_t* queue)
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
        for (int i = 0; i < MPPI_NMAX + 2; ++i) xs.v[i] = in[bu.ctrl].x0[i];
        xs.parity = in[bu.ctrl].parity;
        rollout_tile<MODEL, S, PT, IND, MAP>(p, bu.tile, xs, smem);
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

// The batched kernel of one model's `key` (kind key / kTileSizes: layout
// form, runtime P, indicator, each without and with a costmap; tile size
// 16 << key % kTileSizes).
template <int MODEL, int S>
BatchRolloutKernel batch_kernel_of_kind(int kind)
{
    constexpr int PD = MODEL == MPPI_CAR ? 8 : 7;
    switch (kind) {
    case 0: return k_batch_rollout<MODEL, S, PD, false, false>;
    case 1: return k_batch_rollout<MODEL, S, PD, false, true>;
    case 2: return k_batch_rollout<MODEL, S, 0, false, false>;
    case 3: return k_batch_rollout<MODEL, S, 0, false, true>;
    case 4: return k_batch_rollout<MODEL, S, 0, true, false>;
    default: return k_batch_rollout<MODEL, S, 0, true, true>;
    }
}

template <int MODEL>
BatchRolloutKernel batch_kernel_of(int key)
{
    const int kind = key / kTileSizes;
    switch (key % kTileSizes) {
    case 0: return batch_kernel_of_kind<MODEL, 16>(kind);
    case 1: return batch_kernel_of_kind<MODEL, 32>(kind);
    case 2: return batch_kernel_of_kind<MODEL, 64>(kind);
    case 3: return batch_kernel_of_kind<MODEL, 128>(kind);
    default: return batch_kernel_of_kind<MODEL, 256>(kind);
    }
}

template <int MODEL, int S>
hipError_t launch_rollout_ms(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    constexpr int PD = MODEL == MPPI_CAR ? 8 : 7;
    const dim3 g(p.tiles), b(kRollBlock);
    const bool map = p.sdf != nullptr;
    if (p.cost_mode == MPPI_COST_INDICATOR) {
        if (map) hipLaunchKernelGGL((k_rollout<MODEL, S, 0, true, true>), g, b, lds, s, p, a);
        else hipLaunchKernelGGL((k_rollout<MODEL, S, 0, true, false>), g, b, lds, s, p, a);
    } else if (p.P == PD && p.shape_kind != kShapeGeneral) {
        if (map) hipLaunchKernelGGL((k_rollout<MODEL, S, PD, false, true>), g, b, lds, s, p, a);
        else hipLaunchKernelGGL((k_rollout<MODEL, S, PD, false, false>), g, b, lds, s, p, a);
    } else {
        if (map) hipLaunchKernelGGL((k_rollout<MODEL, S, 0, false, true>), g, b, lds, s, p, a);
        else hipLaunchKernelGGL((k_rollout<MODEL, S, 0, false, false>), g, b, lds, s, p, a);
    }
    return hipGetLastError();
}

template <int MODEL>
hipError_t launch_rollout_m(const DevParams& p, const StepArgs& a, size_t lds, hipStream_t s)
{
    switch (p.spt) {
    case 16: return launch_rollout_ms<MODEL, 16>(p, a, lds, s);
    case 32: return launch_rollout_ms<MODEL, 32>(p, a, lds, s);
    case 64: return launch_rollout_ms<MODEL, 64>(p, a, lds, s);
    case 128: return launch_rollout_ms<MODEL, 128>(p, a, lds, s);
    case 256: return launch_rollout_ms<MODEL, 256>(p, a, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace dbas
