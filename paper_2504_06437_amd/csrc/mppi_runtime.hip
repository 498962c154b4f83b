// Host runtime of the DBaS-Log-MPPI library: handle lifecycle, configuration
// checks, device buffers, the single-controller step, inspection, and the
// batched step (persistent kernel captured in a HIP graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mppi_internal.hpp"
#include "mppi_runtime.hpp"

using namespace dbas;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

const char* kStatusNames[] = {"MPPI_OK", "MPPI_E_INVALID", "MPPI_E_NOMEM", "MPPI_E_DEVICE", "MPPI_E_NUMERIC",
                              "MPPI_E_BUSY"};

bool finite_all(const float* v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Spin until the completion mark of iteration `want` appears in the pinned
// result block; false after about 50 ms.
bool wait_completion(const HostResult* r, uint64_t want)
{
    const volatile uint64_t* seq = &r->seq;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t i = 1;; ++i) {
        if (*seq == want) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return true;
        }
        if ((i & 1023u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) return false;
        __builtin_ia32_pause();
    }
}

// Savitzky-Golay weights for every step of a horizon of T: row t holds the
// 2m+1 weights a_j with which the smoothed value at t is sum_j a_j y[s + j],
// s = clamp(t - m, 0, T - 2m - 1): the value at t of the least-squares
// polynomial of degree p through the window.  With V the window's Vandermonde
// matrix (positions relative to t, scaled by 1/m) and V = QR by modified
// Gram-Schmidt, the fit's value at t is e0^T R^-1 Q^T y, so a = Q z with
// R^T z = e0.  FP64 throughout.
std::vector<float> savitzky_golay_weights(int T, int m, int p)
{
    const int W = 2 * m + 1, C = p + 1;
    std::vector<float> out((size_t)T * W);
    std::vector<double> Q((size_t)W * C), R((size_t)C * C), z(C);
    for (int t = 0; t < T; ++t) {
        const int s = std::min(std::max(t - m, 0), T - W);
        for (int j = 0; j < W; ++j) {
            const double x = (double)(s + j - t) / (double)m;
            double v = 1.0;
            for (int k = 0; k < C; ++k, v *= x) Q[(size_t)j * C + k] = v;
        }
        std::fill(R.begin(), R.end(), 0.0);
        for (int k = 0; k < C; ++k) {
            for (int i = 0; i < k; ++i) {
                double d = 0.0;
                for (int j = 0; j < W; ++j) d += Q[(size_t)j * C + i] * Q[(size_t)j * C + k];
                R[(size_t)i * C + k] = d;
                for (int j = 0; j < W; ++j) Q[(size_t)j * C + k] -= d * Q[(size_t)j * C + i];
            }
            double nrm = 0.0;
            for (int j = 0; j < W; ++j) nrm += Q[(size_t)j * C + k] * Q[(size_t)j * C + k];
            nrm = std::sqrt(nrm);
            R[(size_t)k * C + k] = nrm;
            for (int j = 0; j < W; ++j) Q[(size_t)j * C + k] /= nrm;
        }
        // R^T z = e0 (forward substitution)
        for (int k = 0; k < C; ++k) {
            double v = k == 0 ? 1.0 : 0.0;
            for (int i = 0; i < k; ++i) v -= R[(size_t)i * C + k] * z[i];
            z[k] = v / R[(size_t)k * C + k];
        }
        for (int j = 0; j < W; ++j) {
            double a = 0.0;
            for (int k = 0; k < C; ++k) a += Q[(size_t)j * C + k] * z[k];
            out[(size_t)t * W + j] = (float)a;
        }
    }
    return out;
}

}  // namespace

int mppi_ctrl::fail(int status, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    if (status == MPPI_E_DEVICE) poisoned = true;
    return status;
}

int mppi_ctrl::hip_fail(hipError_t e, const char* what)
{
    (void)hipGetLastError();
    return fail(MPPI_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                         \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return (h)->hip_fail(e_, #expr);   \
    } while (0)

#define CHECK_HANDLE(h)                                                    \
    do {                                                                   \
        if (!(h)) return MPPI_E_INVALID;                                   \
        if ((h)->poisoned) return MPPI_E_DEVICE;                           \
    } while (0)

// ---------------------------------------------------------------------------
// configuration
// ---------------------------------------------------------------------------
extern "C" int mppi_config_default(int32_t model, int32_t K, int32_t T, mppi_config* c)
{
    if (!c || model < MPPI_QUAD6 || model > MPPI_CAR) return MPPI_E_INVALID;
    std::memset(c, 0, sizeof *c);
    c->abi_version = MPPI_ABI_VERSION;
    c->model = model;
    c->K = K;
    c->T = T;
    c->mass = 0.5f;
    c->gravity = 9.81f;
    c->arm = 0.2f;
    c->inertia = 0.005f;
    c->wheelbase = 4.0f;
    c->sigma[0] = c->sigma[1] = 0.5f;
    c->mu_ln = 0.0f;
    c->sigma_ln = 0.3f;
    c->lambda = 1.0f;
    c->gamma_u = 2.0f;
    c->gamma_b = 0.5f;
    c->r_b = 0.1f;
    c->h_eps = 1e-4f;
    c->seed = 0;
    c->normaliser = MPPI_NORM_AUTO;
    c->init_mode = MPPI_INIT_REPEAT;
    c->tile_samples = 0;
    c->explore_mu = 0.4f;
    c->sgf_order = 2;
    c->sampling = MPPI_SAMPLE_NLN;
    c->cost_mode = MPPI_COST_DBAS;
    c->collision_weight = 1000.0f;
    const int n = state_dim(model);
    for (int a = 0; a < n; ++a) c->Q[a] = a < 2 ? 1.0f : 0.1f;
    for (int a = 0; a < n; ++a) c->Qf[a] = 10.0f * c->Q[a];
    if (model == MPPI_CAR) {
        c->dt = 0.05f;
        c->u_min[0] = -1.013f; c->u_max[0] = 1.013f;
        c->u_min[1] = -2.0f; c->u_max[1] = 2.0f;
        const float pts[8][2] = {{2, 1.5f}, {2, -1.5f}, {-2, 1.5f}, {-2, -1.5f}, {2, 0}, {-2, 0}, {0, 1.5f}, {0, -1.5f}};
        c->P = 8;
        std::memcpy(c->shape, pts, sizeof pts);
    } else {
        c->dt = 0.02f;
        if (model == MPPI_QUAD6) {
            const float half = 0.5f * c->mass * c->gravity;
            c->u_min[0] = c->u_min[1] = -half;
            c->u_max[0] = c->u_max[1] = half;
        } else {
            c->u_min[0] = -4.0f; c->u_max[0] = 4.0f;
            c->u_min[1] = -0.981f; c->u_max[1] = 0.981f;
            c->sigma[0] = std::sqrt(0.4f);
            c->sigma[1] = std::sqrt(0.12f);
        }
        c->P = 7;
        for (int i = 0; i < 7; ++i) {
            c->shape[i][0] = -0.2f + 0.4f * (float)i / 6.0f;
            c->shape[i][1] = 0.0f;
        }
    }
    return MPPI_OK;
}

namespace dbas {

std::string validate_config(const mppi_config* c)
{
    char b[256];
    if (!c) return "config is NULL";
    if (c->abi_version != MPPI_ABI_VERSION) {
        snprintf(b, sizeof b, "abi_version %u, library has %u", c->abi_version, MPPI_ABI_VERSION);
        return b;
    }
    if (c->model < MPPI_QUAD6 || c->model > MPPI_CAR) return "unknown model";
    if (c->K < 1 || c->K > MPPI_KMAX) return "K out of range";
    if (c->T < 1 || c->T > MPPI_TMAX) return "T out of range";
    if (c->P < 1 || c->P > MPPI_PMAX) return "P out of range";
    const float scal[] = {c->dt, c->mass, c->gravity, c->arm, c->inertia, c->wheelbase, c->mu_ln, c->sigma_ln,
                          c->lambda, c->gamma_u, c->gamma_b, c->r_b, c->h_eps};
    if (!finite_all(scal, sizeof scal / sizeof scal[0])) return "non-finite parameter";
    if (!finite_all(&c->shape[0][0], 2 * (size_t)c->P)) return "non-finite shape point";
    if (!finite_all(c->Q, MPPI_NMAX) || !finite_all(c->Qf, MPPI_NMAX)) return "non-finite Q/Qf";
    if (!(c->dt > 0)) return "dt must be > 0";
    if (!(c->lambda > 0)) return "lambda must be > 0";
    if (!(c->gamma_b > 0 && c->gamma_b < 1)) return "gamma_b must lie in (0,1)";
    if (!(c->h_eps > 0)) return "h_eps must be > 0";
    if (c->sigma_ln < 0) return "sigma_ln must be >= 0";
    for (int i = 0; i < MPPI_M; ++i) {
        if (!std::isfinite(c->sigma[i]) || c->sigma[i] < 0) return "sigma must be finite and >= 0";
        if (!std::isfinite(c->u_min[i]) || !std::isfinite(c->u_max[i]) || c->u_min[i] > c->u_max[i])
            return "input limits must be finite with u_min <= u_max";
    }
    if (c->model != MPPI_CAR && !(c->mass > 0)) return "mass must be > 0";
    if (c->model == MPPI_QUAD6 && !(c->inertia > 0)) return "inertia must be > 0";
    if (c->model == MPPI_CAR && !(c->wheelbase > 0)) return "wheelbase must be > 0";
    if (c->normaliser < MPPI_NORM_AUTO || c->normaliser > MPPI_NORM_OFF) return "unknown normaliser mode";
    if (c->init_mode != MPPI_INIT_REPEAT && c->init_mode != MPPI_INIT_ZERO) return "unknown init mode";
    if (c->tile_samples != 0 && !tile_samples_supported(c->tile_samples))
        return "tile_samples must be 0, 16, 32, 64, 128 or 256";
    if (!(c->h_eps >= 1e-9f && c->h_eps <= 1e6f)) return "h_eps must lie in [1e-9, 1e6]";
    if (c->export_noise != 0 && c->export_noise != 1) return "export_noise must be 0 or 1";
    if (c->adaptive_explore != 0 && c->adaptive_explore != 1) return "adaptive_explore must be 0 or 1";
    if (c->adaptive_explore && !(c->explore_mu > 0.0f && c->explore_mu < 1.0f))
        return "explore_mu must lie in (0, 1)";
    if (c->sgf_half_window < 0 || c->sgf_half_window > 16) return "sgf_half_window must lie in 0..16";
    if (c->sgf_half_window > 0) {
        if (c->T < 2 * c->sgf_half_window + 1) return "smoothing needs T >= 2 sgf_half_window + 1";
        if (c->sgf_order < 0 || c->sgf_order > 2 * c->sgf_half_window || c->sgf_order > 8)
            return "sgf_order must lie in 0..min(2 sgf_half_window, 8)";
    }
    if (c->sampling != MPPI_SAMPLE_NLN && c->sampling != MPPI_SAMPLE_NORMAL) return "unknown sampling law";
    if (c->cost_mode != MPPI_COST_DBAS && c->cost_mode != MPPI_COST_INDICATOR) return "unknown cost mode";
    if (!std::isfinite(c->collision_weight) || c->collision_weight < 0) return "collision_weight must be finite and >= 0";
    if (c->cost_mode == MPPI_COST_INDICATOR && c->adaptive_explore)
        return "adaptive exploration follows the barrier cost: it needs cost_mode MPPI_COST_DBAS";
    for (int i = 0; i < 2; ++i)
        if (c->reserved[i] != 0) return "reserved fields must be zero";
    return "";
}

}  // namespace dbas

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
mppi_ctrl::~mppi_ctrl()
{
    if (device >= 0) (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* ptr : allocations) (void)hipFree(ptr);
    if (d_obs) (void)hipFree(d_obs);
    if (d_sdf) (void)hipFree(d_sdf);
    if (d_sdf4) (void)hipFree(d_sdf4);
    if (h_res) (void)hipHostFree(h_res);
    for (hipEvent_t e : prof_events)
        if (e) (void)hipEventDestroy(e);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void* mppi_ctrl::dalloc(size_t bytes, int* status)
{
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *status = fail(MPPI_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        return nullptr;
    }
    allocations.push_back(ptr);
    return ptr;
}

int mppi_ctrl::sync()
{
    HIP_TRY(this, hipSetDevice(device));
    HIP_TRY(this, hipStreamSynchronize(stream));
    return MPPI_OK;
}

int mppi_ctrl::read_state(CtrlState* out)
{
    int s = sync();
    if (s) return s;
    HIP_TRY(this, hipMemcpy(out, p.st, sizeof *out, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

int mppi_ctrl::write_state_field(size_t offset, const void* src, size_t bytes)
{
    int s = sync();
    if (s) return s;
    HIP_TRY(this, hipMemcpy(reinterpret_cast<char*>(p.st) + offset, src, bytes, hipMemcpyHostToDevice));
    return MPPI_OK;
}

namespace dbas {

// Samples per tile: the largest tile (at most 64) that still gives every CU of
// the chip a tile, and that fits the LDS budget (tile_fits).  Used when the
// configuration leaves tile_samples at 0 and no measured choice is known.
// Returns 0 when no tile shape fits.
int heuristic_tile_samples(int K, int J, int T, int n, int sgf_m)
{
    int S = 16;
    while (S < 64 && (long)K / (2 * S) >= 256) S *= 2;
    while (S < kMaxTile && (K + S - 1) / S > kMaxTiles) S *= 2;
    for (int c = S; c >= 16; c /= 2)
        if (tile_fits(J, T, n, c, sgf_m) && (K + c - 1) / c <= kMaxTiles) return c;
    for (int c = S * 2; c <= kMaxTile; c *= 2)
        if (tile_fits(J, T, n, c, sgf_m) && (K + c - 1) / c <= kMaxTiles) return c;
    return 0;
}

// Is there any tile shape for these sizes?
bool any_tile_fits(int K, int J, int T, int n, int sgf_m) { return heuristic_tile_samples(K, J, T, n, sgf_m) != 0; }

}  // namespace dbas

int mppi_ctrl::configure_tiles(int S)
{
    if (!tile_samples_supported(S) || !tile_fits(p.J, cfg.T, p.n, S, p.sgf_m))
        return fail(MPPI_E_INVALID,
                    "J=%d obstacles with T=%d%s do not fit the rollout's LDS budget at %d samples per tile", p.J,
                    cfg.T, p.sgf_m > 0 ? " and smoothing" : "", S);
    p.spt = S;
    p.tiles = (cfg.K + S - 1) / S;
    if (p.tiles > kMaxTiles) return fail(MPPI_E_INVALID, "K=%d needs more than %d tiles of %d samples", cfg.K, kMaxTiles, S);
    return MPPI_OK;
}

int mppi_ctrl::alloc_tile_buffers()
{
    int st = MPPI_OK;
    const int T = cfg.T, tiles = p.tiles;
    p.rho_b = static_cast<double*>(dalloc(sizeof(double) * tiles, &st));
    p.eta_b = static_cast<double*>(dalloc(sizeof(double) * tiles, &st));
    p.f_b = static_cast<double*>(dalloc(sizeof(double) * tiles, &st));
    p.flag_b = static_cast<int32_t*>(dalloc(sizeof(int32_t) * tiles, &st));
    p.partN = static_cast<double*>(dalloc(sizeof(double) * (size_t)2 * T * tiles, &st));
    if (st) return st;
    HIP_TRY(this, hipMemset(p.f_b, 0, sizeof(double) * tiles));
    return MPPI_OK;
}

namespace dbas {

// The kernel parameters a configuration fixes (no buffers, no obstacles).
void params_from_config(const mppi_config* cfg, DevParams& p)
{
    std::memset(&p, 0, sizeof p);
    const int K = cfg->K, T = cfg->T, n = state_dim(cfg->model);
    p.model = cfg->model;
    p.K = K;
    p.Kp = round_up(K, 64);
    p.T = T;
    p.P = cfg->P;
    p.J = 0;
    p.n = n;
    p.normaliser = cfg->normaliser;
    p.init_mode = cfg->init_mode;
    p.dt = cfg->dt;
    p.mass = cfg->mass;
    p.gravity = cfg->gravity;
    p.arm = cfg->arm;
    p.inertia = cfg->inertia;
    p.wheelbase = cfg->wheelbase;
    for (int i = 0; i < kM; ++i) {
        p.u_min[i] = cfg->u_min[i];
        p.u_max[i] = cfg->u_max[i];
        p.sigma[i] = cfg->sigma[i];
    }
    p.mu_ln = cfg->mu_ln;
    p.sigma_ln = cfg->sigma_ln;
    p.lambda = cfg->lambda;
    p.gamma_u = cfg->gamma_u;
    p.gamma_b = cfg->gamma_b;
    p.r_b = cfg->r_b;
    {
        // the common part c_t = gamma_B (c_{t-1} - beta_d), c_0 = 0, of the
        // barrier state sums over t = 1..T to -beta_d gamma_B/(1-gamma_B)
        // (T - gamma_B (1 - gamma_B^T)/(1 - gamma_B)); its cost is R_B times that
        const double g = (double)cfg->gamma_b;
        const double geo = g * (1.0 - std::pow(g, (double)cfg->T)) / (1.0 - g);
        p.beta_d_weight = -(double)cfg->r_b * g / (1.0 - g) * ((double)cfg->T - geo);
    }
    p.h_eps = cfg->h_eps;
    for (int a = 0; a < MPPI_NMAX; ++a) {
        p.Q[a] = a < n ? cfg->Q[a] : 0.0f;
        p.Qf[a] = a < n ? cfg->Qf[a] : 0.0f;
    }
    std::memcpy(p.shape, cfg->shape, sizeof p.shape);
    p.shape_kind = shape_form(p.model, p.P, p.shape);
    p.export_noise = cfg->export_noise ? 1 : 0;
    p.adaptive = cfg->adaptive_explore ? 1 : 0;
    p.explore_mu = cfg->explore_mu;
    p.sgf_m = cfg->sgf_half_window;
    p.sampling = cfg->sampling;
    p.cost_mode = cfg->cost_mode;
    p.collision_weight = cfg->collision_weight;
    p.seed_lo = (uint32_t)cfg->seed;
    p.seed_hi = (uint32_t)(cfg->seed >> 32);
}

}  // namespace dbas

extern "C" int mppi_create(const mppi_config* cfg, const mppi_device* dev, mppi_t** out)
{
    return create_ctrl(cfg, dev, false, out);
}

// external_scratch: leave the per-iteration sample buffers (noise, costs,
// exponentials, tile partials) unallocated; the owner (the server) supplies
// them per launch from its own pool.
int dbas::create_ctrl(const mppi_config* cfg, const mppi_device* dev, bool external_scratch, mppi_ctrl** out)
{
    if (!out) return MPPI_E_INVALID;
    *out = nullptr;
    std::string why = validate_config(cfg);
    if (!why.empty()) {
        set_global_error("mppi_create: " + why);
        return MPPI_E_INVALID;
    }
    mppi_ctrl* h = new (std::nothrow) mppi_ctrl();
    if (!h) return MPPI_E_NOMEM;
    h->cfg = *cfg;
    h->external_scratch = external_scratch;
    h->device = dev ? dev->device : 0;
    int st = MPPI_OK;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) {
        set_global_error(std::string("hipSetDevice: ") + hipGetErrorString(e));
        delete h;
        return MPPI_E_DEVICE;
    }
    if (dev && dev->stream) {
        h->stream = static_cast<hipStream_t>(dev->stream);
    } else {
        e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) {
            set_global_error(std::string("hipStreamCreate: ") + hipGetErrorString(e));
            delete h;
            return MPPI_E_DEVICE;
        }
        h->own_stream = true;
    }

    DevParams& p = h->p;
    params_from_config(cfg, p);
    const int K = cfg->K, T = cfg->T, n = state_dim(cfg->model);

    st = h->configure_tiles(cfg->tile_samples ? cfg->tile_samples
                                              : heuristic_tile_samples(K, 0, T, n, cfg->sgf_half_window));
    if (st) {
        set_global_error("mppi_create: " + h->err);
        delete h;
        return st;
    }
    h->tiles_fixed = cfg->tile_samples != 0;

    p.U = static_cast<float*>(h->dalloc(sizeof(float) * 2 * T * kM, &st));
    p.Ustar = static_cast<float*>(h->dalloc(sizeof(float) * T * kM, &st));
    if (!external_scratch) {
        if (p.export_noise) p.du = static_cast<float*>(h->dalloc(sizeof(float) * (size_t)T * kM * p.Kp, &st));
        p.S = static_cast<float*>(h->dalloc(sizeof(float) * 2 * (size_t)p.Kp, &st));
        p.e = static_cast<float*>(h->dalloc(sizeof(float) * (size_t)p.Kp, &st));
    }
    p.xref = static_cast<float*>(h->dalloc(sizeof(float) * (size_t)(T + 1) * n, &st));
    p.st = static_cast<CtrlState*>(h->dalloc(sizeof(CtrlState), &st));
    if (p.sgf_m > 0 && !st) {
        const std::vector<float> coef = savitzky_golay_weights(T, p.sgf_m, cfg->sgf_order);
        float* d = static_cast<float*>(h->dalloc(sizeof(float) * coef.size(), &st));
        if (!st && hipMemcpy(d, coef.data(), sizeof(float) * coef.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            st = h->fail(MPPI_E_DEVICE, "uploading the smoothing weights failed");
        }
        p.sgf_coef = d;
    }
    if (st) {
        set_global_error(h->err);
        delete h;
        return st;
    }
    if (!st && !external_scratch) st = h->alloc_tile_buffers();
    if (st) {
        set_global_error(h->err);
        delete h;
        return st;
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&h->h_res), sizeof(HostResult), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&p.res), h->h_res, 0);
    if (e != hipSuccess) {
        set_global_error(std::string("pinned result buffer: ") + hipGetErrorString(e));
        delete h;
        return MPPI_E_NOMEM;
    }
    std::memset(h->h_res, 0, sizeof(HostResult));

    CtrlState s0;
    std::memset(&s0, 0, sizeof s0);
    s0.S_e = 1.0f;
    e = hipMemset(p.U, 0, sizeof(float) * 2 * T * kM);
    if (e == hipSuccess) e = hipMemset(p.Ustar, 0, sizeof(float) * T * kM);
    if (!external_scratch) {
        if (e == hipSuccess && p.du) e = hipMemset(p.du, 0, sizeof(float) * (size_t)T * kM * p.Kp);
        if (e == hipSuccess) e = hipMemset(p.S, 0, sizeof(float) * 2 * (size_t)p.Kp);
        if (e == hipSuccess) e = hipMemset(p.e, 0, sizeof(float) * (size_t)p.Kp);
    }
    if (e == hipSuccess) e = hipMemset(const_cast<float*>(p.xref), 0, sizeof(float) * (size_t)(T + 1) * n);
    if (e == hipSuccess) e = hipMemcpy(p.st, &s0, sizeof s0, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_global_error(std::string("initialising buffers: ") + hipGetErrorString(e));
        delete h;
        return MPPI_E_DEVICE;
    }
    *out = h;
    return MPPI_OK;
}

extern "C" void mppi_destroy(mppi_t* h) { delete h; }

// The tile shape depends on (model, K, T, J, P); re-choose it when J changes
// and the configuration did not fix it.
int mppi_ctrl::retile()
{
    if (tiles_fixed) return tile_fits(p.J, cfg.T, p.n, p.spt, p.sgf_m) ? MPPI_OK : configure_tiles(p.spt);
    const int S = choose_tile_samples(this);
    if (S == 0) return fail(MPPI_E_INVALID, "no tile shape fits the LDS budget");
    if (S == p.spt) return configure_tiles(S);
    if (external_scratch) {
        ++version;
        return configure_tiles(S);
    }
    int s = sync();
    if (s) return s;
    for (double* ptr : {p.rho_b, p.eta_b, p.f_b}) {
        allocations.erase(std::find(allocations.begin(), allocations.end(), (void*)ptr));
        (void)hipFree(ptr);
    }
    allocations.erase(std::find(allocations.begin(), allocations.end(), (void*)p.flag_b));
    (void)hipFree(p.flag_b);
    allocations.erase(std::find(allocations.begin(), allocations.end(), (void*)p.partN));
    (void)hipFree(p.partN);
    p.rho_b = p.eta_b = p.f_b = p.partN = nullptr;
    p.flag_b = nullptr;
    ++version;
    const int st = configure_tiles(S);
    if (st) return st;
    return alloc_tile_buffers();
}

extern "C" int mppi_set_obstacles(mppi_t* h, int32_t J, const float* cxcyr, int32_t mem)
{
    CHECK_HANDLE(h);
    if (J < 0 || J > MPPI_JMAX) return h->fail(MPPI_E_INVALID, "J=%d outside 0..%d", J, MPPI_JMAX);
    if (J > 0 && !cxcyr) return h->fail(MPPI_E_INVALID, "obstacles pointer is NULL");
    if (h->tiles_fixed ? !tile_fits(J, h->cfg.T, h->p.n, h->p.spt, h->p.sgf_m)
                       : !any_tile_fits(h->cfg.K, J, h->cfg.T, h->p.n, h->p.sgf_m))
        return h->fail(MPPI_E_INVALID, "J=%d obstacles with T=%d%s exceed the rollout's LDS budget", J, h->cfg.T,
                       h->p.sgf_m > 0 ? " and smoothing" : "");
    std::vector<float> tmp;
    if (J > 0 && mem == MPPI_MEM_HOST) {
        if (!finite_all(cxcyr, (size_t)3 * J)) return h->fail(MPPI_E_INVALID, "non-finite obstacle");
        for (int j = 0; j < J; ++j)
            if (cxcyr[3 * j + 2] < 0) return h->fail(MPPI_E_INVALID, "negative obstacle radius");
    }
    int s = h->sync();
    if (s) return s;
    if (J > h->obs_cap) {
        if (h->d_obs) (void)hipFree(h->d_obs);
        h->d_obs = nullptr;
        HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&h->d_obs), sizeof(float) * 3 * (size_t)J));
        h->obs_cap = J;
    }
    if (J > 0) {
        HIP_TRY(h, hipMemcpy(h->d_obs, cxcyr, sizeof(float) * 3 * (size_t)J,
                             mem == MPPI_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    }
    h->p.obs = h->d_obs;
    h->p.J = J;
    ++h->version;
    return h->retile();
}

extern "C" int mppi_set_costmap(mppi_t* h, int32_t W, int32_t H, float x0, float y0, float res, const float* sdf,
                                int32_t mem)
{
    CHECK_HANDLE(h);
    if (!sdf) {
        const bool had = h->p.sdf != nullptr;
        h->p.sdf = nullptr;
        h->p.sdf4 = nullptr;
        h->p.map_w = h->p.map_h = 0;
        ++h->version;
        // the costmap is part of the tile shape's key: choose again
        return had ? h->retile() : MPPI_OK;
    }
    if (W < 2 || H < 2 || (long)W * H > (1L << 26)) return h->fail(MPPI_E_INVALID, "costmap must be at least 2x2");
    if (!(res > 0) || !std::isfinite(res) || !std::isfinite(x0) || !std::isfinite(y0))
        return h->fail(MPPI_E_INVALID, "costmap origin/resolution invalid");
    if (mem == MPPI_MEM_HOST && !finite_all(sdf, (size_t)W * H)) return h->fail(MPPI_E_INVALID, "non-finite costmap");
    int s = h->sync();
    if (s) return s;
    const size_t bytes = sizeof(float) * (size_t)W * H;
    if (bytes > h->sdf_bytes) {
        if (h->d_sdf) (void)hipFree(h->d_sdf);
        h->d_sdf = nullptr;
        HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&h->d_sdf), bytes));
        h->sdf_bytes = bytes;
    }
    HIP_TRY(h, hipMemcpy(h->d_sdf, sdf, bytes, mem == MPPI_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    const size_t bytes4 = sizeof(float4) * (size_t)(W - 1) * (H - 1);
    if (bytes4 > h->sdf4_bytes) {
        if (h->d_sdf4) (void)hipFree(h->d_sdf4);
        h->d_sdf4 = nullptr;
        HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&h->d_sdf4), bytes4));
        h->sdf4_bytes = bytes4;
    }
    HIP_TRY(h, launch_sdf_cells(h->d_sdf, W, H, h->d_sdf4, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const bool had = h->p.sdf != nullptr;
    h->p.sdf = h->d_sdf;
    h->p.sdf4 = h->d_sdf4;
    h->p.map_w = W;
    h->p.map_h = H;
    h->p.map_x0 = x0;
    h->p.map_y0 = y0;
    h->p.map_res = res;
    ++h->version;
    // the costmap is part of the tile shape's key: choose again
    return had ? MPPI_OK : h->retile();
}

extern "C" int mppi_set_reference(mppi_t* h, const float* x_ref, int32_t mem)
{
    CHECK_HANDLE(h);
    if (!x_ref) return h->fail(MPPI_E_INVALID, "x_ref is NULL");
    const size_t cnt = (size_t)(h->cfg.T + 1) * h->p.n;
    if (mem == MPPI_MEM_HOST && !finite_all(x_ref, cnt)) return h->fail(MPPI_E_INVALID, "non-finite reference");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipMemcpyAsync(const_cast<float*>(h->p.xref), x_ref, sizeof(float) * cnt,
                              mem == MPPI_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
    if (mem == MPPI_MEM_HOST) HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MPPI_OK;
}

extern "C" int mppi_set_exploration(mppi_t* h, float S_e)
{
    CHECK_HANDLE(h);
    if (!(S_e > 0) || !std::isfinite(S_e)) return h->fail(MPPI_E_INVALID, "S_e must be finite and > 0");
    return h->write_state_field(offsetof(CtrlState, S_e), &S_e, sizeof S_e);
}

extern "C" int mppi_set_controls(mppi_t* h, const float* U, int32_t mem)
{
    CHECK_HANDLE(h);
    if (!U) return h->fail(MPPI_E_INVALID, "U is NULL");
    const size_t cnt = (size_t)h->cfg.T * kM;
    if (mem == MPPI_MEM_HOST && !finite_all(U, cnt)) return h->fail(MPPI_E_INVALID, "non-finite controls");
    CtrlState st;
    int s = h->read_state(&st);
    if (s) return s;
    HIP_TRY(h, hipMemcpy(h->p.U + (size_t)(h->iter & 1u) * cnt, U, sizeof(float) * cnt,
                         mem == MPPI_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    return MPPI_OK;
}

int mppi_ctrl::launch_step(const float* x0_host, const float* x0_dev, float* u0_dev, bool mark)
{
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.mark = mark ? 1u : 0u;
    if (x0_host) std::memcpy(a.x0, x0_host, sizeof(float) * p.n);
    a.x0_ptr = x0_dev;
    a.u0_dev = u0_dev;
    a.parity = iter & 1u;
    HIP_TRY(this, hipSetDevice(device));
    hipEvent_t* ev = nullptr;
    if (profiling && prof_seen++ % prof_every == 0) {
        if (prof_used * 3 < (int)prof_events.size()) ev = &prof_events[(size_t)prof_used++ * 3];
        else ++prof_dropped;
    }
    if (ev) HIP_TRY(this, hipEventRecord(ev[0], stream));
    HIP_TRY(this, launch_rollout(p, a, stream));
    if (ev) HIP_TRY(this, hipEventRecord(ev[1], stream));
    HIP_TRY(this, launch_update(p, a, stream));
    if (p.adaptive) HIP_TRY(this, launch_explore(p, a, stream));
    ++iter;
    if (ev) HIP_TRY(this, hipEventRecord(ev[2], stream));
    return MPPI_OK;
}

extern "C" int mppi_profile_enable(mppi_t* h, int32_t every)
{
    CHECK_HANDLE(h);
    if (every < 0) return h->fail(MPPI_E_INVALID, "profiling period must be >= 0");
    const bool on = every > 0;
    if (on && h->prof_events.empty()) {
        HIP_TRY(h, hipSetDevice(h->device));
        h->prof_events.resize(3 * 4096, nullptr);
        // timing only: the host reads them after synchronising the stream, so
        // they need no system-scope fence (which would add a cache write-back
        // to every timed launch)
        for (auto& e : h->prof_events) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    h->profiling = on;
    h->prof_every = on ? every : 1;
    h->prof_seen = 0;
    h->prof_used = 0;
    h->prof_dropped = 0;
    return MPPI_OK;
}

extern "C" int mppi_profile_read(mppi_t* h, mppi_profile* out)
{
    CHECK_HANDLE(h);
    if (!out) return MPPI_E_INVALID;
    int s = h->sync();
    if (s) return s;
    out->iterations = h->prof_used;
    out->dropped = h->prof_dropped;
    out->rollout_ms = out->update_ms = 0.0;
    for (int i = 0; i < h->prof_used; ++i) {
        float a = 0.0f, b = 0.0f;
        HIP_TRY(h, hipEventElapsedTime(&a, h->prof_events[3 * i], h->prof_events[3 * i + 1]));
        HIP_TRY(h, hipEventElapsedTime(&b, h->prof_events[3 * i + 1], h->prof_events[3 * i + 2]));
        out->rollout_ms += a;
        out->update_ms += b;
    }
    h->prof_used = 0;
    h->prof_dropped = 0;
    return MPPI_OK;
}

extern "C" int mppi_step(mppi_t* h, const float* x0, float* u0)
{
    CHECK_HANDLE(h);
    if (!x0 || !u0) return h->fail(MPPI_E_INVALID, "x0/u0 is NULL");
    if (!finite_all(x0, h->p.n)) return h->fail(MPPI_E_INVALID, "non-finite x0");
    int s = h->launch_step(x0, nullptr, nullptr, true);
    if (s) return s;
    // the update kernel marks completion in pinned memory after u0 and the
    // status; spin on it (a stream synchronisation wakes up later), and fall
    // back to the synchronisation -- which also reports errors -- after 50 ms
    if (!wait_completion(h->h_res, h->iter)) HIP_TRY(h, hipStreamSynchronize(h->stream));
    const HostResult* r = h->h_res;
    u0[0] = r->u0[0];
    u0[1] = r->u0[1];
    if (r->status != MPPI_OK) return h->fail(r->status, "iteration status %d (%s)", r->status, mppi_status_string(r->status));
    return MPPI_OK;
}

extern "C" int mppi_step_async(mppi_t* h, const float* x0_device, float* u0_device)
{
    CHECK_HANDLE(h);
    if (!x0_device) return h->fail(MPPI_E_INVALID, "x0_device is NULL");
    return h->launch_step(nullptr, x0_device, u0_device);
}

extern "C" int mppi_synchronize(mppi_t* h)
{
    CHECK_HANDLE(h);
    int s = h->sync();
    if (s) return s;
    CtrlState st;
    HIP_TRY(h, hipMemcpy(&st, h->p.st, sizeof st, hipMemcpyDeviceToHost));
    return h->iter == 0 ? MPPI_OK : st.status;
}

extern "C" int mppi_get_controls(mppi_t* h, float* U)
{
    CHECK_HANDLE(h);
    if (!U) return MPPI_E_INVALID;
    CtrlState st;
    int s = h->read_state(&st);
    if (s) return s;
    const size_t cnt = (size_t)h->cfg.T * kM;
    HIP_TRY(h, hipMemcpy(U, h->p.U + (size_t)(h->iter & 1u) * cnt, sizeof(float) * cnt, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

extern "C" int mppi_get_last_optimal(mppi_t* h, float* Ustar)
{
    CHECK_HANDLE(h);
    if (!Ustar) return MPPI_E_INVALID;
    int s = h->sync();
    if (s) return s;
    HIP_TRY(h, hipMemcpy(Ustar, h->p.Ustar, sizeof(float) * h->cfg.T * kM, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

extern "C" int mppi_get_costs(mppi_t* h, double* S)
{
    CHECK_HANDLE(h);
    if (!S) return MPPI_E_INVALID;
    int s = h->sync();
    if (s) return s;
    std::vector<float> buf(2 * (size_t)h->p.Kp);
    CtrlState st;
    HIP_TRY(h, hipMemcpy(&st, h->p.st, sizeof st, hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(buf.data(), h->p.S, sizeof(float) * buf.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < h->cfg.K; ++k) S[k] = ((double)buf[k] + (double)buf[h->p.Kp + k]) + st.cshift;
    return MPPI_OK;
}

extern "C" int mppi_get_weights(mppi_t* h, double* w)
{
    CHECK_HANDLE(h);
    if (!w) return MPPI_E_INVALID;
    double* d_w = nullptr;
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&d_w), sizeof(double) * h->cfg.K));
    hipError_t e = launch_weights(h->p, d_w, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(w, d_w, sizeof(double) * h->cfg.K, hipMemcpyDeviceToHost);
    (void)hipFree(d_w);
    if (e != hipSuccess) return h->hip_fail(e, "mppi_get_weights");
    return MPPI_OK;
}

extern "C" int mppi_get_noise(mppi_t* h, float* du)
{
    CHECK_HANDLE(h);
    if (!du) return MPPI_E_INVALID;
    if (!h->p.export_noise) return h->fail(MPPI_E_INVALID, "the noise is only kept with export_noise = 1");
    int s = h->sync();
    if (s) return s;
    const int K = h->cfg.K, T = h->cfg.T, Kp = h->p.Kp;
    std::vector<float> buf((size_t)T * kM * Kp);
    HIP_TRY(h, hipMemcpy(buf.data(), h->p.du, sizeof(float) * buf.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < K; ++k)
        for (int t = 0; t < T; ++t)
            for (int c = 0; c < kM; ++c) du[((size_t)k * T + t) * kM + c] = buf[(size_t)(t * kM + c) * Kp + k];
    return MPPI_OK;
}

extern "C" int mppi_get_step_info(mppi_t* h, mppi_step_info* info)
{
    CHECK_HANDLE(h);
    if (!info) return MPPI_E_INVALID;
    CtrlState st;
    int s = h->read_state(&st);
    if (s) return s;
    info->counter = st.last_counter;
    info->status = h->iter == 0 ? MPPI_OK : st.status;
    info->fp64_tiles = st.fp64_tiles;
    info->rho = st.rho;
    info->eta = st.eta;
    info->beta0 = st.beta0;
    info->beta_d = st.beta_d;
    info->tile_samples = h->p.spt;
    info->tiles = h->p.tiles;
    info->S_e = st.S_e;
    info->cost_b = st.cost_b;
    info->barrier_form = h->p.cost_mode == MPPI_COST_INDICATOR ? 0 : h->p.shape_kind;
    info->noise_kept = tile_keeps_noise(h->p.J, h->cfg.T, h->p.n, h->p.spt) ? 1 : 0;
    return MPPI_OK;
}

extern "C" int mppi_get_philox_words(mppi_t* h, uint64_t counter, uint32_t* words)
{
    CHECK_HANDLE(h);
    if (!words) return MPPI_E_INVALID;
    const size_t n = (size_t)h->cfg.K * h->cfg.T * 4;
    uint32_t* d = nullptr;
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&d), sizeof(uint32_t) * n));
    hipError_t e = launch_philox_words(h->p, counter, d, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(words, d, sizeof(uint32_t) * n, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return h->hip_fail(e, "mppi_get_philox_words");
    return MPPI_OK;
}

extern "C" int mppi_get_state(mppi_t* h, mppi_state* out)
{
    CHECK_HANDLE(h);
    if (!out || !out->U || out->T != h->cfg.T) return h->fail(MPPI_E_INVALID, "state buffer must have T=%d", h->cfg.T);
    CtrlState st;
    int s = h->read_state(&st);
    if (s) return s;
    out->counter = st.counter;
    out->S_e = st.S_e;
    const size_t cnt = (size_t)h->cfg.T * kM;
    HIP_TRY(h, hipMemcpy(out->U, h->p.U + (size_t)(h->iter & 1u) * cnt, sizeof(float) * cnt, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

extern "C" int mppi_set_state(mppi_t* h, const mppi_state* in)
{
    CHECK_HANDLE(h);
    if (!in || !in->U || in->T != h->cfg.T) return h->fail(MPPI_E_INVALID, "state buffer must have T=%d", h->cfg.T);
    if (!(in->S_e > 0) || !std::isfinite(in->S_e)) return h->fail(MPPI_E_INVALID, "S_e must be finite and > 0");
    int s = mppi_set_controls(h, in->U, MPPI_MEM_HOST);
    if (s) return s;
    s = h->write_state_field(offsetof(CtrlState, counter), &in->counter, sizeof in->counter);
    if (s) return s;
    return h->write_state_field(offsetof(CtrlState, S_e), &in->S_e, sizeof in->S_e);
}

extern "C" const char* mppi_last_error(const mppi_t* h) { return h ? h->err.c_str() : global_error(); }

extern "C" const char* mppi_status_string(int32_t s)
{
    return (s >= 0 && s <= 5) ? kStatusNames[s] : "MPPI_E_UNKNOWN";
}

extern "C" void* mppi_stream(const mppi_t* h) { return h ? (void*)h->stream : nullptr; }
