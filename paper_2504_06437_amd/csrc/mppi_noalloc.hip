// mppi_step_noalloc: one iteration with no handle and no allocation, for
// callers that cannot allocate device memory.  The per-iteration scratch
// (iteration state, compensated costs, tile exponentials, tile minima,
// normalisers and update partials) lives in one static device array per GPU;
// its device address is taken once per device with hipGetSymbolAddress (the
// array's name is only a host-side stand-in), and the kernels receive
// pointers carved from that address exactly as they receive a controller's
// own buffers.  Every call on a GPU shares that GPU's array: calls on one
// GPU must not overlap (issue them on one stream, or wait in between).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "mppi_internal.hpp"
#include "mppi_runtime.hpp"

using namespace dbas;

namespace {

static __device__ __align__(256) unsigned char scratch[MPPI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (the device is current).
hipError_t scratch_address(int device, unsigned char** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
    return hipSuccess;
}

// The iteration state the rollout reads (Philox step counter, S_e); every
// other field starts at zero.  A kernel, not a memset, so the call stays
// capturable.
__global__ __launch_bounds__(64) void k_noalloc_init(CtrlState* st, uint64_t counter, float S_e)
{
    if (threadIdx.x != 0) return;
    CtrlState s{};
    s.counter = counter;
    s.S_e = S_e;
    *st = s;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Scratch bytes one iteration of this shape needs.
size_t scratch_bytes(int Kp, int T, int tiles)
{
    size_t b = align_up(sizeof(CtrlState));
    b += align_up(sizeof(float) * 2 * (size_t)Kp);            // S (hi, lo)
    b += align_up(sizeof(float) * (size_t)Kp);                // e
    b += 3 * align_up(sizeof(double) * (size_t)tiles);        // rho_b, eta_b, f_b
    b += align_up(sizeof(int32_t) * (size_t)tiles);           // flag_b
    b += align_up(sizeof(double) * 2 * (size_t)T * tiles);    // partN
    return b;
}

int fail(int status, const std::string& why)
{
    set_global_error("mppi_step_noalloc: " + why);
    return status;
}

}  // namespace

extern "C" int mppi_step_noalloc(const mppi_config* cfg, const mppi_problem* prob, int32_t device, void* stream,
                                 const float* x0_dev, const float* U_dev, uint64_t counter, float S_e,
                                 float* Ustar_dev, float* Unext_dev, float* u0_dev, int32_t* status_dev)
{
    const std::string why = validate_config(cfg);
    if (!why.empty()) return fail(MPPI_E_INVALID, why);
    if (!prob || !x0_dev || !U_dev || !Ustar_dev || !Unext_dev || !prob->x_ref)
        return fail(MPPI_E_INVALID, "a required pointer is NULL");
    if (cfg->adaptive_explore || cfg->sgf_half_window > 0 || cfg->export_noise)
        return fail(MPPI_E_INVALID, "adaptive exploration, smoothing and noise export need a controller handle");
    if (prob->J < 0 || prob->J > MPPI_JMAX || (prob->J > 0 && !prob->obs))
        return fail(MPPI_E_INVALID, "obstacle count outside 0..MPPI_JMAX or obstacles NULL");
    const bool has_map = prob->sdf != nullptr;
    if (has_map && (prob->map_w < 2 || prob->map_h < 2 || !(prob->map_res > 0)))
        return fail(MPPI_E_INVALID, "costmap must be at least 2x2 with res > 0");
    if (!(S_e > 0) || !(S_e < 3.4e38f)) return fail(MPPI_E_INVALID, "S_e must be finite and > 0");
    if (device < 0 || device >= kMaxDevices) return fail(MPPI_E_INVALID, "device index out of range");

    DevParams p;
    params_from_config(cfg, p);
    p.J = prob->J;
    p.obs = prob->obs;
    p.xref = prob->x_ref;
    if (has_map) {
        p.sdf = prob->sdf;
        p.map_w = prob->map_w;
        p.map_h = prob->map_h;
        p.map_x0 = prob->map_x0;
        p.map_y0 = prob->map_y0;
        p.map_res = prob->map_res;
    }
    // no timing here (it would allocate): the configured tile, else the heuristic one
    const int S = cfg->tile_samples ? cfg->tile_samples : heuristic_tile_samples(cfg->K, p.J, cfg->T, p.n, 0);
    if (S == 0 || !tile_samples_supported(S) || !tile_fits(p.J, cfg->T, p.n, S, 0))
        return fail(MPPI_E_INVALID, "the obstacles and horizon do not fit the rollout's LDS budget");
    p.spt = S;
    p.tiles = (cfg->K + S - 1) / S;
    if (p.tiles > kMaxTiles) return fail(MPPI_E_INVALID, "too many sample tiles");
    const size_t need = scratch_bytes(p.Kp, p.T, p.tiles);
    if (need > (size_t)MPPI_NOALLOC_SCRATCH_BYTES)
        return fail(MPPI_E_INVALID, "K=" + std::to_string(cfg->K) + ", T=" + std::to_string(cfg->T) + " needs " +
                                        std::to_string(need) + " scratch bytes, more than MPPI_NOALLOC_SCRATCH_BYTES");

    hipError_t e = hipSetDevice(device);
    unsigned char* base = nullptr;
    if (e == hipSuccess) e = scratch_address(device, &base);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MPPI_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* r = base + off;
        off += align_up(bytes);
        return r;
    };
    p.st = reinterpret_cast<CtrlState*>(take(sizeof(CtrlState)));
    p.S = reinterpret_cast<float*>(take(sizeof(float) * 2 * (size_t)p.Kp));
    p.e = reinterpret_cast<float*>(take(sizeof(float) * (size_t)p.Kp));
    p.rho_b = reinterpret_cast<double*>(take(sizeof(double) * (size_t)p.tiles));
    p.eta_b = reinterpret_cast<double*>(take(sizeof(double) * (size_t)p.tiles));
    p.f_b = reinterpret_cast<double*>(take(sizeof(double) * (size_t)p.tiles));
    p.flag_b = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)p.tiles));
    p.partN = reinterpret_cast<double*>(take(sizeof(double) * 2 * (size_t)p.T * p.tiles));
    p.U = const_cast<float*>(U_dev);
    p.Unext = Unext_dev;
    p.Ustar = Ustar_dev;
    p.res = nullptr;

    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.x0_ptr = x0_dev;
    a.u0_dev = u0_dev;
    a.status_dev = status_dev;
    a.parity = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_noalloc_init, dim3(1), dim3(64), 0, s, p.st, counter, S_e);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_rollout(p, a, s);
    if (e == hipSuccess) e = launch_update(p, a, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MPPI_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    }
    return MPPI_OK;
}
