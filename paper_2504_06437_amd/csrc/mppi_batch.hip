// Batched iteration of many controllers in one persistent launch, captured
// once into a HIP graph, and the library's global error slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mppi_internal.hpp"
#include "mppi_runtime.hpp"

using namespace dbas;

namespace {
thread_local std::string g_error;
}

void set_global_error(const std::string& s) { g_error = s; }
const char* global_error() { return g_error.c_str(); }

// ---------------------------------------------------------------------------
// Batch
// ---------------------------------------------------------------------------
struct mppi_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<mppi_ctrl*> ctrls;
    std::vector<uint64_t> versions;
    std::vector<DevParams> params;
    DevParams* d_params = nullptr;
    BatchUnit* d_units = nullptr;
    RowUnit* d_rows = nullptr;
    int32_t* d_exp = nullptr;       // controllers with adaptive exploration
    uint32_t* d_queue = nullptr;
    BatchIn* d_in = nullptr;
    BatchIn* h_in = nullptr;        // pinned staging of the per-step states and buffer parities
    int nunits = 0, nrows = 0, nexp = 0;
    UnitGroups groups{};
    size_t lds_exp = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;

    ~mppi_batch()
    {
        (void)hipSetDevice(device);
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* p : {(void*)d_params, (void*)d_units, (void*)d_rows, (void*)d_exp, (void*)d_queue, (void*)d_in})
            if (p) (void)hipFree(p);
        if (h_in) (void)hipHostFree(h_in);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    int fail(int st, const std::string& s)
    {
        err = s;
        return st;
    }

    int hip(hipError_t e, const char* what)
    {
        if (e == hipSuccess) return MPPI_OK;
        (void)hipGetLastError();
        return fail(MPPI_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }

    // (Re)build the work lists and the graph from the controllers' current shapes.
    int build()
    {
        const int n = (int)ctrls.size();
        params.resize(n);
        versions.resize(n);
        std::vector<BatchWork> work;
        std::vector<RowUnit> rows;
        std::vector<int32_t> exp_ids;
        lds_exp = 0;
        for (int c = 0; c < n; ++c) {
            params[c] = ctrls[c]->p;
            params[c].lg_pack = tile_lg_pack(params[c].J, params[c].T, params[c].n, params[c].spt, params[c].P);
            versions[c] = ctrls[c]->version;
            const DevParams& p = params[c];
            const double cost = tile_cost(p.spt, p.K, p.T, p.P, p.J);
            const size_t lds = tile_lds_bytes(p.J, p.T, p.n, p.spt);
            const int group = batch_group(p);
            for (int t = 0; t < p.tiles; ++t) work.push_back({cost, group, lds, BatchUnit{c, t}});
            for (int r = 0; r < 2 * p.T; r += kUpdBlock / kWave) rows.push_back(RowUnit{c, r});
            if (p.adaptive) {
                exp_ids.push_back(c);
                lds_exp = std::max(lds_exp, explore_lds_bytes(p.J, p.T));
            }
        }
        std::vector<BatchUnit> units(work.size());
        groups = group_units(work, units.data());
        nunits = (int)units.size();
        nrows = (int)rows.size();
        nexp = (int)exp_ids.size();

        int st;
        if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
        if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
        for (void** p : {(void**)&d_params, (void**)&d_units, (void**)&d_rows, (void**)&d_exp})
            if (*p) { (void)hipFree(*p); *p = nullptr; }
        if ((st = hip(hipMalloc(&d_params, sizeof(DevParams) * n), "hipMalloc params"))) return st;
        if ((st = hip(hipMalloc(&d_units, sizeof(BatchUnit) * nunits), "hipMalloc units"))) return st;
        if ((st = hip(hipMalloc(&d_rows, sizeof(RowUnit) * nrows), "hipMalloc rows"))) return st;
        if ((st = hip(hipMemcpy(d_params, params.data(), sizeof(DevParams) * n, hipMemcpyHostToDevice), "params"))) return st;
        if ((st = hip(hipMemcpy(d_units, units.data(), sizeof(BatchUnit) * nunits, hipMemcpyHostToDevice), "units"))) return st;
        if ((st = hip(hipMemcpy(d_rows, rows.data(), sizeof(RowUnit) * nrows, hipMemcpyHostToDevice), "rows"))) return st;
        if (nexp) {
            if ((st = hip(hipMalloc(&d_exp, sizeof(int32_t) * nexp), "hipMalloc explore list"))) return st;
            if ((st = hip(hipMemcpy(d_exp, exp_ids.data(), sizeof(int32_t) * nexp, hipMemcpyHostToDevice), "explore list")))
                return st;
        }

        int cus = 0;
        if ((st = hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "CU count"))) return st;

        // capture: per-step inputs H2D, persistent rollout, row update, and the
        // exploration rate of the controllers that adapt it
        if ((st = hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture"))) return st;
        hipError_t e = hipMemcpyAsync(d_in, h_in, sizeof(BatchIn) * n, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = launch_batch_rollouts(d_params, d_units, groups, d_in, d_queue, cus, stream);
        if (e == hipSuccess) e = launch_batch_update(d_params, d_rows, nrows, d_in, nullptr, stream);
        if (e == hipSuccess && nexp) e = launch_batch_explore(d_params, d_exp, nexp, d_in, lds_exp, stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream, &g);
        if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip(e, "captured launch"); }
        if ((st = hip(e2, "end capture"))) return st;
        graph = g;
        return hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    }
};

extern "C" int mppi_batch_create(mppi_t* const* ctrls, int32_t n, const mppi_device* dev, mppi_batch_t** out)
{
    if (!out || !ctrls || n < 1) return MPPI_E_INVALID;
    *out = nullptr;
    mppi_batch* b = new (std::nothrow) mppi_batch();
    if (!b) return MPPI_E_NOMEM;
    b->device = dev ? dev->device : 0;
    for (int c = 0; c < n; ++c) {
        if (!ctrls[c] || ctrls[c]->poisoned || ctrls[c]->device != b->device) {
            set_global_error("mppi_batch_create: controllers must be valid handles on the batch's device");
            delete b;
            return MPPI_E_INVALID;
        }
        for (int d = 0; d < c; ++d)
            if (ctrls[d] == ctrls[c]) {
                set_global_error("mppi_batch_create: a controller appears twice");
                delete b;
                return MPPI_E_INVALID;
            }
        b->ctrls.push_back(ctrls[c]);
    }
    int st = MPPI_OK;
    if (!st) st = b->hip(hipSetDevice(b->device), "hipSetDevice");
    if (!st && dev && dev->stream) b->stream = static_cast<hipStream_t>(dev->stream);
    else if (!st) {
        st = b->hip(hipStreamCreate(&b->stream), "hipStreamCreate");
        b->own_stream = true;
    }
    for (mppi_ctrl* c : b->ctrls)
        if (!st) st = c->sync();
    if (!st) st = b->hip(hipMalloc(&b->d_queue, sizeof(uint32_t) * 2 * kBatchGroups), "hipMalloc queue");
    if (!st) st = b->hip(hipMemset(b->d_queue, 0, sizeof(uint32_t) * 2 * kBatchGroups), "queue init");
    if (!st) st = b->hip(hipMalloc(&b->d_in, sizeof(BatchIn) * n), "hipMalloc inputs");
    if (!st) st = b->hip(hipHostMalloc(reinterpret_cast<void**>(&b->h_in), sizeof(BatchIn) * n, 0), "hipHostMalloc inputs");
    if (!st) {
        std::memset(b->h_in, 0, sizeof(BatchIn) * n);
        st = b->build();
    }
    if (st) {
        set_global_error(b->err);
        delete b;
        return st;
    }
    *out = b;
    return MPPI_OK;
}

extern "C" void mppi_batch_destroy(mppi_batch_t* b) { delete b; }

extern "C" int mppi_batch_step(mppi_batch_t* b, const float* x0s, float* u0s, int32_t* statuses)
{
    if (!b || !x0s || !u0s) return MPPI_E_INVALID;
    const int n = (int)b->ctrls.size();
    int st = b->hip(hipSetDevice(b->device), "hipSetDevice");
    if (st) return st;
    bool stale = false;
    for (int c = 0; c < n; ++c) {
        mppi_ctrl* h = b->ctrls[c];
        if (h->poisoned) return b->fail(MPPI_E_DEVICE, "controller handle is poisoned");
        for (int a = 0; a < h->p.n; ++a)
            if (!std::isfinite(x0s[(size_t)c * MPPI_NMAX + a])) return b->fail(MPPI_E_INVALID, "non-finite x0");
        if (h->version != b->versions[c]) stale = true;
    }
    // a controller's own stream may still hold work of a standalone step
    for (mppi_ctrl* h : b->ctrls)
        if ((st = h->sync())) return b->fail(st, h->err);
    if (stale) {
        if ((st = b->hip(hipStreamSynchronize(b->stream), "sync"))) return st;
        if ((st = b->build())) return st;
    }
    for (int c = 0; c < n; ++c) {
        BatchIn& in = b->h_in[c];
        std::memset(&in, 0, sizeof in);
        std::memcpy(in.x0, x0s + (size_t)c * MPPI_NMAX, sizeof(float) * b->ctrls[c]->p.n);
        in.parity = b->ctrls[c]->iter & 1u;
    }
    if ((st = b->hip(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch"))) return st;
    for (mppi_ctrl* h : b->ctrls) ++h->iter;
    if ((st = b->hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize"))) return st;
    int first = MPPI_OK;
    for (int c = 0; c < n; ++c) {
        const HostResult* r = b->ctrls[c]->h_res;
        u0s[2 * c] = r->u0[0];
        u0s[2 * c + 1] = r->u0[1];
        if (statuses) statuses[c] = r->status;
        if (r->status != MPPI_OK && first == MPPI_OK) first = r->status;
    }
    return first;
}

extern "C" const char* mppi_batch_last_error(const mppi_batch_t* b) { return b ? b->err.c_str() : global_error(); }
