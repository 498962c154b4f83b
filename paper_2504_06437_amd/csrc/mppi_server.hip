// Serving layer: robots submit control-step requests; a scheduler thread
// admits them (oldest first, one in flight per robot, within the launch-slot
// limit and the device-memory budget for sample scratch) and runs each admitted
// group as one persistent batched launch on a free stream, while earlier
// launches are still running on the others (continuous batching).  A thread
// per stream waits for its launch, publishes the results and returns the
// scratch to the arena.
//
// Resident per robot (device): warm start U (double-buffered), the last U*,
// the Philox counter and other iteration state, obstacles.  Per request
// (arena): noise, costs, exponentials and tile partials, i.e. everything that
// scales with K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mppi_internal.hpp"
#include "mppi_runtime.hpp"
#include "server_core.hpp"

using namespace dbas;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Byte offsets, within one request's scratch, of the buffers an iteration of
// controller p writes.
struct ScratchLayout {
    size_t du, S, e, rho_b, eta_b, f_b, flag_b, partN, total;
};

ScratchLayout scratch_layout(const DevParams& p)
{
    ScratchLayout L{};
    size_t o = 0;
    auto take = [&](size_t n) {
        const size_t r = o;
        o += align256(n);
        return r;
    };
    L.du = take(p.export_noise ? sizeof(float) * (size_t)p.T * kM * p.Kp : 0);
    L.S = take(sizeof(float) * 2 * (size_t)p.Kp);
    L.e = take(sizeof(float) * (size_t)p.Kp);
    L.rho_b = take(sizeof(double) * (size_t)p.tiles);
    L.eta_b = take(sizeof(double) * (size_t)p.tiles);
    L.f_b = take(sizeof(double) * (size_t)p.tiles);
    L.flag_b = take(sizeof(int32_t) * (size_t)p.tiles);
    L.partN = take(sizeof(double) * 2 * (size_t)p.T * (size_t)p.tiles);
    L.total = o;
    return L;
}

struct Request {
    int32_t robot = 0;
    float x0[MPPI_NMAX] = {};
    std::vector<float> xref;   // empty: the robot's last reference
    double t_arrival = 0.0, t_done = 0.0;
    float u0[kM] = {0.0f, 0.0f};
    int32_t status = MPPI_OK;
    bool done = false;
};

struct Robot {
    mppi_ctrl* h = nullptr;
    std::vector<float> xref;   // last reference (host copy, staged with every launch)
    ScratchLayout layout{};
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;          // owned by a launch from admission to completion
    bool launched = false;      // the launch is issued; its waiter may take it
    hipError_t launch_error = hipSuccess;
    std::vector<serve::Admission::Pick> picks;
    char* h_stage = nullptr;    // pinned staging of the launch's inputs
    char* d_stage = nullptr;
    size_t stage_cap = 0;
    uint32_t* d_queue = nullptr;
    std::thread waiter;
};

}  // namespace

struct mppi_server {
    mppi_server_config cfg{};
    int device = 0;
    int cus = 0;
    std::mutex mu;
    std::condition_variable cv_sched;   // submissions, completions, stop
    std::condition_variable cv_done;    // request completions
    std::condition_variable cv_slot;    // issued launches (for the waiters)
    bool stop = false;
    uint64_t gen = 0;                   // bumps on every submission and completion
    std::vector<Robot> robots;
    serve::Admission adm;
    serve::Arena arena;
    char* d_arena = nullptr;
    std::vector<Slot> slots;
    std::unordered_map<int64_t, Request> reqs;
    int64_t next_ticket = 1;
    int in_flight = 0;
    mppi_server_stats stats{};
    int64_t batched_requests = 0;
    serve::AdmitStats admit_stats;
    std::thread sched;
    std::string err;

    int fail(int status, const std::string& s)
    {
        err = s;
        return status;
    }

    int free_slot() const
    {
        for (int i = 0; i < (int)slots.size(); ++i)
            if (!slots[i].busy) return i;
        return -1;
    }

    serve::Limits limits() const { return serve::Limits{cfg.max_slots, cfg.max_batch}; }

    // Lays out the launch of `picks` in the slot's pinned staging; returns the
    // bytes to copy.  Called with the lock held.
    size_t stage(Slot& sl, UnitGroups* groups, int* nrows_out, size_t* off_in, size_t* off_rows, size_t* off_units,
                 int* nexp_out, size_t* off_exp, size_t* lds_exp_out);
    void scheduler();
    void waiter(int si);
};

size_t mppi_server::stage(Slot& sl, UnitGroups* groups, int* nrows_out, size_t* off_in, size_t* off_rows,
                          size_t* off_units, int* nexp_out, size_t* off_exp, size_t* lds_exp_out)
{
    const auto& picks = sl.picks;
    const int n = (int)picks.size();
    int nunits = 0, nrows = 0;
    size_t ref_floats = 0;
    for (const auto& pk : picks) {
        const DevParams& p = robots[pk.robot].h->p;
        nunits += p.tiles;
        nrows += (2 * p.T + kUpdBlock / kWave - 1) / (kUpdBlock / kWave);
        ref_floats += (size_t)(p.T + 1) * p.n;
    }
    size_t o = 0;
    const size_t off_params = o;
    o += align256(sizeof(DevParams) * n);
    *off_in = o;
    o += align256(sizeof(BatchIn) * n);
    *off_rows = o;
    o += align256(sizeof(RowUnit) * nrows);
    *off_units = o;
    o += align256(sizeof(BatchUnit) * nunits);
    *off_exp = o;
    o += align256(sizeof(int32_t) * n);
    const size_t off_ref = o;
    o += align256(sizeof(float) * ref_floats);
    const size_t total = o;

    if (total > sl.stage_cap) {
        // the slot is idle: its last launch has completed
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        if (sl.d_stage) (void)hipFree(sl.d_stage);
        sl.h_stage = nullptr;
        sl.d_stage = nullptr;
        sl.stage_cap = 0;
        const size_t cap = total * 2;
        if (hipHostMalloc(reinterpret_cast<void**>(&sl.h_stage), cap, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&sl.d_stage), cap) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        sl.stage_cap = cap;
    }

    auto* params = reinterpret_cast<DevParams*>(sl.h_stage + off_params);
    auto* in = reinterpret_cast<BatchIn*>(sl.h_stage + *off_in);
    auto* rows = reinterpret_cast<RowUnit*>(sl.h_stage + *off_rows);
    auto* units = reinterpret_cast<BatchUnit*>(sl.h_stage + *off_units);
    float* refs = reinterpret_cast<float*>(sl.h_stage + off_ref);
    auto* exp_ids = reinterpret_cast<int32_t*>(sl.h_stage + *off_exp);
    int nexp = 0;
    size_t lds_exp = 0;
    size_t ref_at = 0;
    std::vector<BatchWork> work;
    work.reserve(nunits);
    int r_at = 0;
    for (int i = 0; i < n; ++i) {
        Robot& rb = robots[picks[i].robot];
        Request& rq = reqs[picks[i].ticket];
        mppi_ctrl* h = rb.h;
        DevParams q = h->p;
        q.lg_pack = tile_lg_pack(q.J, q.T, q.n, q.spt, q.P);
        char* base = d_arena + picks[i].offset;
        const ScratchLayout& L = rb.layout;
        q.du = q.export_noise ? reinterpret_cast<float*>(base + L.du) : nullptr;
        q.S = reinterpret_cast<float*>(base + L.S);
        q.e = reinterpret_cast<float*>(base + L.e);
        q.rho_b = reinterpret_cast<double*>(base + L.rho_b);
        q.eta_b = reinterpret_cast<double*>(base + L.eta_b);
        q.f_b = reinterpret_cast<double*>(base + L.f_b);
        q.flag_b = reinterpret_cast<int32_t*>(base + L.flag_b);
        q.partN = reinterpret_cast<double*>(base + L.partN);
        const size_t cnt = (size_t)(q.T + 1) * q.n;
        if (!rq.xref.empty()) rb.xref.swap(rq.xref);
        std::memcpy(refs + ref_at, rb.xref.data(), sizeof(float) * cnt);
        q.xref = reinterpret_cast<const float*>(sl.d_stage + off_ref) + ref_at;
        ref_at += cnt;
        params[i] = q;

        std::memset(&in[i], 0, sizeof(BatchIn));
        std::memcpy(in[i].x0, rq.x0, sizeof(float) * q.n);
        in[i].parity = h->iter & 1u;
        ++h->iter;

        for (int r = 0; r < 2 * q.T; r += kUpdBlock / kWave) rows[r_at++] = RowUnit{i, r};
        const double cost = tile_cost(q.spt, q.K, q.T, q.P, q.J);
        const size_t lds = tile_lds_bytes(q.J, q.T, q.n, q.spt);
        const int group = batch_group(q);
        for (int t = 0; t < q.tiles; ++t) work.push_back({cost, group, lds, BatchUnit{i, t}});
        if (q.adaptive) {
            exp_ids[nexp++] = i;
            lds_exp = std::max(lds_exp, explore_lds_bytes(q.J, q.T));
        }
    }
    *nexp_out = nexp;
    *lds_exp_out = lds_exp;
    *groups = group_units(work, units);
    *nrows_out = nrows;
    return total;
}

void mppi_server::scheduler()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t seen = ~0ull;
    for (;;) {
        cv_sched.wait(lk, [&] {
            return stop || (gen != seen && free_slot() >= 0 && adm.admissible(in_flight, limits()));
        });
        if (stop) break;
        seen = gen;
        const int si = free_slot();
        Slot& sl = slots[si];
        sl.picks = adm.admit(arena, in_flight, limits(), &admit_stats);
        if (sl.picks.empty()) continue;     // budget or slots: wait for a completion
        seen = ~0ull;                       // look again at once: more may fit in another slot
        sl.busy = true;
        in_flight += (int)sl.picks.size();
        size_t off_in = 0, off_rows = 0, off_units = 0, off_exp = 0, lds_exp = 0;
        int nrows = 0, nexp = 0;
        UnitGroups groups{};
        const size_t bytes = stage(sl, &groups, &nrows, &off_in, &off_rows, &off_units, &nexp, &off_exp, &lds_exp);
        ++stats.launches;
        batched_requests += (int64_t)sl.picks.size();
        lk.unlock();
        hipError_t e = bytes ? hipSuccess : hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipMemcpyAsync(sl.d_stage, sl.h_stage, bytes, hipMemcpyHostToDevice, sl.stream);
        const auto* d_params = reinterpret_cast<const DevParams*>(sl.d_stage);
        const auto* d_in = reinterpret_cast<const BatchIn*>(sl.d_stage + off_in);
        const auto* d_rows = reinterpret_cast<const RowUnit*>(sl.d_stage + off_rows);
        const auto* d_units = reinterpret_cast<const BatchUnit*>(sl.d_stage + off_units);
        if (e == hipSuccess) e = launch_batch_rollouts(d_params, d_units, groups, d_in, sl.d_queue, cus, sl.stream);
        if (e == hipSuccess) e = launch_batch_update(d_params, d_rows, nrows, d_in, nullptr, sl.stream);
        if (e == hipSuccess && nexp)
            e = launch_batch_explore(d_params, reinterpret_cast<const int32_t*>(sl.d_stage + off_exp), nexp, d_in,
                                     lds_exp, sl.stream);
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
        if (e != hipSuccess) (void)hipGetLastError();
        lk.lock();
        sl.launch_error = e;
        sl.launched = true;
        cv_slot.notify_all();
    }
}

void mppi_server::waiter(int si)
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    Slot& sl = slots[si];
    for (;;) {
        cv_slot.wait(lk, [&] { return sl.launched || stop; });
        if (!sl.launched) break;            // stopping, and nothing of this slot is in flight
        hipError_t e = sl.launch_error;
        lk.unlock();
        if (e == hipSuccess) e = hipEventSynchronize(sl.done);
        const double t = now_s();
        lk.lock();
        for (const auto& pk : sl.picks) {
            Request& rq = reqs[pk.ticket];
            const HostResult* hr = robots[pk.robot].h->h_res;
            if (e == hipSuccess) {
                rq.u0[0] = hr->u0[0];
                rq.u0[1] = hr->u0[1];
                rq.status = hr->status;
            } else {
                rq.status = MPPI_E_DEVICE;
            }
            rq.t_done = t;
            rq.done = true;
            adm.complete(arena, pk);
            ++stats.completed;
        }
        if (e != hipSuccess) err = std::string("launch failed: ") + hipGetErrorString(e);
        in_flight -= (int)sl.picks.size();
        sl.picks.clear();
        sl.launched = false;
        sl.busy = false;
        ++gen;
        cv_sched.notify_all();
        cv_done.notify_all();
    }
}

namespace {

void destroy_server(mppi_server* s)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    if (s->sched.joinable()) s->sched.join();
    s->cv_slot.notify_all();
    for (Slot& sl : s->slots)
        if (sl.waiter.joinable()) sl.waiter.join();
    (void)hipSetDevice(s->device);
    for (Robot& r : s->robots) delete r.h;
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        if (sl.d_stage) (void)hipFree(sl.d_stage);
        if (sl.d_queue) (void)hipFree(sl.d_queue);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->d_arena) (void)hipFree(s->d_arena);
    delete s;
}

}  // namespace

extern "C" int mppi_server_create(const mppi_server_config* cfg, mppi_server_t** out)
{
    if (!out) return MPPI_E_INVALID;
    *out = nullptr;
    if (!cfg) return MPPI_E_INVALID;
    if (cfg->abi_version != MPPI_ABI_VERSION) {
        set_global_error("mppi_server_create: abi_version mismatch");
        return MPPI_E_INVALID;
    }
    if (cfg->budget_bytes <= 0 || cfg->max_slots < 1 || cfg->streams < 1 || cfg->streams > 8 || cfg->max_batch < 1) {
        set_global_error("mppi_server_create: need budget_bytes > 0, max_slots >= 1, 1 <= streams <= 8, max_batch >= 1");
        return MPPI_E_INVALID;
    }
    mppi_server* s = new (std::nothrow) mppi_server();
    if (!s) return MPPI_E_NOMEM;
    s->cfg = *cfg;
    s->device = cfg->device;
    s->slots.resize(cfg->streams);
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_arena), (size_t)cfg->budget_bytes);
    for (Slot& sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreate(&sl.stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sl.d_queue), sizeof(uint32_t) * 2 * kBatchGroups);
        if (e == hipSuccess) e = hipMemset(sl.d_queue, 0, sizeof(uint32_t) * 2 * kBatchGroups);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_global_error(std::string("mppi_server_create: ") + hipGetErrorString(e));
        destroy_server(s);
        return e == hipErrorOutOfMemory ? MPPI_E_NOMEM : MPPI_E_DEVICE;
    }
    s->arena.reset((size_t)cfg->budget_bytes);
    for (int i = 0; i < (int)s->slots.size(); ++i) s->slots[i].waiter = std::thread(&mppi_server::waiter, s, i);
    s->sched = std::thread(&mppi_server::scheduler, s);
    *out = s;
    return MPPI_OK;
}

extern "C" void mppi_server_destroy(mppi_server_t* s)
{
    if (s) destroy_server(s);
}

extern "C" int mppi_server_add_robot(mppi_server_t* s, const mppi_config* cfg, int32_t J, const float* cxcyr,
                                     int32_t* id)
{
    if (!s || !cfg || !id) return MPPI_E_INVALID;
    mppi_device dev;
    std::memset(&dev, 0, sizeof dev);
    dev.device = s->device;
    dev.stream = s->slots[0].stream;
    mppi_ctrl* h = nullptr;
    int st = create_ctrl(cfg, &dev, true, &h);
    if (st) {
        std::lock_guard<std::mutex> lk(s->mu);
        return s->fail(st, std::string("add_robot: ") + global_error());
    }
    st = mppi_set_obstacles(h, J, cxcyr, MPPI_MEM_HOST);
    if (st) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->fail(st, "add_robot: " + h->err);
        delete h;
        return st;
    }
    Robot rb;
    rb.h = h;
    rb.xref.assign((size_t)(cfg->T + 1) * h->p.n, 0.0f);
    rb.layout = scratch_layout(h->p);
    std::lock_guard<std::mutex> lk(s->mu);
    if (rb.layout.total > s->arena.capacity()) {
        delete h;
        return s->fail(MPPI_E_INVALID, "add_robot: one request needs " + std::to_string(rb.layout.total) +
                                           " scratch bytes, more than the budget");
    }
    s->robots.push_back(std::move(rb));
    *id = s->adm.add_robot(s->robots.back().layout.total);
    return MPPI_OK;
}

extern "C" int mppi_server_submit(mppi_server_t* s, int32_t id, const float* x0, const float* x_ref,
                                  double t_arrival, int64_t* ticket)
{
    if (!s || !x0 || !ticket) return MPPI_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int)s->robots.size()) return s->fail(MPPI_E_INVALID, "submit: unknown robot id");
    const mppi_ctrl* h = s->robots[id].h;
    const int n = h->p.n;
    for (int a = 0; a < n; ++a)
        if (!std::isfinite(x0[a])) return s->fail(MPPI_E_INVALID, "submit: non-finite x0");
    Request rq;
    rq.robot = id;
    std::memcpy(rq.x0, x0, sizeof(float) * n);
    if (x_ref) {
        const size_t cnt = (size_t)(h->cfg.T + 1) * n;
        for (size_t i = 0; i < cnt; ++i)
            if (!std::isfinite(x_ref[i])) return s->fail(MPPI_E_INVALID, "submit: non-finite reference");
        rq.xref.assign(x_ref, x_ref + cnt);
    }
    rq.t_arrival = t_arrival;
    const int64_t t = s->next_ticket++;
    s->reqs.emplace(t, std::move(rq));
    s->adm.submit(id, t);
    ++s->stats.submitted;
    ++s->gen;
    *ticket = t;
    lk.unlock();
    s->cv_sched.notify_one();
    return MPPI_OK;
}

namespace {

int take_result(mppi_server* s, std::unordered_map<int64_t, Request>::iterator it, float* u0, double* latency,
                int32_t* status)
{
    const Request& rq = it->second;
    if (u0) {
        u0[0] = rq.u0[0];
        u0[1] = rq.u0[1];
    }
    if (latency) *latency = rq.t_done - rq.t_arrival;
    if (status) *status = rq.status;
    s->reqs.erase(it);
    return MPPI_OK;
}

}  // namespace

extern "C" int mppi_server_poll(mppi_server_t* s, int64_t ticket, float* u0, double* latency, int32_t* status)
{
    if (!s) return MPPI_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return s->fail(MPPI_E_INVALID, "poll: unknown ticket");
    if (!it->second.done) return MPPI_E_BUSY;
    return take_result(s, it, u0, latency, status);
}

extern "C" int mppi_server_wait(mppi_server_t* s, int64_t ticket, float* u0, double* latency, int32_t* status)
{
    if (!s) return MPPI_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return s->fail(MPPI_E_INVALID, "wait: unknown ticket");
    s->cv_done.wait(lk, [&] { return it->second.done; });
    return take_result(s, it, u0, latency, status);
}

extern "C" double mppi_server_now(const mppi_server_t*) { return now_s(); }

extern "C" int mppi_server_get_stats(mppi_server_t* s, mppi_server_stats* out)
{
    if (!s || !out) return MPPI_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->deferred_budget = s->admit_stats.deferred_budget;
    out->deferred_slots = s->admit_stats.deferred_slots;
    out->peak_bytes_in_flight = (int64_t)s->arena.peak();
    out->mean_batch = s->stats.launches ? (double)s->batched_requests / (double)s->stats.launches : 0.0;
    return MPPI_OK;
}

extern "C" int mppi_server_get_robot(mppi_server_t* s, int32_t id, float* U, uint64_t* counter)
{
    if (!s) return MPPI_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int)s->robots.size()) return s->fail(MPPI_E_INVALID, "get_robot: unknown robot id");
    s->cv_done.wait(lk, [&] { return !s->adm.busy(id) && s->adm.pending(id) == 0; });
    mppi_ctrl* h = s->robots[id].h;
    hipError_t e = hipSetDevice(s->device);
    if (U && e == hipSuccess)
        e = hipMemcpy(U, h->p.U + (size_t)(h->iter & 1u) * h->cfg.T * kM, sizeof(float) * h->cfg.T * kM,
                      hipMemcpyDeviceToHost);
    if (counter && e == hipSuccess) {
        CtrlState cs;
        e = hipMemcpy(&cs, h->p.st, sizeof cs, hipMemcpyDeviceToHost);
        *counter = cs.counter;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return s->fail(MPPI_E_DEVICE, std::string("get_robot: ") + hipGetErrorString(e));
    }
    return MPPI_OK;
}

extern "C" const char* mppi_server_last_error(const mppi_server_t* s)
{
    return s ? s->err.c_str() : global_error();
}
