// Tile autotuner: samples per tile S for a (model, K, T, J, P, costmap,
// smoothing, cost mode) shape.  S sets the tile's reduction order, so one shape must get
// one S in every process for its results to repeat; the choice is looked up,
// in order, in
//   1. the process's own cache (every choice made or read so far),
//   2. the tuning cache file named by MPPI_TUNE_CACHE (if set),
//   3. the table of measured choices shipped beside the library
//      (tile_table.txt, written by the package's tune script on an MI355X;
//      MPPI_TILE_TABLE names another file, or none when empty),
// and only then measured: every candidate that fits is timed on the
// controller's own data with scratch outputs (unless MPPI_AUTOTUNE=0, which
// takes the heuristic), and the choice is appended to the cache file.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "mppi_internal.hpp"
#include "mppi_runtime.hpp"

using namespace dbas;

namespace {

using ShapeKey = std::tuple<int, int, int, int, int, int, int, int>;   // model K T J P map sgf_m cost_mode
std::mutex g_tune_mu;
std::map<ShapeKey, int> g_tune_cache;
bool g_tables_read = false;

bool autotune_enabled()
{
    const char* v = std::getenv("MPPI_AUTOTUNE");
    return !(v && v[0] == '0');
}

std::string library_dir()
{
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&library_dir), &info) && info.dli_fname) {
        std::string s = info.dli_fname;
        const size_t slash = s.rfind('/');
        return slash == std::string::npos ? std::string(".") : s.substr(0, slash);
    }
    return ".";
}

bool shape_ok(const ShapeKey& k, int S)
{
    const int K = std::get<1>(k), T = std::get<2>(k), J = std::get<3>(k), sgf = std::get<6>(k);
    const int n = state_dim(std::get<0>(k));
    return tile_samples_supported(S) && tile_fits(J, T, n, S, sgf) && (K + S - 1) / S <= kMaxTiles;
}

// Lines "model K T J P map sgf_m cost_mode S"; '#' starts a comment line.
// The first entry of a shape wins.
void read_table(const char* path)
{
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int v[9];
        if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7],
                        &v[8]) != 9)
            continue;
        const ShapeKey k{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
        if (v[0] >= MPPI_QUAD6 && v[0] <= MPPI_CAR && shape_ok(k, v[8])) g_tune_cache.emplace(k, v[8]);
    }
    std::fclose(f);
}

void read_tables_locked()
{
    if (g_tables_read) return;
    g_tables_read = true;
    read_table(std::getenv("MPPI_TUNE_CACHE"));
    const char* table = std::getenv("MPPI_TILE_TABLE");
    if (table) read_table(table);
    else read_table((library_dir() + "/tile_table.txt").c_str());
}

void append_cache(const ShapeKey& k, int S)
{
    const char* path = std::getenv("MPPI_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), S);
    std::fclose(f);
}

// Time the rollout kernel of `h` with S samples per tile; returns ms or -1.
float time_rollout(mppi_ctrl* h, int S, int reps)
{
    DevParams q = h->p;
    q.spt = S;
    q.tiles = (q.K + q.spt - 1) / q.spt;
    const size_t tiles = (size_t)q.tiles;
    void* buf = nullptr;
    const size_t bytes = sizeof(CtrlState) + sizeof(float) * ((size_t)q.T * kM * q.Kp + 3 * (size_t)q.Kp) +
                         sizeof(double) * (3 * tiles + 2 * (size_t)q.T * tiles) + sizeof(int32_t) * tiles + 256;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return -1.0f;
    }
    char* c = static_cast<char*>(buf);
    auto take = [&](size_t n) {
        char* r = c;
        c += (n + 15) & ~(size_t)15;
        return r;
    };
    q.st = reinterpret_cast<CtrlState*>(take(sizeof(CtrlState)));
    q.du = reinterpret_cast<float*>(take(sizeof(float) * (size_t)q.T * kM * q.Kp));
    q.S = reinterpret_cast<float*>(take(sizeof(float) * 2 * (size_t)q.Kp));
    q.e = reinterpret_cast<float*>(take(sizeof(float) * (size_t)q.Kp));
    q.rho_b = reinterpret_cast<double*>(take(sizeof(double) * tiles));
    q.eta_b = reinterpret_cast<double*>(take(sizeof(double) * tiles));
    q.f_b = reinterpret_cast<double*>(take(sizeof(double) * tiles));
    q.flag_b = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * tiles));
    q.partN = reinterpret_cast<double*>(take(sizeof(double) * 2 * (size_t)q.T * tiles));
    q.res = nullptr;
    float best = -1.0f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.parity = h->iter & 1u;
    for (int r = 0; ok && r <= reps; ++r) {
        // a fresh copy of the real state for every run
        ok = hipMemcpyAsync(q.st, h->p.st, sizeof(CtrlState), hipMemcpyDeviceToDevice, h->stream) == hipSuccess;
        ok = ok && hipEventRecord(e0, h->stream) == hipSuccess;
        ok = ok && launch_rollout(q, a, h->stream) == hipSuccess;
        ok = ok && hipEventRecord(e1, h->stream) == hipSuccess;
        ok = ok && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (ok && r > 0 && (best < 0 || ms < best)) best = ms;   // r = 0 warms up
    }
    if (!ok) (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(buf);
    return ok ? best : -1.0f;
}

}  // namespace

namespace dbas {

int choose_tile_samples(mppi_ctrl* h)
{
    const DevParams& p = h->p;
    const ShapeKey key{p.model, p.K, p.T, p.J, p.P, p.sdf != nullptr ? 1 : 0, p.sgf_m, p.cost_mode};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        read_tables_locked();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    int S = heuristic_tile_samples(p.K, p.J, p.T, p.n, p.sgf_m);
    if (S == 0) return 0;
    bool timed = false;
    if (autotune_enabled() && p.J > 0 && h->sync() == MPPI_OK) {
        float best = -1.0f;
        for (int cand : {16, 32, 64, 128, 256}) {
            if (!shape_ok(key, cand)) continue;
            const float ms = time_rollout(h, cand, 3);
            if (ms > 0 && (best < 0 || ms < best * 0.97f)) {
                best = ms;
                S = cand;
                timed = true;
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto ins = g_tune_cache.emplace(key, S);
    if (ins.second && timed) append_cache(key, S);
    return ins.first->second;
}

}  // namespace dbas
