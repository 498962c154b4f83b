// Host-only check of the serving layer's scheduling core (arena + admission)
// with a fake executor: random robots, random submissions and launches that
// complete after random delays.  Prints "OK" and exits 0 when every invariant
// held; prints the first violation and exits 1 otherwise.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "server_core.hpp"

using dbas::serve::Admission;
using dbas::serve::AdmitStats;
using dbas::serve::Arena;
using dbas::serve::Limits;

#define CHECK(cond, ...)                                                   \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::printf("FAIL line %d: %s: ", __LINE__, #cond);            \
            std::printf(__VA_ARGS__);                                      \
            std::printf("\n");                                             \
            std::exit(1);                                                  \
        }                                                                  \
    } while (0)

static void check_arena_layout(const Arena& a)
{
    size_t free_total = 0, last_end = 0;
    bool first = true;
    for (auto& r : a.free_ranges()) {
        CHECK(r.second > 0, "empty free range");
        CHECK(r.first + r.second <= a.capacity(), "free range beyond capacity");
        if (!first) CHECK(r.first > last_end, "free ranges overlap or touch without coalescing (%zu, %zu)", r.first, last_end);
        last_end = r.first + r.second;
        free_total += r.second;
        first = false;
    }
    CHECK(free_total + a.used() == a.capacity(), "used %zu + free %zu != capacity %zu", a.used(), free_total,
          a.capacity());
}

static void arena_unit()
{
    Arena a(4096, 256);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0, "first fit at 0");
    CHECK(a.alloc(256, &o2) && o2 == 256, "second at 256");
    CHECK(a.alloc(1000, &o3) && o3 == 512, "third at 512");
    CHECK(a.used() == 256 + 256 + 1024, "used after three");
    a.release(o2, 256);
    check_arena_layout(a);
    CHECK(a.alloc(200, &o4) && o4 == 256, "hole reused");
    a.release(o1, 100);
    a.release(o4, 200);
    a.release(o3, 1000);
    check_arena_layout(a);
    CHECK(a.used() == 0 && a.free_ranges().size() == 1, "all coalesced back");
    CHECK(a.peak() == 1536, "peak %zu", a.peak());
    size_t big;
    CHECK(!a.alloc(4097, &big), "oversize refused");
    CHECK(a.alloc(4096, &big) && big == 0, "whole arena");
    size_t none;
    CHECK(!a.alloc(1, &none), "full arena refuses");
    a.release(big, 4096);

    // random alloc/free keeps the free list exact
    std::mt19937_64 rng(11);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || (rng() % 3 != 0)) {
            size_t n = 1 + rng() % 900, off;
            if (a.alloc(n, &off)) {
                for (auto& l : live)
                    CHECK(off + a.round(n) <= l.first || l.first + a.round(l.second) <= off, "overlapping allocations");
                live.push_back({off, n});
            }
        } else {
            size_t i = rng() % live.size();
            a.release(live[i].first, live[i].second);
            live.erase(live.begin() + i);
        }
        if (it % 97 == 0) check_arena_layout(a);
    }
    for (auto& l : live) a.release(l.first, l.second);
    check_arena_layout(a);
    CHECK(a.used() == 0, "all released");
}

struct Launch {
    std::vector<Admission::Pick> picks;
    int finish_at;
};

static void admission_sim(uint64_t seed, int n_robots, size_t budget, Limits lim, int streams, int n_requests)
{
    std::mt19937_64 rng(seed);
    Arena arena(budget, 256);
    Admission adm;
    std::vector<size_t> bytes(n_robots);
    for (int r = 0; r < n_robots; ++r) {
        bytes[r] = 256 * (1 + rng() % (budget / 256 / 3));   // each fits the budget alone
        CHECK(adm.add_robot(bytes[r]) == r, "robot ids are dense");
    }
    std::vector<std::vector<int64_t>> submitted(n_robots), completed(n_robots);
    std::map<int64_t, int> owner;
    std::vector<Launch> running;
    AdmitStats st;
    int64_t next_ticket = 1;
    int in_flight = 0, submitted_n = 0, completed_n = 0, launches = 0, clock = 0;
    size_t in_flight_bytes = 0;
    while (completed_n < n_requests) {
        ++clock;
        // arrivals
        int arrivals = submitted_n < n_requests ? (int)(rng() % 4) : 0;
        for (int i = 0; i < arrivals && submitted_n < n_requests; ++i) {
            int r = (int)(rng() % n_robots);
            adm.submit(r, next_ticket);
            submitted[r].push_back(next_ticket);
            owner[next_ticket] = r;
            ++next_ticket;
            ++submitted_n;
        }
        // completions
        for (size_t i = 0; i < running.size();) {
            if (running[i].finish_at <= clock) {
                for (auto& p : running[i].picks) {
                    adm.complete(arena, p);
                    completed[p.robot].push_back(p.ticket);
                    in_flight_bytes -= arena.round(p.bytes);
                    --in_flight;
                    ++completed_n;
                }
                running.erase(running.begin() + i);
            } else {
                ++i;
            }
        }
        // launches while a stream is free
        while ((int)running.size() < streams && adm.admissible(in_flight, lim)) {
            // heads of idle robots before admission
            std::vector<std::pair<int64_t, int>> heads;
            for (int r = 0; r < n_robots; ++r) {
                const size_t done = completed[r].size() + (adm.busy(r) ? 1 : 0);
                if (!adm.busy(r) && adm.pending(r) > 0) heads.push_back({submitted[r][done], r});
            }
            std::sort(heads.begin(), heads.end());
            auto picks = adm.admit(arena, in_flight, lim, &st);
            if (picks.empty()) break;
            CHECK((int)picks.size() <= lim.max_batch, "batch %zu > max_batch", picks.size());
            // the picks are exactly the oldest heads, in order
            for (size_t i = 0; i < picks.size(); ++i) {
                CHECK(picks[i].ticket == heads[i].first && picks[i].robot == heads[i].second,
                      "pick %zu is not the %zu-th oldest head", i, i);
                CHECK(owner[picks[i].ticket] == picks[i].robot, "ticket owner");
                CHECK(picks[i].bytes == bytes[picks[i].robot], "scratch size");
                in_flight_bytes += arena.round(picks[i].bytes);
            }
            in_flight += (int)picks.size();
            CHECK(in_flight <= lim.max_slots, "in flight %d > max_slots", in_flight);
            CHECK(arena.used() == in_flight_bytes && arena.used() <= arena.capacity(), "arena accounting");
            std::set<int> robots_in_flight;
            for (auto& l : running)
                for (auto& p : l.picks) robots_in_flight.insert(p.robot);
            for (auto& p : picks) {
                CHECK(!robots_in_flight.count(p.robot), "robot %d has two requests in flight", p.robot);
                robots_in_flight.insert(p.robot);
            }
            running.push_back(Launch{picks, clock + 1 + (int)(rng() % 5)});
            ++launches;
        }
        check_arena_layout(arena);
        CHECK(clock < 10 * n_requests + 1000, "no progress (liveness)");
    }
    for (int r = 0; r < n_robots; ++r) CHECK(completed[r] == submitted[r], "robot %d served out of order", r);
    CHECK(arena.used() == 0 && in_flight == 0, "drained");
    std::printf("sim seed=%llu robots=%d budget=%zu slots=%d batch=%d streams=%d: %d requests, %d launches, "
                "deferred budget %lld slots %lld, peak %zu\n",
                (unsigned long long)seed, n_robots, budget, lim.max_slots, lim.max_batch, streams, n_requests, launches,
                (long long)st.deferred_budget, (long long)st.deferred_slots, arena.peak());
}

int main()
{
    arena_unit();
    admission_sim(1, 16, 1 << 20, Limits{64, 64}, 2, 5000);
    admission_sim(2, 64, 1 << 16, Limits{64, 16}, 2, 5000);      // small budget: admission deferred
    admission_sim(3, 256, 1 << 22, Limits{8, 4}, 3, 20000);      // few slots
    admission_sim(4, 3, 1 << 14, Limits{1, 1}, 1, 2000);         // one at a time
    std::printf("OK\n");
    return 0;
}
