// Scheduling core of the serving layer: the device-memory arena that holds
// in-flight sample scratch, and the admission policy that forms each launch.
// Plain C++ with no HIP dependency, so that the policy can be exercised on the
// host with a fake executor.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace dbas {
namespace serve {

// First-fit allocator over [0, capacity) with coalescing of freed ranges.
// Offsets and sizes are multiples of `align`.
class Arena {
public:
    explicit Arena(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

    void reset(size_t capacity, size_t align = 256)
    {
        align_ = align;
        cap_ = capacity / align * align;
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = peak_ = 0;
    }

    size_t round(size_t n) const { return (n + align_ - 1) / align_ * align_; }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

    bool alloc(size_t n, size_t* off)
    {
        n = round(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }

    void release(size_t off, size_t n)
    {
        n = round(n ? n : 1);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        // merge with the following range
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        // merge with the preceding range
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    // Free ranges as (offset, size), in address order (for checks).
    std::vector<std::pair<size_t, size_t>> free_ranges() const { return {free_.begin(), free_.end()}; }

private:
    size_t align_ = 256, cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Limits {
    int max_slots;     // most requests in flight over all launches
    int max_batch;     // most requests in one launch
};

struct AdmitStats {
    int64_t deferred_budget = 0;   // admissions stopped because the arena was full
    int64_t deferred_slots = 0;    // admissions stopped by max_slots
};

// Per-robot FIFO of pending tickets; a robot has at most one request in
// flight, because its next iteration starts from the warm start the current
// one writes.
class Admission {
public:
    struct Pick {
        int robot;
        int64_t ticket;
        size_t offset;     // arena offset of the request's scratch
        size_t bytes;
    };

    int add_robot(size_t scratch_bytes)
    {
        robots_.push_back(Robot{scratch_bytes, {}, false});
        return (int)robots_.size() - 1;
    }

    int robots() const { return (int)robots_.size(); }
    size_t scratch_bytes(int r) const { return robots_[r].bytes; }
    bool busy(int r) const { return robots_[r].busy; }
    size_t pending(int r) const { return robots_[r].fifo.size(); }

    // Tickets must increase over all submissions (they order admission).
    void submit(int r, int64_t ticket) { robots_[r].fifo.push_back(ticket); }

    // Is there a request that could start now if a launch were free?
    bool admissible(int in_flight, const Limits& lim) const
    {
        if (in_flight >= lim.max_slots) return false;
        for (const Robot& r : robots_)
            if (!r.busy && !r.fifo.empty()) return true;
        return false;
    }

    // Form the next launch: the oldest head-of-queue requests of idle robots,
    // while slots, the batch size and the arena allow.  Admission stops at the
    // first request whose scratch does not fit, so a large request is never
    // overtaken indefinitely by smaller ones behind it.
    std::vector<Pick> admit(Arena& arena, int in_flight, const Limits& lim, AdmitStats* st)
    {
        std::vector<std::pair<int64_t, int>> heads;
        for (int i = 0; i < (int)robots_.size(); ++i)
            if (!robots_[i].busy && !robots_[i].fifo.empty()) heads.push_back({robots_[i].fifo.front(), i});
        std::sort(heads.begin(), heads.end());
        std::vector<Pick> out;
        for (const auto& h : heads) {
            if (in_flight + (int)out.size() >= lim.max_slots) {
                if (st) ++st->deferred_slots;
                break;
            }
            if ((int)out.size() >= lim.max_batch) break;
            Robot& r = robots_[h.second];
            size_t off = 0;
            if (!arena.alloc(r.bytes, &off)) {
                if (st) ++st->deferred_budget;
                break;
            }
            r.fifo.pop_front();
            r.busy = true;
            out.push_back(Pick{h.second, h.first, off, r.bytes});
        }
        return out;
    }

    // The request of robot r finished: its scratch returns to the arena.
    void complete(Arena& arena, const Pick& p)
    {
        arena.release(p.offset, p.bytes);
        robots_[p.robot].busy = false;
    }

private:
    struct Robot {
        size_t bytes;
        std::deque<int64_t> fifo;
        bool busy;
    };
    std::vector<Robot> robots_;
};

}  // namespace serve
}  // namespace dbas
