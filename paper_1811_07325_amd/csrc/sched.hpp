// Host-only parts of the serving engine, free of device calls so that they
// can be tested on any machine: the first-fit arena that places requests in
// device memory, the percentile rule of the latency statistics, one
// admission pass of the scheduler, and the size-aware order and large-request
// cap it runs with by default.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace stk {

// First-fit allocator over [0, size) in 256-byte units, coalescing freed
// ranges with their neighbours.
class Arena {
public:
    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size) {
        free_.clear();
        size_ = size;
        used_ = 0;
        if (size) free_[0] = size;
    }

    bool alloc(size_t bytes, size_t* off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }

    void free(size_t off, size_t bytes) {
        bytes = round(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);   // merge with the next range
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {  // merge with the previous range
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    static size_t round(size_t b) { return (b + 255) / 256 * 256; }
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0, used_ = 0;
};

// Nearest-rank percentile (0 < q <= 1) of ascending values; 0 when empty.
inline double nearest_rank(const std::vector<double>& sorted, double q) {
    if (sorted.empty()) return 0.0;
    const size_t rank = (size_t)std::max(1.0, std::ceil(q * (double)sorted.size()));
    return sorted[std::min(rank, sorted.size()) - 1];
}

// One admission pass over `waiting` (arrival order).  While slot_free(),
// each request is offered to take(q): true removes it from the queue
// (admitted, or failed for good); false means it does not fit now, and it is
// passed over and counted in q->passed.  The pass ends after max_pass
// requests were passed over; and once the oldest request has been passed
// over more than max_head_passes times nothing behind it is admitted any
// more, so the requests in flight drain until it fits: no request waits
// forever.  Returns the number of requests removed.
template <class Req, class SlotFree, class Take>
int admission_pass(std::deque<Req*>& waiting, SlotFree slot_free, Take take, int max_pass, int max_head_passes) {
    int removed = 0, passed = 0;
    for (auto it = waiting.begin(); it != waiting.end();) {
        if (!slot_free()) break;
        const bool head = it == waiting.begin();
        if (head && (*it)->passed > max_head_passes) {
            // the oldest request has waited long enough: only it may go next
            if (take(*it)) {
                waiting.erase(it);
                ++removed;
                it = waiting.begin();
                continue;
            }
            ++(*it)->passed;
            break;
        }
        if (take(*it)) {
            it = waiting.erase(it);
            ++removed;
            continue;
        }
        ++(*it)->passed;
        if (++passed > max_pass) break;
        ++it;
    }
    return removed;
}

// Size-aware admission order (applied before each admission pass):
// requests that have waited longer than `aging` first, oldest first, so none
// waits for ever; the others by ascending modelled cost, ties in arrival
// order.  Small requests then no longer queue behind large ones.
template <class Req, class Arrival, class Cost>
void order_waiting(std::deque<Req*>& waiting, double now, double aging, Arrival arrival, Cost cost) {
    std::stable_sort(waiting.begin(), waiting.end(), [&](const Req* a, const Req* b) {
        const bool oa = now - arrival(a) > aging, ob = now - arrival(b) > aging;
        if (oa != ob) return oa;
        if (oa) return arrival(a) < arrival(b);
        return cost(a) < cost(b);
    });
}

// At most `cap` requests whose modelled cost reaches `threshold` in flight:
// a large request's kernels then share the device with small ones only, and
// large requests queue for each other instead of stretching each other's
// service time.
struct LargeCap {
    double threshold = 0;
    int cap = 1;
    int inflight = 0;
    bool large(double cost) const { return cost >= threshold; }
    bool admits(double cost) const { return !large(cost) || inflight < cap; }
};

}  // namespace stk
