// Serving engine: continuous batching of independent multiply requests.
//
// Requests arrive through stark_submit (any thread) into a queue.  An engine
// thread admits them whenever a slot (a HIP stream of its own) is free and
// the request's device footprint fits the remaining HBM budget: smallest
// modelled time first (requests that have waited long first of all), at most
// one large request in flight; a request that does not fit lets at most
// kMaxBypass others go first, so nothing starves.  Admitted requests run concurrently
// on their slot streams; completion is observed with HIP events and frees the
// slot and the memory for the next arrivals.  Each request's kernels and
// their order are fixed by its plan, so its result does not depend on what
// else is running.
#pragma once
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/stark.h"
#include "plan.hpp"
#include "sched.hpp"

struct stark_ctx;

namespace stk {

// Device memory of the served requests: segments allocated when admissions
// need them (at least kSegmentBytes each, at most the budget in total), each
// carved first-fit by an Arena.  A budget is not allocated up front: on a
// device whose memory was freed before, allocating tens of GiB takes seconds.
class SegmentedArena {
public:
    static constexpr size_t kSegmentBytes = size_t(4) << 30;
    enum Result { kOk, kWait, kFail };
    explicit SegmentedArena(size_t budget = 0) : budget_(budget) {}
    // `idle`: nothing is in flight, so every segment is empty and may be
    // replaced by one large enough.  kWait: no room until requests finish;
    // kFail: the device refused the memory while idle.
    Result alloc(size_t bytes, bool idle, int* seg, size_t* off);
    void free(int seg, size_t off, size_t bytes) { segs_[seg].arena.free(off, bytes); used_ -= round(bytes); }
    char* base(int seg) const { return static_cast<char*>(segs_[seg].base); }
    size_t used() const { return used_; }
    size_t budget() const { return budget_; }
    size_t allocated() const { return allocated_; }
    void release();

private:
    static size_t round(size_t b) { return (b + 255) / 256 * 256; }
    struct Seg {
        void* base;
        Arena arena;
    };
    std::vector<Seg> segs_;
    size_t budget_, allocated_ = 0, used_ = 0;
};

// Depth used for a request when it asks for STARK_DEPTH_AUTO and the
// autotuner has no record for its size.
int default_serving_depth(int64_t n, int precision);

// Device bytes a request holds while it runs.
size_t request_footprint(const Plan& p, bool gen_operands, bool own_c);

class Engine {
public:
    static constexpr int kMaxBypass = 8;             // passed-over requests per admission pass
    static constexpr int kMaxHeadPasses = 1000;      // then the oldest request goes next
    static constexpr size_t kMaxQueue = 1 << 16;
    static constexpr size_t kLatWindow = 1 << 20;   // latencies kept for p50 / p99

    Engine(stark_ctx* ctx, size_t budget, int slots, hipError_t* err);
    ~Engine();

    stark_status submit(const stark_request& r, uint64_t* ticket);
    stark_status poll(uint64_t ticket, stark_result* out);
    stark_status stats(stark_stats_t* out);
    void reset_stats();

private:
    struct Req {
        uint64_t ticket = 0;
        stark_request r{};
        Plan plan;
        size_t bytes = 0, off = 0;
        int seg = -1;                 // arena segment
        int passed = 0;               // admission passes that went over it
        bool gen = false, own_c = false;
        int slot = -1;
        double t_submit = 0, t_admit = 0, t_done = 0;
        double cost_s = 0;            // modelled time on an idle device (model_seconds)
        stark_status status = STARK_OK;
        double checksum = 0;
        float gpu_ms = 0;
    };
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        double* partials = nullptr;   // device, checksum reduction
        bool busy = false;
        Req* req = nullptr;
    };

    void loop();
    bool admit(Req* q, int slot);
    void finish(int slot);
    void publish_failure(Req* q, stark_status status);

    stark_ctx* ctx_;
    double* host_sums_ = nullptr; // pinned, one per slot
    // Engine thread only (no lock): the requests waiting for admission, the
    // slots, the device memory and the count of requests in flight.
    SegmentedArena mem_;
    std::vector<Slot> slots_;
    std::deque<Req*> waiting_;
    int inflight_ = 0;
    // Guarded by mu_: arrivals, the live requests' published results, stats.
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Req*> arrivals_;
    std::map<uint64_t, Req*> live_;     // submitted, not yet polled
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    std::thread thread_;
    // statistics
    std::vector<double> lat_ms_;       // ring of the last kLatWindow latencies
    size_t lat_next_ = 0;
    uint64_t completed_ = 0, failed_ = 0;
    double flops_ = 0, first_admit_ = -1, last_done_ = 0;
    size_t max_bytes_ = 0, used_pub_ = 0, waiting_pub_ = 0;
    int inflight_pub_ = 0, max_inflight_ = 0;
    int64_t fault_tag_ = -1;   // STARK_FAULT_INJECT: tag of a request made to fail
    // leaf GEMMs of served requests launch one workgroup per tile, so that a
    // large request's GEMM does not hold every CU until it ends
    // (STARK_SERVE_PERSISTENT=1: the persistent grid of stark_gemm)
    bool persistent_ = false;
    // Admission (sched.hpp): by default the size-aware order (requests that
    // waited longer than aging_ms first, then by modelled time) and at most
    // one large request (modelled time >= 2 ms) in flight; STARK_SERVE_FIFO=1
    // admits in arrival order with no cap.  STARK_SERVE_AGING_MS,
    // STARK_SERVE_LARGE_MS and STARK_SERVE_LARGE_CAP override the defaults.
    bool fifo_ = false;
    double aging_ms_ = 25.0;
    LargeCap large_{2e-3, 1};
};

double now_us();

}  // namespace stk
