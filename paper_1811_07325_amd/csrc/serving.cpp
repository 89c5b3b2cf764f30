// Serving engine (see engine.hpp) and the stark_submit / stark_poll /
// stark_stats entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "ctx.hpp"
#include "engine.hpp"
#include "launch.hpp"

namespace stk {

double now_us() {
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

SegmentedArena::Result SegmentedArena::alloc(size_t bytes, bool idle, int* seg, size_t* off) {
    for (size_t i = 0; i < segs_.size(); ++i)
        if (segs_[i].arena.alloc(bytes, off)) {
            *seg = (int)i;
            used_ += round(bytes);
            return kOk;
        }
    const size_t need = round(bytes);
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (need <= budget_ - allocated_) {
            const size_t size = std::min(std::max(need, kSegmentBytes), budget_ - allocated_);
            void* p = nullptr;
            if (hipMalloc(&p, size) == hipSuccess) {
                segs_.push_back(Seg{p, Arena(size)});
                allocated_ += size;
                if (!segs_.back().arena.alloc(bytes, off)) return kFail;   // cannot happen: size >= need
                *seg = (int)segs_.size() - 1;
                used_ += need;
                return kOk;
            }
            (void)hipGetLastError();
        }
        // no room in the budget, or the device refused: when idle every
        // segment is empty, so give them back and try once more
        if (!idle || segs_.empty()) break;
        release();
    }
    return idle ? kFail : kWait;
}

void SegmentedArena::release() {
    for (auto& s : segs_) (void)hipFree(s.base);
    segs_.clear();
    allocated_ = 0;
    used_ = 0;
}

int default_serving_depth(int64_t n, int precision) { return model_depth(n, precision); }

size_t request_footprint(const Plan& p, bool gen, bool own_c) {
    const size_t nn = (size_t)p.n * (size_t)p.n * 4;
    size_t b = (p.bytes + 255) / 256 * 256;
    if (gen) b += 2 * ((nn + 255) / 256 * 256);
    if (own_c) b += (nn + 255) / 256 * 256;
    return b;
}

// ----------------------------------------------------------------------------
// Engine
// ----------------------------------------------------------------------------
Engine::Engine(stark_ctx* ctx, size_t budget, int slots, hipError_t* err) : ctx_(ctx), mem_(budget) {
    *err = hipSetDevice(ctx->device);
    if (*err == hipSuccess) *err = hipHostMalloc(reinterpret_cast<void**>(&host_sums_), sizeof(double) * slots);
    if (*err != hipSuccess) return;
    slots_.resize(slots);
    for (auto& s : slots_) {
        if ((*err = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess) return;
        if ((*err = hipEventCreate(&s.ev0)) != hipSuccess) return;
        if ((*err = hipEventCreate(&s.ev1)) != hipSuccess) return;
        if ((*err = hipMalloc(reinterpret_cast<void**>(&s.partials), 257 * sizeof(double))) != hipSuccess) return;
    }
    if (const char* f = std::getenv("STARK_FAULT_INJECT")) fault_tag_ = std::atoll(f);
    if (const char* f = std::getenv("STARK_SERVE_PERSISTENT")) persistent_ = std::atoi(f) != 0;
    if (const char* f = std::getenv("STARK_SERVE_FIFO")) fifo_ = std::atoi(f) != 0;
    if (const char* f = std::getenv("STARK_SERVE_AGING_MS")) aging_ms_ = std::atof(f);
    if (const char* f = std::getenv("STARK_SERVE_LARGE_MS")) large_.threshold = std::atof(f) * 1e-3;
    if (const char* f = std::getenv("STARK_SERVE_LARGE_CAP")) large_.cap = std::max(1, std::atoi(f));

    thread_ = std::thread([this] { loop(); });
}

Engine::~Engine() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (thread_.joinable()) thread_.join();
    (void)hipSetDevice(ctx_->device);
    for (auto& s : slots_) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.ev0) (void)hipEventDestroy(s.ev0);
        if (s.ev1) (void)hipEventDestroy(s.ev1);
        if (s.partials) (void)hipFree(s.partials);
    }
    for (auto& kv : live_) delete kv.second;   // every request is in live_ until polled
    mem_.release();
    if (host_sums_) (void)hipHostFree(host_sums_);
}

stark_status Engine::submit(const stark_request& r, uint64_t* ticket) {
    if (r.n <= 0 || planes_for((int)r.precision) < 0) {
        set_error("bad request (n=%lld precision=%d)", (long long)r.n, (int)r.precision);
        return STARK_EINVAL;
    }
    const bool gen = (r.A == nullptr);
    if (gen != (r.B == nullptr)) { set_error("A and B must both be given or both be NULL"); return STARK_EINVAL; }
    {   // user operands get the alignment and overlap checks of stark_gemm
        const uintptr_t bits = (uintptr_t)r.A | (uintptr_t)r.B | (uintptr_t)r.C;
        if (bits & 15) { set_error("A, B and C must be 16-byte aligned"); return STARK_EINVAL; }
        if (!gen && r.C) {
            const stark_status rc = check_operands(r.A, r.B, r.C, r.n);
            if (rc != STARK_OK) return rc;
        }
    }
    std::unique_ptr<Req> q(new Req());
    q->r = r;
    q->gen = gen;
    q->own_c = (r.C == nullptr);
    int depth = r.depth, tile = 0;
    if (depth == STARK_DEPTH_AUTO) {
        std::lock_guard<std::mutex> lk(ctx_->mu);
        auto it = ctx_->tune.find({r.n, (int)r.precision});
        if (it != ctx_->tune.end()) {
            depth = it->second.depth;
            tile = it->second.tile;
        } else {
            depth = default_serving_depth(r.n, (int)r.precision);
        }
    }
    const int clamped = std::min(std::max(depth, 0), max_depth_for(r.n));
    if (clamped != depth) tile = 0;
    depth = clamped;
    const std::string why = make_plan(r.n, depth, (int)r.precision, q->plan, tile);
    if (!why.empty()) { set_error("%s", why.c_str()); return STARK_EINVAL; }
    q->bytes = request_footprint(q->plan, q->gen, q->own_c);
    q->cost_s = model_seconds(q->plan);
    if (q->bytes > mem_.budget()) {
        set_error("request needs %zu bytes, budget is %zu", q->bytes, mem_.budget());
        return STARK_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (arrivals_.size() + waiting_pub_ >= kMaxQueue) { set_error("queue full"); return STARK_EBUSY; }
    q->ticket = next_ticket_++;
    q->t_submit = now_us();
    *ticket = q->ticket;
    live_[q->ticket] = q.get();
    arrivals_.push_back(q.release());
    cv_.notify_one();
    return STARK_OK;
}

stark_status Engine::poll(uint64_t ticket, stark_result* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(ticket);
    if (it == live_.end()) { set_error("unknown ticket %llu", (unsigned long long)ticket); return STARK_ENOTFOUND; }
    Req* q = it->second;
    if (q->t_done == 0) return STARK_PENDING;
    if (out) {
        out->tag = q->r.tag;
        out->depth = q->plan.depth;
        out->status = q->status;
        out->t_submit_us = q->t_submit;
        out->t_admit_us = q->t_admit;
        out->t_done_us = q->t_done;
        out->gpu_ms = q->gpu_ms;
        out->checksum = q->checksum;
    }
    const stark_status st = q->status;
    live_.erase(it);
    delete q;
    return st;
}

stark_status Engine::stats(stark_stats_t* out) {
    std::lock_guard<std::mutex> lk(mu_);
    out->completed = completed_;
    out->failed = failed_;
    const double span_s = (last_done_ - first_admit_) * 1e-6;
    out->throughput_tflops = (first_admit_ >= 0 && span_s > 0) ? flops_ / span_s * 1e-12 : 0.0;
    std::vector<double> l = lat_ms_;
    std::sort(l.begin(), l.end());
    out->p50_ms = nearest_rank(l, 0.50);
    out->p99_ms = nearest_rank(l, 0.99);
    out->max_inflight_bytes = (double)max_bytes_;
    out->max_concurrent = max_inflight_;
    return STARK_OK;
}

void Engine::reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    lat_ms_.clear();
    lat_next_ = 0;
    completed_ = failed_ = 0;
    flops_ = 0;
    first_admit_ = -1;
    last_done_ = 0;
    max_bytes_ = used_pub_;
    max_inflight_ = inflight_pub_;
}

// The engine thread alone touches waiting_, slots_, mem_ and inflight_, so
// choosing, reserving and launching a request need no lock; mu_ is taken
// only to publish results and statistics (and to take arrivals), so
// stark_submit / stark_poll / stark_stats never wait behind kernel launches.

void Engine::publish_failure(Req* q, stark_status status) {
    std::lock_guard<std::mutex> lk(mu_);
    q->status = status;
    ++failed_;
    inflight_pub_ = inflight_;
    q->t_done = now_us();   // last: poll may retire the request from here on
}

bool Engine::admit(Req* q, int si) {
    const bool big = large_.large(q->cost_s);
    if (!fifo_ && !large_.admits(q->cost_s)) return false;
    size_t off;
    int seg;
    const SegmentedArena::Result got = mem_.alloc(q->bytes, inflight_ == 0, &seg, &off);
    if (got == SegmentedArena::kWait) return false;
    if (got == SegmentedArena::kFail) {   // nothing in flight and the device refused the memory
        publish_failure(q, STARK_ENOMEM);
        return true;
    }
    Slot& s = slots_[si];
    q->seg = seg;
    q->off = off;
    q->slot = si;
    q->t_admit = now_us();
    s.busy = true;
    s.req = q;
    ++inflight_;
    if (big) ++large_.inflight;
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (first_admit_ < 0) first_admit_ = q->t_admit;
        inflight_pub_ = inflight_;
        max_inflight_ = std::max(max_inflight_, inflight_);
        used_pub_ = mem_.used();
        max_bytes_ = std::max(max_bytes_, used_pub_);
    }

    const size_t nn = (size_t)q->r.n * (size_t)q->r.n * 4;
    const size_t nn_al = (nn + 255) / 256 * 256;
    char* base = mem_.base(seg) + off;
    char* ws = base;
    char* cur = base + (q->plan.bytes + 255) / 256 * 256;
    const float* A = q->r.A;
    const float* B = q->r.B;
    float* C = q->r.C;
    if (q->gen) {
        A = reinterpret_cast<float*>(cur); cur += nn_al;
        B = reinterpret_cast<float*>(cur); cur += nn_al;
    }
    if (q->own_c) { C = reinterpret_cast<float*>(cur); cur += nn_al; }

    hipError_t e = hipSuccess;
    stark_status rc = STARK_OK;
    if ((int64_t)q->r.tag == fault_tag_) {
        rc = STARK_EDEVICE;   // injected failure: nothing is launched
    } else {
        e = hipEventRecord(s.ev0, s.stream);
        if (e == hipSuccess && q->gen) e = launch_generate_normal(const_cast<float*>(A), q->r.n * q->r.n, 2 * q->r.seed, s.stream);
        if (e == hipSuccess && q->gen) e = launch_generate_normal(const_cast<float*>(B), q->r.n * q->r.n, 2 * q->r.seed + 1, s.stream);
        if (e == hipSuccess)
            rc = run_plan(ctx_, q->plan, make_desc(q->plan, A, B, C, ws), STARK_PHASE_ALL, s.stream, persistent_);
        if (e == hipSuccess && rc == STARK_OK && q->own_c) {
            e = launch_sum_f64(C, q->r.n * q->r.n, s.partials, s.partials + 256, s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&host_sums_[si], s.partials + 256, sizeof(double), hipMemcpyDeviceToHost, s.stream);
        }
        if (e == hipSuccess && rc == STARK_OK) e = hipEventRecord(s.ev1, s.stream);
    }
    if (e != hipSuccess || rc != STARK_OK) {
        // make sure nothing of this request is still running before its memory is reused
        (void)hipStreamSynchronize(s.stream);
        (void)hipGetLastError();
        mem_.free(q->seg, q->off, q->bytes);
        s.busy = false;
        s.req = nullptr;
        --inflight_;
        if (big) --large_.inflight;
        publish_failure(q, rc != STARK_OK ? rc : STARK_EDEVICE);
    }
    return true;
}

void Engine::finish(int si) {
    Slot& s = slots_[si];
    Req* q = s.req;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, s.ev0, s.ev1);
    const double checksum = q->own_c ? host_sums_[si] : 0.0;
    mem_.free(q->seg, q->off, q->bytes);
    s.busy = false;
    s.req = nullptr;
    --inflight_;
    if (large_.large(q->cost_s)) --large_.inflight;
    std::lock_guard<std::mutex> lk(mu_);
    q->gpu_ms = ms;
    q->checksum = checksum;
    q->status = STARK_OK;
    ++completed_;
    const double t = now_us();
    const double lat = (t - q->t_submit) * 1e-3;
    if (lat_ms_.size() < kLatWindow) lat_ms_.push_back(lat);
    else lat_ms_[lat_next_] = lat;
    lat_next_ = (lat_next_ + 1) % kLatWindow;
    flops_ += 2.0 * (double)q->r.n * (double)q->r.n * (double)q->r.n;
    last_done_ = t;
    inflight_pub_ = inflight_;
    used_pub_ = mem_.used();
    q->t_done = t;   // last: poll may retire the request from here on
}

void Engine::loop() {
    (void)hipSetDevice(ctx_->device);
    while (true) {
        bool stopping;
        {
            std::unique_lock<std::mutex> lk(mu_);
            if (arrivals_.empty() && waiting_.empty() && inflight_ == 0 && !stop_)
                cv_.wait_for(lk, std::chrono::milliseconds(5));
            while (!arrivals_.empty()) {
                waiting_.push_back(arrivals_.front());
                arrivals_.pop_front();
            }
            waiting_pub_ = waiting_.size();   // at most one pass stale: only bounds the queue
            stopping = stop_;
        }
        bool progress = false;
        // completions
        for (int si = 0; si < (int)slots_.size(); ++si) {
            if (!slots_[si].busy) continue;
            const hipError_t e = hipEventQuery(slots_[si].ev1);
            if (e == hipSuccess) {
                finish(si);
                progress = true;
            } else if (e != hipErrorNotReady) {
                Req* q = slots_[si].req;
                mem_.free(q->seg, q->off, q->bytes);
                slots_[si].busy = false;
                slots_[si].req = nullptr;
                --inflight_;
                if (large_.large(q->cost_s)) --large_.inflight;
                (void)hipGetLastError();
                publish_failure(q, STARK_EDEVICE);
                progress = true;
            }
        }
        // admissions: size-aware order (or arrival order), requests that do
        // not fit passed over a bounded number of times (sched.hpp)
        int free_slot = -1;
        auto slot_free = [&] {
            free_slot = -1;
            for (int si = 0; si < (int)slots_.size(); ++si)
                if (!slots_[si].busy) { free_slot = si; break; }
            return free_slot >= 0;
        };
        if (!fifo_ && waiting_.size() > 1)
            order_waiting(waiting_, now_us(), aging_ms_ * 1e3, [](const Req* q) { return q->t_submit; },
                          [](const Req* q) { return q->cost_s; });
        if (admission_pass(waiting_, slot_free, [&](Req* q) { return admit(q, free_slot); }, kMaxBypass,
                           kMaxHeadPasses) > 0)
            progress = true;
        if (stopping && waiting_.empty() && inflight_ == 0) break;
        if (!progress && inflight_ > 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// Guards the creation of a context's engine (first stark_submit) against
// readers of the pointer (stark_poll, stark_stats on other threads).
static std::mutex g_engine_mu;

static Engine* engine_of(stark_ctx* ctx) {
    std::lock_guard<std::mutex> lk(g_engine_mu);
    return ctx->engine.get();
}

static stark_status ensure_engine(stark_ctx* ctx) {
    if (ctx->engine) return STARK_OK;
    hipError_t err = hipSuccess;
    std::unique_ptr<Engine> e(new Engine(ctx, ctx->hbm_budget, ctx->max_slots, &err));
    if (err != hipSuccess) {
        set_error("serving engine start failed: %s", hipGetErrorString(err));
        return STARK_EDEVICE;
    }
    ctx->engine = std::move(e);
    return STARK_OK;
}

}  // namespace stk

using namespace stk;

extern "C" {

stark_status stark_submit(stark_ctx* ctx, const stark_request* r, uint64_t* ticket) {
    if (!ctx || !r || !ticket) { set_error("NULL argument"); return STARK_EINVAL; }
    Engine* e = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_engine_mu);
        const stark_status rc = ensure_engine(ctx);
        if (rc != STARK_OK) return rc;
        e = ctx->engine.get();
    }
    return e->submit(*r, ticket);
}

stark_status stark_poll(stark_ctx* ctx, uint64_t ticket, stark_result* out) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    Engine* e = engine_of(ctx);
    if (!e) { set_error("unknown ticket %llu", (unsigned long long)ticket); return STARK_ENOTFOUND; }
    return e->poll(ticket, out);
}

stark_status stark_stats_reset(stark_ctx* ctx) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    Engine* e = engine_of(ctx);
    if (e) e->reset_stats();
    return STARK_OK;
}

stark_status stark_stats(stark_ctx* ctx, stark_stats_t* out) {
    if (!ctx || !out) { set_error("NULL argument"); return STARK_EINVAL; }
    std::memset(out, 0, sizeof *out);
    Engine* e = engine_of(ctx);
    if (!e) return STARK_OK;
    return e->stats(out);
}

}  // extern "C"
