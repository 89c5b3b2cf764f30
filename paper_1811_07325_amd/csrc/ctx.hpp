// Library context: device, workspace, graph cache, autotuner state and the
// serving engine.  Internal to the library (the ABI sees an opaque pointer).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/stark.h"
#include "plan.hpp"

namespace stk {

class Engine;  // serving (serving.cpp)

// Thread-local error message of the ABI.
void set_error(const char* fmt, ...);
const char* get_error();

#define STK_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::stk::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return STARK_EDEVICE;                                                         \
        }                                                                                 \
    } while (0)

struct GraphKey {
    int64_t n;
    int depth, precision, tile;
    const void *A, *B, *C, *ws;
    hipStream_t stream;
    bool operator<(const GraphKey& o) const {
        return std::tie(n, depth, precision, tile, A, B, C, ws, stream) <
               std::tie(o.n, o.depth, o.precision, o.tile, o.A, o.B, o.C, o.ws, o.stream);
    }
    bool operator==(const GraphKey& o) const { return !(*this < o) && !(o < *this); }
};

struct TuneEntry {
    int depth;
    int tile;   // leaf-GEMM tile class (0: the planner's rule)
    double ms;
    double err;
    bool in_tol;  // err within the tolerance the point was measured against
};

}  // namespace stk

struct stark_ctx {
    int device = 0;
    int num_cu = 256;
    std::mutex mu;                 // guards everything below except the engine
    // workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    // rectangular products: packed operand blocks and block products (grown on demand)
    void* rect = nullptr;
    size_t rect_bytes = 0;
    // graph cache (keyed by plan + pointers + stream), LRU
    std::map<stk::GraphKey, hipGraphExec_t> graphs;
    std::list<stk::GraphKey> graph_lru;
    std::map<stk::GraphKey, int> graph_seen;
    hipStream_t side_stream = nullptr;   // used when the caller passes the null stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // end of the last call that used the workspace or the rectangular blocks
    hipEvent_t ws_done = nullptr;
    bool ws_recorded = false;
    // autotuner
    std::map<std::pair<int64_t, int>, stk::TuneEntry> tune;
    std::string tune_path;
    double tune_tol = 1e-5;
    // serving
    size_t hbm_budget = 0;
    int max_slots = 4;
    std::unique_ptr<stk::Engine> engine;
};

namespace stk {

// Enqueue one multiply (all phases in `mask`) eagerly on `st`.
// persistent = false launches the leaf GEMM with one workgroup per tile
// instead of one resident wave of workgroups (served requests: the GPU is
// shared with other streams).  Results are the same either way.
stark_status run_plan(stark_ctx* ctx, const Plan& p, const ProbDesc& d, unsigned mask, hipStream_t st,
                      bool persistent = true);
// The same without a context: num_cu compute units on the current device.
stark_status run_plan_cu(int num_cu, const Plan& p, const ProbDesc& d, unsigned mask, hipStream_t st,
                         bool persistent = true);

// Enqueue one multiply through the graph cache (eager on first sight).
stark_status run_cached(stark_ctx* ctx, const Plan& p, const float* A, const float* B, float* C,
                        void* ws, hipStream_t st);

// Make sure the context workspace holds `bytes` (caller lock held).
stark_status ensure_workspace(stark_ctx* ctx, size_t bytes);

// The workspace and the rectangular blocks hold one call's intermediates at a
// time.  ws_wait orders the work a call is about to enqueue on `st` after the
// previous such call's work (whatever stream that used); ws_done records the
// end of this call's work on `st`.  Caller lock held.
stark_status ws_wait(stark_ctx* ctx, hipStream_t st);
stark_status ws_done(stark_ctx* ctx, hipStream_t st, stark_status rc);

// User operands of one multiply: non-NULL, n > 0, 16-byte aligned, C
// overlapping neither A nor B.  Sets the error message.
stark_status check_operands(const float* A, const float* B, const float* C, int64_t n);

// Autotuner (tuner.cpp): depth and leaf-GEMM tile class for (n, precision),
// measuring on the caller's operands if the size is new.  Caller lock held.
stark_status tuned_depth(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, int precision,
                         hipStream_t st, int* depth, int* tile);
void tuner_load(stark_ctx* ctx);
// record_fallback: when no point is within tol, record the most accurate
// one (flagged) instead of nothing.
stark_status tune_range(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, int precision,
                        int dmin, int dmax, double tol, bool record_fallback, hipStream_t st,
                        std::vector<TuneEntry>& results, int* depth, int* tile);

// Leaf-GEMM grid for `tiles` tiles: resident blocks per CU x CUs, capped.
int gemm_grid(stark_ctx* ctx, int planes, int tile, int64_t tiles);
int gemm_grid_cu(int num_cu, int planes, int tile, int64_t tiles);

// Batched (batched.cpp).  plan_batched: the plans of stark_gemm_batched
// (ctx may be null: no autotuner records; lock held otherwise); "" or an
// error naming the problem.
std::string plan_batched(stark_ctx* ctx, int count, const int64_t* n, int depth, int precision,
                         std::vector<Plan>& plans);
stark_status gemm_batched(stark_ctx* ctx, int count, const float* const* A, const float* const* B,
                          float* const* C, const int64_t* n, int depth, int precision, hipStream_t st);
void batched_release(stark_ctx* ctx);

}  // namespace stk
