// Batched multiplies: many independent problems of uneven sizes share every
// launch.  Level l of the divide covers the level-l nodes of every problem
// deep enough to have them; one grouped persistent launch per leaf-tile class
// multiplies every leaf of every problem (the batch planner puts them all on
// one class unless its model finds mixed classes faster); the combine
// levels mirror the divide.  The problem table and the per-launch block
// prefixes live in a small device buffer owned by the cache entry, and the
// launch sequence is captured into a hipGraph the second time the same batch
// (pointers, sizes, depth, precision, stream) is seen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"

namespace stk {

namespace {

enum LaunchKind { kPad, kDivide, kAbsmax, kScaleExp, kSplit, kGemm, kCombine, kCombine2, kPeel };

struct BatchLaunch {
    LaunchKind kind;
    int level;      // divide / combine level; peel: the largest residue of the launch
    int tile;       // gemm tile class
    bool fused;     // gemm: binary32 leaves formed in the GEMM (plans with fuse);
                    // level-0 combine: some problem peels (fix-up variant)
    int64_t total;  // blocks (or tiles for the gemm)
    size_t prefix;  // index of the prefix array in the device buffer (in int64 units)
};

struct BatchEntry {
    void* dev = nullptr;           // ProbDesc[count] followed by prefix arrays
    int count = 0;
    int planes = 0;
    bool fp16 = false;
    int variant = 0;
    std::vector<BatchLaunch> launches;
    hipGraphExec_t exec = nullptr;
    int uses = 0;
    uint64_t last_use = 0;
};

struct BatchKey {
    std::vector<const void*> ptrs;
    std::vector<int64_t> sizes;
    std::vector<int> plans;   // depth and tile class of every problem
    int precision;
    const void* ws;
    hipStream_t stream;
    bool operator<(const BatchKey& o) const {
        return std::tie(ptrs, sizes, plans, precision, ws, stream) <
               std::tie(o.ptrs, o.sizes, o.plans, o.precision, o.ws, o.stream);
    }
};

std::mutex g_batch_mu;
std::map<std::pair<stark_ctx*, BatchKey>, BatchEntry> g_batches;
uint64_t g_batch_clock = 0;
constexpr size_t kMaxBatches = 64;   // cached batches per context (least recently used evicted)

void release_entry(BatchEntry& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.dev) (void)hipFree(e.dev);
    e.exec = nullptr;
    e.dev = nullptr;
}

// Make room for one more entry of `ctx`.  The victim's last launch belongs to
// an earlier call, which has finished once the last call's end event has
// (every call waits for the one before it).  Lock held.
stark_status evict_for(stark_ctx* ctx) {
    auto victim = g_batches.end();
    size_t mine = 0;
    for (auto it = g_batches.begin(); it != g_batches.end(); ++it) {
        if (it->first.first != ctx) continue;
        ++mine;
        if (victim == g_batches.end() || it->second.last_use < victim->second.last_use) victim = it;
    }
    if (mine < kMaxBatches) return STARK_OK;
    if (ctx->ws_recorded) STK_HIP(hipEventSynchronize(ctx->ws_done));
    release_entry(victim->second);
    g_batches.erase(victim);
    return STARK_OK;
}

stark_status enqueue(stark_ctx* ctx, const BatchEntry& e, hipStream_t st) {
    const ProbDesc* table = static_cast<const ProbDesc*>(e.dev);
    const int64_t* pre = reinterpret_cast<const int64_t*>(static_cast<const char*>(e.dev) +
                                                          sizeof(ProbDesc) * e.count);
    for (const BatchLaunch& l : e.launches) {
        const TableProb src{table, pre + l.prefix, e.count};
        switch (l.kind) {
            case kPad: STK_HIP(launch_pad(src, l.total, st)); break;
            case kDivide: STK_HIP(launch_divide(src, l.level, e.variant, l.total, st)); break;
            case kAbsmax: STK_HIP(launch_absmax(src, l.total, st)); break;
            case kScaleExp: STK_HIP(launch_scale_exp(src, l.total, st)); break;
            case kSplit: STK_HIP(launch_split(src, e.planes, e.variant, l.total, st)); break;
            case kGemm:
                STK_HIP(launch_gemm(src, e.planes, l.tile, e.fp16, l.total,
                                    gemm_grid(ctx, e.planes, l.tile, l.total), st, l.fused));
                break;
            case kCombine: STK_HIP(launch_combine(src, l.level, e.variant, l.total, st, l.fused)); break;
            case kCombine2: STK_HIP(launch_combine2(src, l.level, e.variant, l.total, st, l.fused)); break;
            case kPeel: STK_HIP(launch_peel(src, l.level, l.total, st)); break;
        }
    }
    return STARK_OK;
}

}  // namespace

std::string plan_batched(stark_ctx* ctx, int count, const int64_t* n, int depth, int precision,
                         std::vector<Plan>& plans) {
    plans.assign(count, Plan());
    std::vector<char> fixed(count, 0);
    for (int i = 0; i < count; ++i) {
        int d = 0, tile = 0;
        if (depth == STARK_DEPTH_AUTO) {   // the problem's autotuner record, else planned with the batch
            if (!ctx) continue;
            auto it = ctx->tune.find({n[i], precision});
            if (it == ctx->tune.end()) continue;
            d = it->second.depth;
            tile = it->second.tile;
        } else {
            d = std::min(depth, max_depth_for(n[i]));
        }
        const std::string why = make_plan(n[i], d, precision, plans[i], tile);
        if (!why.empty()) return "problem " + std::to_string(i) + ": " + why;
        fixed[i] = 1;
    }
    if (depth == STARK_DEPTH_AUTO) return plan_batch(count, n, precision, plans, fixed);
    return "";
}

stark_status gemm_batched(stark_ctx* ctx, int count, const float* const* A, const float* const* B, float* const* C,
                          const int64_t* n, int depth, int precision, hipStream_t st) {
    std::vector<Plan> plans;
    const std::string why = plan_batched(ctx, count, n, depth, precision, plans);
    if (!why.empty()) { set_error("%s", why.c_str()); return STARK_EINVAL; }
    std::vector<size_t> off(count);
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        off[i] = total;
        total += (plans[i].bytes + 255) / 256 * 256;
    }
    stark_status rc = ensure_workspace(ctx, total);
    if (rc != STARK_OK) return rc;

    BatchKey key;
    for (const Plan& p : plans) {
        key.plans.push_back(p.depth);
        key.plans.push_back(p.tile);
        key.plans.push_back(p.fuse ? 1 : 0);
    }
    key.precision = precision;
    key.ws = ctx->ws;
    key.stream = st ? st : ctx->side_stream;
    for (int i = 0; i < count; ++i) {
        key.ptrs.push_back(A[i]);
        key.ptrs.push_back(B[i]);
        key.ptrs.push_back(C[i]);
        key.sizes.push_back(n[i]);
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batches.find({ctx, key});
    if (it == g_batches.end()) {
        rc = evict_for(ctx);
        if (rc != STARK_OK) return rc;
        BatchEntry e;
        e.count = count;
        e.planes = plans[0].planes;
        e.fp16 = plans[0].scale >= 0;
        e.variant = plans[0].variant;
        // The table lists the problems with the longest leaves (the longest
        // tiles) first: a grouped launch takes its tiles in table order, so
        // the short ones fill the last waves.
        std::vector<int> ord(count);
        for (int i = 0; i < count; ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return plans[a].leaf > plans[b].leaf; });
        std::vector<ProbDesc> descs(count);
        std::vector<Plan> table_plans(count);
        for (int j = 0; j < count; ++j) {
            const int i = ord[j];
            table_plans[j] = plans[i];
            descs[j] = make_desc(plans[i], A[i], B[i], C[i], static_cast<char*>(ctx->ws) + off[i]);
        }
        plans.swap(table_plans);   // from here on, in table order
        std::vector<int64_t> pre;
        auto add_launch = [&](LaunchKind kind, int level, int tile, auto blocks_of, bool fused = false) {
            BatchLaunch l{kind, level, tile, fused, 0, pre.size()};
            int64_t acc = 0;
            for (int i = 0; i < count; ++i) {
                pre.push_back(acc);
                acc += blocks_of(i);
            }
            pre.push_back(acc);
            l.total = acc;
            if (acc > 0) e.launches.push_back(l);
        };
        int max_fp32 = 0, max_depth = 0;
        for (const Plan& p : plans) {
            max_fp32 = std::max(max_fp32, p.fp32_levels);
            max_depth = std::max(max_depth, p.depth);
        }
        add_launch(kPad, 0, 0, [&](int i) { return plans[i].pad_a >= 0 ? blocks_pad(descs[i]) : 0; });
        for (int l = 0; l < max_fp32; ++l)
            add_launch(kDivide, l, 0, [&](int i) {
                return plans[i].fp32_levels > l && plans[i].div_slots[l] > 0 ? blocks_divide(descs[i], l) : 0;
            });
        if (e.fp16) {
            add_launch(kAbsmax, 0, 0, [&](int) { return (int64_t)kScaleParts; });
            add_launch(kScaleExp, 0, 0, [&](int) { return (int64_t)1; });
        }
        if (e.planes > 0) add_launch(kSplit, 0, 0, [&](int i) { return blocks_split(descs[i]); });
        // one launch per tile class (the 256-wide binary32 class: one for the
        // problems whose leaf operands the GEMM forms, one for the others)
        for (int tile : {256, 128, 64})
            for (bool fused : {true, false})
                add_launch(kGemm, 0, tile, [&](int i) {
                    const Plan& p = plans[i];
                    return p.tile == tile && p.fuse == fused
                               ? pow7(p.depth) * gemm_tiles_per_leaf(p.planes, tile, p.leaf) : (int64_t)0;
                }, fused);
        int max_peel = 0;
        for (const Plan& p : plans) max_peel = std::max(max_peel, p.peel);
        // per problem: the two deepest levels in one pass, then one level at a time
        for (int l = max_depth - 1; l >= 0; --l) {
            add_launch(kCombine2, l, 0, [&](int i) {
                return plans[i].depth >= 2 && plans[i].depth - 2 == l ? blocks_combine2(descs[i], l) : 0;
            }, l == 0 && max_peel > 0);
            add_launch(kCombine, l, 0, [&](int i) {
                const int d = plans[i].depth;
                return (d == 1 && l == 0) || l <= d - 3 ? blocks_combine(descs[i], l) : 0;
            }, l == 0 && max_peel > 0);
        }
        // border rows and columns of the peeled problems
        if (max_peel > 0) add_launch(kPeel, max_peel, 0, [&](int i) { return blocks_peel(descs[i]); });
        const size_t bytes = sizeof(ProbDesc) * count + sizeof(int64_t) * pre.size();
        STK_HIP(hipMalloc(&e.dev, bytes));
        std::vector<char> host(bytes);
        std::memcpy(host.data(), descs.data(), sizeof(ProbDesc) * count);
        std::memcpy(host.data() + sizeof(ProbDesc) * count, pre.data(), sizeof(int64_t) * pre.size());
        STK_HIP(hipMemcpy(e.dev, host.data(), bytes, hipMemcpyHostToDevice));
        it = g_batches.emplace(std::make_pair(ctx, key), std::move(e)).first;
    }
    BatchEntry& e = it->second;
    hipStream_t gs = key.stream;
    e.uses++;
    e.last_use = ++g_batch_clock;
    if (e.uses == 1) return enqueue(ctx, e, st);
    if (!e.exec) {
        hipGraph_t g = nullptr;
        STK_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        const stark_status rs = enqueue(ctx, e, gs);
        const hipError_t ec = hipStreamEndCapture(gs, &g);
        if (rs != STARK_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rs;
        }
        STK_HIP(ec);
        const hipError_t ei = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        STK_HIP(ei);
    }
    if (!st) {
        STK_HIP(hipEventRecord(ctx->ev_in, nullptr));
        STK_HIP(hipStreamWaitEvent(gs, ctx->ev_in, 0));
        STK_HIP(hipGraphLaunch(e.exec, gs));
        STK_HIP(hipEventRecord(ctx->ev_out, gs));
        STK_HIP(hipStreamWaitEvent(nullptr, ctx->ev_out, 0));
    } else {
        STK_HIP(hipGraphLaunch(e.exec, gs));
    }
    return STARK_OK;
}

// Release the batch entries of a context (called from stark_destroy after the
// device is idle).
void batched_release(stark_ctx* ctx) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto it = g_batches.begin(); it != g_batches.end();) {
        if (it->first.first == ctx) {
            release_entry(it->second);
            it = g_batches.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace stk
