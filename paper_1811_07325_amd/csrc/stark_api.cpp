// C ABI of the Strassen hot path (include/stark.h) and the launch sequence of
// one multiply.
//
// Launch sequence (Algorithm 2 unrolled level by level; every node of a level
// runs in the same launch, as the paper runs each recursion level in
// parallel, Fig. 2 and Section III-C):
//   [pad]            depth-0 binary32 with padding only
//   divide l = 0..   binary32 operand sums (level 0 zero-pads on the fly)
//   [split]          bf16 paths: last level, operands split into bf16 planes
//   leaf GEMM        one grouped persistent launch over all 7^k leaves
//   combine l = k-1..0  (level 0 writes C, cropping the padding; the two
//                    deepest levels run as one pass)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "ctx.hpp"
#include "engine.hpp"
#include "launch.hpp"

namespace stk {

static thread_local std::string t_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
}
const char* get_error() { return t_err.c_str(); }

int gemm_grid(stark_ctx* ctx, int planes, int tile, int64_t tiles) {
    return gemm_grid_cu(ctx->num_cu, planes, tile, tiles);
}

int gemm_grid_cu(int num_cu, int planes, int tile, int64_t tiles) {
    // resident blocks per CU of every (planes, tile) variant, queried once
    // (thread-safe static initialisation; the serving thread calls this too)
    struct Occ {
        int v[3][3];
        Occ() {
            const int pl[3] = {0, 2, 3}, tl[3] = {128, 64, 256};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v[a][b] = gemm_blocks_per_cu(pl[a], tl[b]);
        }
    };
    static const Occ occ;
    const int pi = planes == 0 ? 0 : planes == 2 ? 1 : 2;
    const int ti = tile == 128 ? 0 : tile == 64 ? 1 : 2;
    const int64_t g = (int64_t)num_cu * occ.v[pi][ti];
    return (int)std::min<int64_t>(g, tiles);
}

stark_status run_plan(stark_ctx* ctx, const Plan& p, const ProbDesc& d, unsigned mask, hipStream_t st,
                      bool persistent) {
    return run_plan_cu(ctx->num_cu, p, d, mask, st, persistent);
}

stark_status run_plan_cu(int num_cu, const Plan& p, const ProbDesc& d, unsigned mask, hipStream_t st,
                         bool persistent) {
    const OneProb src{d};
    if (mask & STARK_PHASE_DIVIDE) {
        if (p.pad_a >= 0) STK_HIP(launch_pad(src, blocks_pad(d), st));
        for (int l = 0; l < p.fp32_levels; ++l)
            if (p.div_slots[l] > 0) STK_HIP(launch_divide(src, l, p.variant, blocks_divide(d, l), st));
        if (p.scale >= 0) {
            STK_HIP(launch_absmax(src, kScaleParts, st));
            STK_HIP(launch_scale_exp(src, 1, st));
        }
        if (p.planes > 0) STK_HIP(launch_split(src, p.planes, p.variant, blocks_split(d), st));
    }
    if (mask & STARK_PHASE_LEAF) {
        const int64_t tiles = pow7(p.depth) * gemm_tiles_per_leaf(p.planes, p.tile, p.leaf);
        // persistent: one resident wave of workgroups loops over the tiles;
        // otherwise one workgroup per tile (capped), so that workgroups
        // retire throughout the launch and kernels of other streams get CUs
        const int grid = persistent ? gemm_grid_cu(num_cu, p.planes, p.tile, tiles)
                                    : (int)std::min<int64_t>(tiles, int64_t(1) << 30);
        STK_HIP(launch_gemm(src, p.planes, p.tile, d.fp16 != 0, tiles, grid, st, p.fuse));
    }
    if (mask & STARK_PHASE_COMBINE) {
        int l = p.depth - 1;
        if (p.depth >= 2) {   // the two deepest levels in one pass
            STK_HIP(launch_combine2(src, p.depth - 2, p.variant, blocks_combine2(d, p.depth - 2), st,
                                    p.depth == 2 && p.peel > 0));
            l = p.depth - 3;
        }
        for (; l >= 0; --l)
            STK_HIP(launch_combine(src, l, p.variant, blocks_combine(d, l), st, l == 0 && p.peel > 0));
        // border rows and columns of a peeled plan (the core's fix-up is in
        // the level-0 combine)
        if (p.peel) STK_HIP(launch_peel(src, p.peel, blocks_peel(d), st));
    }
    return STARK_OK;
}

stark_status ensure_workspace(stark_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return STARK_OK;
    if (!ctx->ws_owned && ctx->ws) {
        set_error("workspace of %zu bytes is smaller than the %zu bytes this multiply needs", ctx->ws_bytes, bytes);
        return STARK_ENOMEM;
    }
    // Library-owned: grow.  In-flight work may still use the old buffer.
    STK_HIP(hipSetDevice(ctx->device));
    if (ctx->ws) {
        STK_HIP(hipDeviceSynchronize());
        for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
        ctx->graphs.clear();
        ctx->graph_lru.clear();
        ctx->graph_seen.clear();
        STK_HIP(hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cannot allocate a %zu-byte workspace", bytes);
        return STARK_ENOMEM;
    }
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    ctx->ws_owned = true;
    return STARK_OK;
}

stark_status ws_wait(stark_ctx* ctx, hipStream_t st) {
    if (ctx->ws_recorded) STK_HIP(hipStreamWaitEvent(st, ctx->ws_done, 0));
    return STARK_OK;
}

stark_status ws_done(stark_ctx* ctx, hipStream_t st, stark_status rc) {
    // recorded after a failure too: part of the call's work may be enqueued
    const hipError_t e = hipEventRecord(ctx->ws_done, st);
    if (e == hipSuccess) ctx->ws_recorded = true;
    if (rc != STARK_OK) return rc;
    STK_HIP(e);
    return STARK_OK;
}

static constexpr size_t kMaxGraphs = 64;

stark_status run_cached(stark_ctx* ctx, const Plan& p, const float* A, const float* B, float* C, void* ws,
                        hipStream_t st) {
    const ProbDesc d = make_desc(p, A, B, C, ws);
    hipStream_t gs = st ? st : ctx->side_stream;   // capture needs a non-null stream
    const GraphKey key{p.n, p.depth, p.precision, p.tile, A, B, C, ws, gs};
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        int& seen = ctx->graph_seen[key];
        if (seen == 0 || ctx->graph_seen.size() > 4096) {
            // first sight of this (plan, pointers, stream): launch eagerly
            seen = 1;
            return run_plan(ctx, p, d, STARK_PHASE_ALL, st);
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        STK_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        const stark_status rs = run_plan(ctx, p, d, STARK_PHASE_ALL, gs);
        const hipError_t ec = hipStreamEndCapture(gs, &g);
        if (rs != STARK_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rs;
        }
        STK_HIP(ec);
        const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        STK_HIP(ei);
        if (ctx->graphs.size() >= kMaxGraphs) {
            // the evicted graph's last launch belongs to an earlier call, which
            // has finished once the last call's end event has (every call
            // waits for the one before it); its stream may be gone by now
            const GraphKey old = ctx->graph_lru.back();
            ctx->graph_lru.pop_back();
            if (ctx->ws_recorded) STK_HIP(hipEventSynchronize(ctx->ws_done));
            (void)hipGraphExecDestroy(ctx->graphs[old]);
            ctx->graphs.erase(old);
        }
        it = ctx->graphs.emplace(key, ge).first;
        ctx->graph_lru.push_front(key);
    } else {
        ctx->graph_lru.remove(key);
        ctx->graph_lru.push_front(key);
    }
    if (!st) {
        // null stream: order the side stream after it, and it after the side stream
        STK_HIP(hipEventRecord(ctx->ev_in, nullptr));
        STK_HIP(hipStreamWaitEvent(gs, ctx->ev_in, 0));
        STK_HIP(hipGraphLaunch(it->second, gs));
        STK_HIP(hipEventRecord(ctx->ev_out, gs));
        STK_HIP(hipStreamWaitEvent(nullptr, ctx->ev_out, 0));
    } else {
        STK_HIP(hipGraphLaunch(it->second, gs));
    }
    return STARK_OK;
}

static bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bn && pb < pa + an;
}

stark_status check_operands(const float* A, const float* B, const float* C, int64_t n) {
    if (!A || !B || !C) { set_error("A, B and C must be non-NULL device pointers"); return STARK_EINVAL; }
    if (n <= 0) { set_error("n must be positive"); return STARK_EINVAL; }
    if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) & 15) {
        set_error("A, B and C must be 16-byte aligned");
        return STARK_EINVAL;
    }
    const size_t bytes = (size_t)n * (size_t)n * sizeof(float);
    if (overlaps(C, bytes, A, bytes) || overlaps(C, bytes, B, bytes)) {
        set_error("C overlaps A or B");
        return STARK_EINVAL;
    }
    return STARK_OK;
}
}  // namespace stk

using namespace stk;

extern "C" {

const char* stark_last_error(void) { return get_error(); }

int stark_max_depth(int64_t n) { return n > 0 ? max_depth_for(n) : 0; }

int stark_model_depth(int64_t n, stark_precision prec) {
    if (n <= 0 || n > ((int64_t)1 << 20) || planes_for((int)prec) < 0) return -1;
    return model_depth(n, (int)prec);
}

stark_status stark_workspace_size(int64_t n, int depth, stark_precision prec, size_t* bytes) {
    if (!bytes) { set_error("bytes is NULL"); return STARK_EINVAL; }
    Plan p;
    const std::string why = make_plan(n, depth, (int)prec, p);
    if (!why.empty()) { set_error("%s", why.c_str()); return STARK_EINVAL; }
    *bytes = p.bytes;
    return STARK_OK;
}

static void describe_plan(const Plan& p, stark_plan_desc* out) {
    std::memset(out, 0, sizeof *out);
    out->n = p.n;
    out->n_pad = p.np;
    out->leaf = p.leaf;
    out->depth = p.depth;
    out->precision = p.precision;
    out->planes = p.planes;
    for (int l = 0; l < STARK_MAX_DEPTH; ++l) {
        out->div_a[l] = l < STK_MAXD ? p.div_a[l] : -1;
        out->div_b[l] = l < STK_MAXD ? p.div_b[l] : -1;
        out->div_slots[l] = l < STK_MAXD ? p.div_slots[l] : 0;
        out->comb[l] = l < STK_MAXD ? p.comb[l] : -1;
    }
    out->leaf_a = p.leaf_a;
    out->leaf_b = p.leaf_b;
    out->leaf_m = p.leaf_m;
    out->pad_a = p.pad_a;
    out->pad_b = p.pad_b;
    out->bytes = p.bytes;
    out->gemm_tile = p.tile;
    out->scale = p.scale;
    const Work w = plan_work(p);
    out->divide_bytes = w.divide_bytes + w.pad_bytes;
    out->split_bytes = w.split_bytes;
    out->combine_bytes = w.combine_bytes;
    out->leaf_flops = w.leaf_flops;
    out->mfma_flops = w.mfma_flops;
    out->variant = p.variant;
    out->fused = p.fuse ? 1 : 0;
    out->peel = p.peel;
    out->peel_flops = w.peel_flops;
}

stark_status stark_plan_info(int64_t n, int depth, stark_precision prec, stark_plan_desc* out) {
    if (!out) { set_error("out is NULL"); return STARK_EINVAL; }
    Plan p;
    const std::string why = make_plan(n, depth, (int)prec, p);
    if (!why.empty()) { set_error("%s", why.c_str()); return STARK_EINVAL; }
    describe_plan(p, out);
    return STARK_OK;
}

stark_status stark_plan_batched(stark_ctx* ctx, int count, const int64_t* n, int depth, stark_precision prec,
                                stark_plan_desc* out) {
    if (count <= 0 || !n || !out) { set_error("bad batch arguments"); return STARK_EINVAL; }
    if (planes_for((int)prec) < 0) { set_error("unknown precision %d", (int)prec); return STARK_EUNSUPPORTED; }
    if (depth < 0 && depth != STARK_DEPTH_AUTO) { set_error("depth must be >= 0 or STARK_DEPTH_AUTO"); return STARK_EINVAL; }
    std::vector<Plan> plans;
    std::string why;
    if (ctx) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        why = plan_batched(ctx, count, n, depth, (int)prec, plans);
    } else {
        why = plan_batched(nullptr, count, n, depth, (int)prec, plans);
    }
    if (!why.empty()) { set_error("%s", why.c_str()); return STARK_EINVAL; }
    for (int i = 0; i < count; ++i) describe_plan(plans[i], &out[i]);
    return STARK_OK;
}

stark_status stark_create(stark_ctx** out, const stark_config* cfg) {
    if (!out) { set_error("out is NULL"); return STARK_EINVAL; }
    *out = nullptr;
    stark_config c{};
    if (cfg) c = *cfg;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device");
        return STARK_EDEVICE;
    }
    if (c.device < 0 || c.device >= ndev) { set_error("device %d out of range", c.device); return STARK_EINVAL; }
    if (c.workspace && c.workspace_bytes == 0) { set_error("workspace given with zero size"); return STARK_EINVAL; }
    std::unique_ptr<stark_ctx> ctx(new stark_ctx());
    ctx->device = c.device;
    STK_HIP(hipSetDevice(c.device));
    STK_HIP(hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, c.device));
    if (c.workspace) {
        ctx->ws = c.workspace;
        ctx->ws_bytes = c.workspace_bytes;
        ctx->ws_owned = false;
    }
    STK_HIP(hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking));
    STK_HIP(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    STK_HIP(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    STK_HIP(hipEventCreateWithFlags(&ctx->ws_done, hipEventDisableTiming));
    size_t free_b = 0, total_b = 0;
    STK_HIP(hipMemGetInfo(&free_b, &total_b));
    ctx->hbm_budget = c.hbm_budget_bytes ? c.hbm_budget_bytes : free_b / 4 * 3;
    ctx->max_slots = c.max_slots > 0 ? c.max_slots : 4;
    if (c.tuner_cache) ctx->tune_path = c.tuner_cache;
    if (const char* tol = std::getenv("STARK_TUNE_TOL")) ctx->tune_tol = std::atof(tol);
    tuner_load(ctx.get());
    // resident-block counts of every leaf-GEMM variant, cached before any
    // second thread (the serving engine) can launch
    for (int pl : {0, 2, 3})
        for (int tile : {256, 128, 64})
            if (pl > 0 || tile != 256) (void)gemm_grid(ctx.get(), pl, tile, 1);
    *out = ctx.release();
    return STARK_OK;
}

stark_status stark_destroy(stark_ctx* ctx) {
    if (!ctx) return STARK_OK;
    stark_status rc = STARK_OK;
    ctx->engine.reset();   // drains and joins the serving thread
    if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        set_error("device synchronisation failed at destroy");
        rc = STARK_EDEVICE;
    }
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    batched_release(ctx);
    if (ctx->ws_owned && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->rect) (void)hipFree(ctx->rect);
    if (ctx->side_stream) (void)hipStreamDestroy(ctx->side_stream);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ws_done) (void)hipEventDestroy(ctx->ws_done);
    delete ctx;
    return rc;
}


stark_status stark_gemm(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, int depth,
                        stark_precision prec, void* stream) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    stark_status rc = check_operands(A, B, C, n);
    if (rc != STARK_OK) return rc;
    if (planes_for((int)prec) < 0) { set_error("unknown precision %d", (int)prec); return STARK_EUNSUPPORTED; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(ctx->mu);
    STK_HIP(hipSetDevice(ctx->device));
    int tile = 0;   // the planner's rule unless the autotuner chose one
    if (depth == STARK_DEPTH_AUTO) {
        if ((rc = ws_wait(ctx, st)) != STARK_OK) return rc;
        rc = ws_done(ctx, st, tuned_depth(ctx, A, B, C, n, (int)prec, st, &depth, &tile));
        if (rc != STARK_OK) return rc;
    }
    Plan p;
    const std::string why = make_plan(n, depth, (int)prec, p, tile);
    if (!why.empty()) { set_error("%s (n=%lld depth=%d)", why.c_str(), (long long)n, depth); return STARK_EINVAL; }
    rc = ensure_workspace(ctx, p.bytes);
    if (rc != STARK_OK) return rc;
    if ((rc = ws_wait(ctx, st)) != STARK_OK) return rc;
    return ws_done(ctx, st, run_cached(ctx, p, A, B, C, ctx->ws, st));
}

stark_status stark_gemm_phases(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, int depth,
                               stark_precision prec, unsigned mask, void* stream) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    stark_status rc = check_operands(A, B, C, n);
    if (rc != STARK_OK) return rc;
    if (mask == 0 || (mask & ~STARK_PHASE_ALL)) { set_error("bad phase mask %u", mask); return STARK_EINVAL; }
    Plan p;
    const std::string why = make_plan(n, depth, (int)prec, p);
    if (!why.empty()) { set_error("%s", why.c_str()); return STARK_EINVAL; }
    std::lock_guard<std::mutex> lk(ctx->mu);
    STK_HIP(hipSetDevice(ctx->device));
    rc = ensure_workspace(ctx, p.bytes);
    if (rc != STARK_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = ws_wait(ctx, st)) != STARK_OK) return rc;
    return ws_done(ctx, st, run_plan(ctx, p, make_desc(p, A, B, C, ctx->ws), mask, st));
}

stark_status stark_tune(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, stark_precision prec,
                        int min_depth, int max_depth, double tol, stark_tune_point* points, int cap, int* count,
                        void* stream) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    stark_status rc = check_operands(A, B, C, n);
    if (rc != STARK_OK) return rc;
    if (planes_for((int)prec) < 0) { set_error("unknown precision %d", (int)prec); return STARK_EUNSUPPORTED; }
    if (min_depth < 0 || max_depth < min_depth) { set_error("bad depth range"); return STARK_EINVAL; }
    std::lock_guard<std::mutex> lk(ctx->mu);
    STK_HIP(hipSetDevice(ctx->device));
    std::vector<TuneEntry> res;
    int depth = 0, tile = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = ws_wait(ctx, st)) != STARK_OK) return rc;
    rc = ws_done(ctx, st,
                 tune_range(ctx, A, B, C, n, (int)prec, min_depth, max_depth, tol, false, st, res, &depth, &tile));
    if (rc != STARK_OK) return rc;
    if (points)
        for (int i = 0; i < cap && i < (int)res.size(); ++i)
            points[i] = stark_tune_point{res[i].depth, res[i].ms, res[i].err, res[i].tile};
    if (count) *count = (int)res.size();
    return STARK_OK;
}

stark_status stark_workspace(stark_ctx* ctx, void** ptr, size_t* bytes) {
    if (!ctx || !ptr || !bytes) { set_error("NULL argument"); return STARK_EINVAL; }
    std::lock_guard<std::mutex> lk(ctx->mu);
    *ptr = ctx->ws;
    *bytes = ctx->ws_bytes;
    return STARK_OK;
}

stark_status stark_gemm_batched(stark_ctx* ctx, int count, const float* const* A, const float* const* B,
                                float* const* C, const int64_t* n, int depth, stark_precision prec, void* stream) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    if (count <= 0 || !A || !B || !C || !n) { set_error("bad batch arguments"); return STARK_EINVAL; }
    for (int i = 0; i < count; ++i) {
        const stark_status rc = check_operands(A[i], B[i], C[i], n[i]);
        if (rc != STARK_OK) return rc;
    }
    if (planes_for((int)prec) < 0) { set_error("unknown precision %d", (int)prec); return STARK_EUNSUPPORTED; }
    if (depth < 0 && depth != STARK_DEPTH_AUTO) { set_error("depth must be >= 0 or STARK_DEPTH_AUTO"); return STARK_EINVAL; }
    std::lock_guard<std::mutex> lk(ctx->mu);
    STK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const stark_status rc = ws_wait(ctx, st);
    if (rc != STARK_OK) return rc;
    return ws_done(ctx, st, gemm_batched(ctx, count, A, B, C, n, depth, (int)prec, st));
}

stark_status stark_matvec_f64(const float* M, const double* x, double* y, int64_t n, void* stream) {
    if (!M || !x || !y || n <= 0) { set_error("bad matvec arguments"); return STARK_EINVAL; }
    STK_HIP(launch_matvec_f64(M, x, y, n, static_cast<hipStream_t>(stream)));
    return STARK_OK;
}

stark_status stark_row_errors(const float* C, int64_t n, const int64_t* rows, int64_t nrows, const double* ref,
                              double* out, void* stream) {
    if (!C || !rows || !ref || !out || n <= 0 || nrows <= 0) { set_error("bad row-error arguments"); return STARK_EINVAL; }
    STK_HIP(launch_row_errors(C, n, rows, nrows, ref, out, static_cast<hipStream_t>(stream)));
    return STARK_OK;
}

stark_status stark_generate_normal(float* X, int64_t n, uint64_t seed, void* stream) {
    if (!X || n <= 0) { set_error("bad generator arguments"); return STARK_EINVAL; }
    if ((uintptr_t)X & 15) { set_error("X must be 16-byte aligned"); return STARK_EINVAL; }
    STK_HIP(launch_generate_normal(X, n * n, seed, static_cast<hipStream_t>(stream)));
    return STARK_OK;
}

}  // extern "C"
