// Autotuner for the recursion depth (the paper's block-size choice: wall clock
// against partition size is U-shaped, with an optimum per matrix size,
// Section V-C) and the leaf-GEMM tile class.  For a new (n, precision) it
// runs every usable depth, each with the planner's tile class and its valid
// neighbours, on the caller's operands, times three runs after a warm-up with
// HIP events, and measures each result's error with Freivalds' check in
// binary64 on the GPU: e = ||C x - A (B x)|| / ||A (B x)|| for a Gaussian x,
// whose square has the squared relative Frobenius error as its expectation.
// The fastest (depth, tile) whose error is within the tolerance (default
// 1e-5, STARK_TUNE_TOL) is recorded.  An explicit tuning request (stark_tune)
// whose points all miss the tolerance records nothing; the automatic depth
// (STARK_DEPTH_AUTO with no record) must run something, so there the most
// accurate point is recorded, flagged as outside the tolerance.  Records
// persist in a small text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"

namespace stk {

static void tuner_save(stark_ctx* ctx) {
    if (ctx->tune_path.empty()) return;
    FILE* f = std::fopen(ctx->tune_path.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "# n precision depth ms freivalds_error tile within_tolerance\n");
    for (const auto& kv : ctx->tune)
        std::fprintf(f, "%lld %d %d %.6f %.6e %d %d\n", (long long)kv.first.first, kv.first.second, kv.second.depth,
                     kv.second.ms, kv.second.err, kv.second.tile, kv.second.in_tol ? 1 : 0);
    std::fclose(f);
}

void tuner_load(stark_ctx* ctx) {
    if (ctx->tune_path.empty()) return;
    FILE* f = std::fopen(ctx->tune_path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        long long n;
        int prec, depth, tile = 0, in_tol = 1;
        double ms, err;
        const int got = std::sscanf(line, "%lld %d %d %lf %lf %d %d", &n, &prec, &depth, &ms, &err, &tile, &in_tol);
        Plan p;
        if (got >= 5 && n > 0 && depth >= 0 && depth <= max_depth_for(n) &&
            make_plan(n, depth, prec, p, got >= 6 ? tile : 0).empty())
            ctx->tune[{(int64_t)n, prec}] = TuneEntry{depth, got >= 6 ? tile : 0, ms, err, in_tol != 0};
    }
    std::fclose(f);
}

stark_status tune_range(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, int precision,
                        int dmin, int dmax, double tol, bool record_fallback, hipStream_t st,
                        std::vector<TuneEntry>& results, int* depth, int* tile) {
    const int maxd = std::min(dmax, max_depth_for(n));
    if (tol <= 0) tol = ctx->tune_tol;
    // Gaussian probe (fixed seed) and A (B x), binary64.
    std::vector<double> hx(n);
    std::mt19937_64 gen(0x5eed5eedULL);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (auto& v : hx) v = nd(gen);
    double *dx = nullptr, *dbx = nullptr, *dabx = nullptr, *dcx = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    stark_status rc = STARK_OK;
    std::vector<double> habx(n), hcx(n);
    results.clear();
    auto fail = [&](const char* what, hipError_t e) {
        set_error("autotuner: %s: %s", what, hipGetErrorString(e));
        rc = STARK_EDEVICE;
    };
    hipError_t e;
    if ((e = hipMalloc(&dx, n * 8)) != hipSuccess || (e = hipMalloc(&dbx, n * 8)) != hipSuccess ||
        (e = hipMalloc(&dabx, n * 8)) != hipSuccess || (e = hipMalloc(&dcx, n * 8)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        fail("allocation", e);
    }
    if (rc == STARK_OK) {
        if ((e = hipMemcpyAsync(dx, hx.data(), n * 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = launch_matvec_f64(B, dx, dbx, n, st)) != hipSuccess ||
            (e = launch_matvec_f64(A, dbx, dabx, n, st)) != hipSuccess ||
            (e = hipMemcpyAsync(habx.data(), dabx, n * 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            fail("reference product", e);
    }
    double nref = 0.0;
    for (double v : habx) nref += v * v;
    nref = std::sqrt(nref);
    // One (depth, tile) point: warm-up, three timed runs, Freivalds error.
    // False stops the search (an error, or a workspace that cannot grow:
    // deeper plans only need more).
    auto measure = [&](const Plan& p) -> bool {
        if (ensure_workspace(ctx, p.bytes) != STARK_OK) return false;
        const ProbDesc desc = make_desc(p, A, B, C, ctx->ws);
        if ((rc = run_plan(ctx, p, desc, STARK_PHASE_ALL, st)) != STARK_OK) return false;
        std::vector<float> times;
        for (int r = 0; r < 3; ++r) {
            float ms = 0.f;
            if ((e = hipEventRecord(e0, st)) != hipSuccess) { fail("event", e); return false; }
            if ((rc = run_plan(ctx, p, desc, STARK_PHASE_ALL, st)) != STARK_OK) return false;
            if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
                fail("timing", e);
                return false;
            }
            times.push_back(ms);
        }
        if ((e = launch_matvec_f64(C, dx, dcx, n, st)) != hipSuccess ||
            (e = hipMemcpyAsync(hcx.data(), dcx, n * 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            fail("error check", e);
            return false;
        }
        double num = 0.0;
        for (int64_t i = 0; i < n; ++i) num += (hcx[i] - habx[i]) * (hcx[i] - habx[i]);
        std::sort(times.begin(), times.end());
        const double err = nref > 0 ? std::sqrt(num) / nref : 0.0;
        results.push_back(TuneEntry{p.depth, p.tile, times[times.size() / 2], err, err <= tol});
        return true;
    };
    bool more = rc == STARK_OK;
    for (int d = std::max(dmin, 0); d <= maxd && more; ++d) {
        Plan rule;
        if (!make_plan(n, d, precision, rule).empty()) continue;
        int tiles[3];
        const int ntiles = tile_candidates(rule, tiles);
        for (int ti = 0; ti < ntiles && more; ++ti) {
            Plan p;
            if (make_plan(n, d, precision, p, tiles[ti]).empty()) more = measure(p);
        }
    }
    if (dx) (void)hipFree(dx);
    if (dbx) (void)hipFree(dbx);
    if (dabx) (void)hipFree(dabx);
    if (dcx) (void)hipFree(dcx);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != STARK_OK) return rc;
    if (results.empty()) {
        set_error("autotuner: no usable depth for n=%lld", (long long)n);
        return STARK_EINVAL;
    }
    const TuneEntry* best = nullptr;
    for (const auto& r : results)
        if (r.in_tol && (!best || r.ms < best->ms)) best = &r;
    if (!best) {
        for (const auto& r : results)
            if (!best || r.err < best->err) best = &r;
        *depth = best->depth;
        *tile = best->tile;
        if (!record_fallback) return STARK_OK;   // nothing within the tolerance: no record
    }
    ctx->tune[{n, precision}] = *best;
    tuner_save(ctx);
    *depth = best->depth;
    *tile = best->tile;
    return STARK_OK;
}

stark_status tuned_depth(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n, int precision,
                         hipStream_t st, int* depth, int* tile) {
    auto it = ctx->tune.find({n, precision});
    if (it != ctx->tune.end()) {
        *depth = it->second.depth;
        *tile = it->second.tile;
        return STARK_OK;
    }
    std::vector<TuneEntry> results;
    return tune_range(ctx, A, B, C, n, precision, 0, 5, 0.0, true, st, results, depth, tile);
}

}  // namespace stk
