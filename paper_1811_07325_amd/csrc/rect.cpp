// Rectangular products C (m x n) = A (m x k) B (k x n).  The paper treats
// n = 2^p and defers other shapes to partitioning (Section III-A); here the
// partition is into square s x s blocks: A and B are packed into zero-padded
// blocks, every block product A_ip B_pj (MB NB KB of them) is one problem of
// a grouped launch of the square path (stark_gemm_batched), and
// C_ij = sum over p of the products, in binary32 in ascending p, cropped.
// s is the smallest multiple of 64 * 2^depth covering min(m, k, n), so every
// block is a square problem with no further padding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"

namespace stk {

static int64_t rect_edge(int64_t m, int64_t k, int64_t n, int depth) {
    const int64_t q = kLeafGranule << depth;
    const int64_t lo = std::min(m, std::min(k, n));
    return (lo + q - 1) / q * q;
}

static stark_status ensure_rect(stark_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->rect_bytes) return STARK_OK;
    if (ctx->rect) {             // in-flight work may still read the old blocks
        STK_HIP(hipDeviceSynchronize());
        STK_HIP(hipFree(ctx->rect));
        ctx->rect = nullptr;
        ctx->rect_bytes = 0;
    }
    if (hipMalloc(&ctx->rect, bytes) != hipSuccess) {
        (void)hipGetLastError();
        ctx->rect = nullptr;
        set_error("cannot allocate %zu bytes for the rectangular blocks", bytes);
        return STARK_ENOMEM;
    }
    ctx->rect_bytes = bytes;
    return STARK_OK;
}

static bool overlap(const void* a, size_t an, const void* b, size_t bn) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bn && pb < pa + an;
}

// Pack, multiply the block products as one batch, reduce (stark_gemm_rect).
static stark_status rect_run(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t m, int64_t k, int64_t n,
                             int64_t s, int64_t MB, int64_t KB, int64_t NB, int depth, int prec, hipStream_t st) {
    const size_t ss = (size_t)s * (size_t)s;
    const int64_t count = MB * NB * KB;
    float* Ablk = static_cast<float*>(ctx->rect);
    float* Bblk = Ablk + (size_t)(MB * KB) * ss;
    float* Pblk = Bblk + (size_t)(KB * NB) * ss;
    STK_HIP(launch_pack_blocks(A, m, k, k, Ablk, s, st));
    STK_HIP(launch_pack_blocks(B, k, n, n, Bblk, s, st));
    std::vector<const float*> pa(count), pb(count);
    std::vector<float*> pc(count);
    std::vector<int64_t> ns(count, s);
    for (int64_t i = 0; i < MB; ++i)
        for (int64_t j = 0; j < NB; ++j)
            for (int64_t p = 0; p < KB; ++p) {
                const int64_t t = (i * NB + j) * KB + p;
                pa[t] = Ablk + (size_t)(i * KB + p) * ss;
                pb[t] = Bblk + (size_t)(p * NB + j) * ss;
                pc[t] = Pblk + (size_t)t * ss;
            }
    const stark_status rc = gemm_batched(ctx, (int)count, pa.data(), pb.data(), pc.data(), ns.data(), depth, prec, st);
    if (rc != STARK_OK) return rc;
    STK_HIP(launch_reduce_blocks(Pblk, C, m, n, s, MB, NB, KB, st));
    return STARK_OK;
}

}  // namespace stk

using namespace stk;

extern "C" {

int64_t stark_rect_block_edge(int64_t m, int64_t k, int64_t n, int depth) {
    if (m <= 0 || k <= 0 || n <= 0 || depth < 0 || depth > STARK_MAX_DEPTH) return -1;
    return rect_edge(m, k, n, depth);
}

stark_status stark_gemm_rect(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t m, int64_t k,
                             int64_t n, int depth, stark_precision prec, void* stream) {
    if (!ctx) { set_error("ctx is NULL"); return STARK_EINVAL; }
    if (!A || !B || !C) { set_error("A, B and C must be non-NULL device pointers"); return STARK_EINVAL; }
    if (m <= 0 || k <= 0 || n <= 0) { set_error("m, k and n must be positive"); return STARK_EINVAL; }
    if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) & 15) {
        set_error("A, B and C must be 16-byte aligned");
        return STARK_EINVAL;
    }
    if (planes_for((int)prec) < 0) { set_error("unknown precision %d", (int)prec); return STARK_EUNSUPPORTED; }
    if (depth == STARK_DEPTH_AUTO) depth = model_depth(std::min(m, std::min(k, n)), (int)prec);
    if (depth < 0 || depth > STARK_MAX_DEPTH) { set_error("depth %d out of range", depth); return STARK_EINVAL; }
    const size_t cb = (size_t)m * (size_t)n * 4;
    if (overlap(C, cb, A, (size_t)m * (size_t)k * 4) || overlap(C, cb, B, (size_t)k * (size_t)n * 4)) {
        set_error("C overlaps A or B");
        return STARK_EINVAL;
    }
    const int64_t s = rect_edge(m, k, n, depth);
    const int64_t MB = (m + s - 1) / s, KB = (k + s - 1) / s, NB = (n + s - 1) / s;
    const int64_t count = MB * NB * KB;
    if (count > 4096) {
        set_error("%lld block products (m=%lld k=%lld n=%lld): more than 4096", (long long)count, (long long)m,
                  (long long)k, (long long)n);
        return STARK_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(ctx->mu);
    STK_HIP(hipSetDevice(ctx->device));
    stark_status rc = ensure_rect(ctx, (size_t)(MB * KB + KB * NB + count) * (size_t)s * (size_t)s * sizeof(float));
    if (rc != STARK_OK) return rc;
    if ((rc = ws_wait(ctx, st)) != STARK_OK) return rc;
    return ws_done(ctx, st, rect_run(ctx, A, B, C, m, k, n, s, MB, KB, NB, depth, (int)prec, st));
}

}  // extern "C"
