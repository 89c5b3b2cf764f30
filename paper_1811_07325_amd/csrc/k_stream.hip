// HBM-streaming kernels of the Strassen hot path (gfx950):
//   k_pad      zero-padded copy of A and B (classical product of a padded size)
//   k_divide   one recursion level of the divide step: the operand sums of
//              all 7^l nodes of level l (Algorithm 1; Section III-C-1)
//   k_split    last divide level(s) of the 16-bit paths: the seven operand
//              pairs of every level-(k-1) node, split into 16-bit planes;
//              B-side planes are written transposed (k contiguous) for the
//              leaf products
//   k_combine  one recursion level of the combine step (Algorithm 1;
//              Section III-C-3): C11..C22 of every node from M1..M7
//   k_combine2 the two deepest combine levels in one pass
// Each takes the variant (Algorithm 1 or Winograd's) as a template argument.
//
// All are memory-bound streams: each thread moves 16-byte vectors, issues all
// of its loads before any store, and the block -> (node, chunk) map keeps a
// block inside one node so the walk that finds the node's operands runs once
// per block.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace stk {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;                          // float4 positions per thread
constexpr int kStreamPerBlock = kStreamThreads * kStreamUnroll;

__device__ __forceinline__ float4 f4add(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float4 f4sub(float4 a, float4 b) {
    return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}

// Four consecutive elements of row r, columns c..c+3 of the leading n x n
// block of a row-major matrix with leading dimension ld, zero outside (used
// only where the source is the user matrix, whose rows need not be 16-byte
// aligned).
__device__ __forceinline__ float4 load4_bounded(const float* X, int64_t ld, int64_t n, int64_t r, int64_t c) {
    const float* p = X + r * ld + c;
    // all four inside: four adjacent loads, which the compiler issues as one
    // 16-byte load (the target accepts 4-byte-aligned vector accesses)
    if (r < n && c + 3 < n) return make_float4(p[0], p[1], p[2], p[3]);
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (r < n && c + e < n) ? p[e] : 0.0f;
    return make_float4(v[0], v[1], v[2], v[3]);
}

// Store the four elements (r, c..c+3) of the leading n x n block of a
// row-major matrix with leading dimension ld, dropping those outside.
__device__ __forceinline__ void store4_bounded(float* X, int64_t ld, int64_t n, int64_t r, int64_t c, float4 v) {
    if (r >= n) return;
    float* p = X + r * ld + c;
    if (c + 3 < n) {   // adjacent stores: one 16-byte store
        p[0] = v.x; p[1] = v.y; p[2] = v.z; p[3] = v.w;
        return;
    }
    const float* e = &v.x;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (c + k < n) p[k] = e[k];
}

__device__ __forceinline__ float4 load4(const float* X, int64_t ld, int64_t n, int64_t r, int64_t c, bool bounded) {
    if (bounded) return load4_bounded(X, ld, n, r, c);
    return *reinterpret_cast<const float4*>(X + r * ld + c);
}

// Elements (r, c..c+3) of the operand of child C1 (0..6 for M1..M7) of a
// node whose operand X has quadrant edge H, formed exactly as k_divide forms
// them (one binary32 add per element, same operand order, and for Winograd's
// variant the same chain: S2 from the rounded S1, ...), so that operand need
// not be stored.  W: 0 Algorithm 1, 1 Winograd's variant.  C1 is a template
// argument so that every load is unconditional and can be issued early.
template <int W, int C1>
__device__ __forceinline__ float4 child4(const float* X, int64_t ld, int64_t n, int64_t H, int64_t r, int64_t c,
                                         int side, bool bounded) {
    auto q = [&](int a, int b) { return load4(X, ld, n, r + a * H, c + b * H, bounded); };
    if (W) {
        if (side == 0) {
            if (C1 == 0) return q(0, 0);
            if (C1 == 1) return q(0, 1);
            if (C1 == 2) return f4sub(q(0, 1), f4sub(f4add(q(1, 0), q(1, 1)), q(0, 0)));   // S4
            if (C1 == 3) return q(1, 1);
            if (C1 == 4) return f4add(q(1, 0), q(1, 1));                                   // S1
            if (C1 == 5) return f4sub(f4add(q(1, 0), q(1, 1)), q(0, 0));                   // S2
            return f4sub(q(0, 0), q(1, 0));                                                // S3
        }
        if (C1 == 0) return q(0, 0);
        if (C1 == 1) return q(1, 0);
        if (C1 == 2) return q(1, 1);
        if (C1 == 3) return f4sub(f4sub(q(1, 1), f4sub(q(0, 1), q(0, 0))), q(1, 0));      // T4
        if (C1 == 4) return f4sub(q(0, 1), q(0, 0));                                      // T1
        if (C1 == 5) return f4sub(q(1, 1), f4sub(q(0, 1), q(0, 0)));                      // T2
        return f4sub(q(1, 1), q(0, 1));                                                   // T3
    }
    if (side == 0) {
        if (C1 == 0) return f4add(q(0, 0), q(1, 1));
        if (C1 == 1) return f4add(q(1, 0), q(1, 1));
        if (C1 == 2) return q(0, 0);
        if (C1 == 3) return q(1, 1);
        if (C1 == 4) return f4add(q(0, 0), q(0, 1));
        if (C1 == 5) return f4sub(q(1, 0), q(0, 0));
        return f4sub(q(0, 1), q(1, 1));
    }
    if (C1 == 0) return f4add(q(0, 0), q(1, 1));
    if (C1 == 1) return q(0, 0);
    if (C1 == 2) return f4sub(q(0, 1), q(1, 1));
    if (C1 == 3) return f4sub(q(1, 0), q(0, 0));
    if (C1 == 4) return q(1, 1);
    if (C1 == 5) return f4add(q(0, 0), q(0, 1));
    return f4add(q(1, 0), q(1, 1));
}

// Calls f(std::integral_constant<int, c>) for a runtime c in 0..6, so the
// callee sees the child index as a constant.
template <class F>
__device__ __forceinline__ void with_child(int c, F&& f) {
    switch (c) {
        case 0: f(std::integral_constant<int, 0>{}); break;
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        default: f(std::integral_constant<int, 6>{}); break;
    }
}

// ---------------------------------------------------------------------------
// Zero-padded copies A -> pad_a, B -> pad_b (np x np).  grid.y = side.
// ---------------------------------------------------------------------------
template <class Src>
__global__ __launch_bounds__(kStreamThreads) void k_pad(Src src) {
    int64_t local;
    const ProbDesc& d = src.get(src.locate(blockIdx.x, local));
    const int side = blockIdx.y;
    const float* X = side ? d.B : d.A;
    float4* out = reinterpret_cast<float4*>(reinterpret_cast<float*>(d.ws) + (side ? d.pad_b : d.pad_a));
    const int64_t rq = d.np / 4;
    const int64_t total = d.np * rq;
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t f = local * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
        if (f < total) {
            const int64_t r = f / rq, c = (f - r * rq) * 4;
            out[f] = load4_bounded(X, d.ldu, d.n, r, c);
        }
    }
}

// ---------------------------------------------------------------------------
// Divide, level l: for every node of the level, read its four quadrants once
// and write the materialised operand blocks: 5 per side (Algorithm 1) or 4
// (Winograd's variant), or all 7 in product order (a) when the level-0
// source is the unpadded user matrix, read with bounds so the padding is
// formed on the fly, and (b) when the level above is not stored (binary32
// path from depth 2 on: the last two levels in one pass), since the view
// operands would point into that level.  grid.y = side (0: A, 1: B).
// ---------------------------------------------------------------------------

// Operand blocks of one node at one float4 position: slot order (5 or 4
// blocks) or product order (7), as listed with slot_of (common.hpp).
template <int W>
__device__ __forceinline__ void divide_store(float4* o, int64_t q4, int side, int slots, float4 x11, float4 x12,
                                             float4 x21, float4 x22) {
    if (W) {
        if (side == 0) {
            const float4 s1 = f4add(x21, x22), s2 = f4sub(s1, x11), s3 = f4sub(x11, x21), s4 = f4sub(x12, s2);
            if (slots == 7) {
                o[0] = x11; o[q4] = x12; o[2 * q4] = s4; o[3 * q4] = x22;
                o[4 * q4] = s1; o[5 * q4] = s2; o[6 * q4] = s3;
            } else {
                o[0] = s1; o[q4] = s2; o[2 * q4] = s3; o[3 * q4] = s4;
            }
        } else {
            const float4 t1 = f4sub(x12, x11), t2 = f4sub(x22, t1), t3 = f4sub(x22, x12), t4 = f4sub(t2, x21);
            if (slots == 7) {
                o[0] = x11; o[q4] = x21; o[2 * q4] = x22; o[3 * q4] = t4;
                o[4 * q4] = t1; o[5 * q4] = t2; o[6 * q4] = t3;
            } else {
                o[0] = t1; o[q4] = t2; o[2 * q4] = t3; o[3 * q4] = t4;
            }
        }
        return;
    }
    if (side == 0) {
        if (slots == 7) {                       // S1..S7
            o[0] = f4add(x11, x22);
            o[q4] = f4add(x21, x22);
            o[2 * q4] = x11;
            o[3 * q4] = x22;
            o[4 * q4] = f4add(x11, x12);
            o[5 * q4] = f4sub(x21, x11);
            o[6 * q4] = f4sub(x12, x22);
        } else {                                // S1, S2, S5, S6, S7
            o[0] = f4add(x11, x22);
            o[q4] = f4add(x21, x22);
            o[2 * q4] = f4add(x11, x12);
            o[3 * q4] = f4sub(x21, x11);
            o[4 * q4] = f4sub(x12, x22);
        }
    } else {
        if (slots == 7) {                       // T1..T7
            o[0] = f4add(x11, x22);
            o[q4] = x11;
            o[2 * q4] = f4sub(x12, x22);
            o[3 * q4] = f4sub(x21, x11);
            o[4 * q4] = x22;
            o[5 * q4] = f4add(x11, x12);
            o[6 * q4] = f4add(x21, x22);
        } else {                                // T1, T3, T4, T6, T7
            o[0] = f4add(x11, x22);
            o[q4] = f4sub(x12, x22);
            o[2 * q4] = f4sub(x21, x11);
            o[3 * q4] = f4add(x11, x12);
            o[4 * q4] = f4add(x21, x22);
        }
    }
}

template <class Src, int W>
__global__ __launch_bounds__(kStreamThreads) void k_divide(Src src, int level) {
    int64_t local;
    const ProbDesc& d = src.get(src.locate(xcd_slot(blockIdx.x, gridDim.x), local));
    const int side = blockIdx.y;
    const bool bounded = (level == 0) && d.bounded0;
    const int64_t m = d.np >> level, h = m >> 1;
    const int64_t hq = h >> 2;               // float4 per quadrant row
    const int64_t q4 = h * hq;               // float4 per quadrant
    const int64_t bpn = (q4 + kStreamPerBlock - 1) / kStreamPerBlock;
    // A level whose parent level is not stored forms the node's operand on
    // the fly from the grandparent's, as child node % 7 (child4); the seven
    // siblings of one chunk are consecutive logical blocks (one XCD, shared
    // grandparent reads in its L2).
    const bool fused = level > 0 && d.div_slots[level - 1] == 0;
    int64_t node, chunk;
    if (fused) {
        const int64_t rest = local / 7;
        chunk = rest % bpn;
        node = 7 * (rest / bpn) + local % 7;
    } else {
        node = local / bpn;
        chunk = local - node * bpn;
    }
    const float* X;
    int64_t ld;
    if (fused) resolve(d, side, level - 1, node / 7, X, ld);
    else resolve(d, side, level, node, X, ld);
    const bool fbounded = fused && level == 1 && d.bounded0;
    const int c1 = (int)(node % 7);
    const int slots = d.div_slots[level];
    float4* out = reinterpret_cast<float4*>(reinterpret_cast<float*>(d.ws) +
                                            (side ? d.div_b[level] : d.div_a[level]) +
                                            node * slots * h * h);

    if (fused) {
        with_child(c1, [&](auto C1) {
            float4 q11[kStreamUnroll], q12[kStreamUnroll], q21[kStreamUnroll], q22[kStreamUnroll];
#pragma unroll
            for (int u = 0; u < kStreamUnroll; ++u) {
                const int64_t f = chunk * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
                if (f < q4) {
                    const int64_t r = f / hq, c = (f - r * hq) * 4;
                    q11[u] = child4<W, C1>(X, ld, d.n, 2 * h, r, c, side, fbounded);
                    q12[u] = child4<W, C1>(X, ld, d.n, 2 * h, r, c + h, side, fbounded);
                    q21[u] = child4<W, C1>(X, ld, d.n, 2 * h, r + h, c, side, fbounded);
                    q22[u] = child4<W, C1>(X, ld, d.n, 2 * h, r + h, c + h, side, fbounded);
                }
            }
#pragma unroll
            for (int u = 0; u < kStreamUnroll; ++u) {
                const int64_t f = chunk * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
                if (f < q4) divide_store<W>(out + f, q4, side, slots, q11[u], q12[u], q21[u], q22[u]);
            }
        });
        return;
    }
    float4 q11[kStreamUnroll], q12[kStreamUnroll], q21[kStreamUnroll], q22[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t f = chunk * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
        if (f < q4) {
            const int64_t r = f / hq, c = (f - r * hq) * 4;
            if (bounded) {
                q11[u] = load4_bounded(X, ld, d.n, r, c);
                q12[u] = load4_bounded(X, ld, d.n, r, c + h);
                q21[u] = load4_bounded(X, ld, d.n, r + h, c);
                q22[u] = load4_bounded(X, ld, d.n, r + h, c + h);
            } else {
                const float* p = X + r * ld + c;
                q11[u] = *reinterpret_cast<const float4*>(p);
                q12[u] = *reinterpret_cast<const float4*>(p + h);
                q21[u] = *reinterpret_cast<const float4*>(p + h * ld);
                q22[u] = *reinterpret_cast<const float4*>(p + h * ld + h);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t f = chunk * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
        if (f < q4) divide_store<W>(out + f, q4, side, slots, q11[u], q12[u], q21[u], q22[u]);
    }
}

// ---------------------------------------------------------------------------
// bf16 split.  hi = RNE(x), then mid/lo = RNE(residual); residuals are exact
// in binary32.  v_cvt_pk_bf16_f32 rounds to nearest even.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    __bf16 b = (__bf16)x;
    return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ uint16_t f16_bits(float x) {
    _Float16 h = (_Float16)x;     // v_cvt_f16_f32: round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_value(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
}
__device__ __forceinline__ float bf16_value(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// Seven operand values of the products of one node at one position, in
// product order: Algorithm 1 (W = 0) or Winograd's variant (W = 1).
template <int W>
__device__ __forceinline__ void seven(int side, float x11, float x12, float x21, float x22, float* o) {
    if (W) {
        if (side == 0) {
            const float s1 = x21 + x22, s2 = s1 - x11, s3 = x11 - x21, s4 = x12 - s2;
            o[0] = x11; o[1] = x12; o[2] = s4; o[3] = x22; o[4] = s1; o[5] = s2; o[6] = s3;
        } else {
            const float t1 = x12 - x11, t2 = x22 - t1, t3 = x22 - x12, t4 = t2 - x21;
            o[0] = x11; o[1] = x21; o[2] = x22; o[3] = t4; o[4] = t1; o[5] = t2; o[6] = t3;
        }
        return;
    }
    if (side == 0) {
        o[0] = x11 + x22; o[1] = x21 + x22; o[2] = x11; o[3] = x22;
        o[4] = x11 + x12; o[5] = x21 - x11; o[6] = x12 - x22;
    } else {
        o[0] = x11 + x22; o[1] = x11; o[2] = x12 - x22; o[3] = x21 - x11;
        o[4] = x22; o[5] = x11 + x12; o[6] = x21 + x22;
    }
}

// Last divide level of the bf16 paths.  NOUT = 7: every node of level
// depth-1 gives the seven operand pairs of its children (the leaves);
// NOUT = 1 (depth 0): the root operands themselves.  Each output block (leaf
// edge L) is written as P bf16 planes in the blocked layout of blk_offset
// (common.hpp): A side with rows = rows of S, B side with rows = columns of T
// (transposed), so the leaf GEMM reads both k-contiguous.
//
// A block covers a kSplitRows x 64 tile of output positions; thread t owns
// rows kSplitRPT*(t/16).. and columns 4*(t%16)..+3 of it, read as float4
// (16 threads cover a 256-byte row segment).  A side: the tile of each
// output and plane goes through LDS (rows of 64 + 8 16-bit terms) and is
// written back in 16-byte chunks, one whole 1 KB block of the blocked layout
// per wave store.  B side: the tile is transposed through LDS (rows of
// kSplitRows + 8 16-bit terms) and written back in 16-byte chunks of T^T
// rows.  Both sides take kSplitRound outputs at a time.
#ifndef STK_SPLIT_ROWS
#define STK_SPLIT_ROWS 32
#endif
constexpr int kSplitTile = 64;                      // tile columns
constexpr int kSplitRows = STK_SPLIT_ROWS;          // tile rows (64 or 32)
constexpr int kSplitRPT = kSplitRows / 16;          // rows per thread
constexpr int kSplitLdsRow = kSplitRows + 8;        // bf16 per LDS row of T^T (16-byte aligned)
static_assert(kSplitRows == 64 || kSplitRows == 32, "split tile rows");

#ifndef STK_SPLIT_ROUND2
#define STK_SPLIT_ROUND2 2
#endif
template <int P> struct SplitRound { static constexpr int R = STK_SPLIT_ROUND2; };
template <> struct SplitRound<3> { static constexpr int R = (STK_SPLIT_ROUND2 + 1) / 2; };

// v[o][i][e]: output o at tile row i, column e of this thread's 4 x 4 piece.
// FUSED: X is the operand of the grandparent (edge 4L) and the parent's
// quadrant values are formed on the fly as child c1's operand (child4).
template <int NOUT, bool FUSED, int W, int C1>
__device__ __forceinline__ void split_values(const float* X, int64_t ld, int64_t n, int64_t L, int64_t r0, int64_t c0,
                                             int side, bool bounded, float (&v)[NOUT][kSplitRPT][4]) {
    auto quad = [&](int64_t r, int64_t c) {
        return FUSED ? child4<W, C1>(X, ld, n, 2 * L, r, c, side, bounded) : load4(X, ld, n, r, c, bounded);
    };
#pragma unroll
    for (int i = 0; i < kSplitRPT; ++i) {
        const int64_t r = r0 + i;
        if (NOUT == 7) {
            const float4 x11 = quad(r, c0);
            const float4 x12 = quad(r, c0 + L);
            const float4 x21 = quad(r + L, c0);
            const float4 x22 = quad(r + L, c0 + L);
            const float* p11 = &x11.x; const float* p12 = &x12.x;
            const float* p21 = &x21.x; const float* p22 = &x22.x;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float s7[7];
                seven<W>(side, p11[e], p12[e], p21[e], p22[e], s7);
#pragma unroll
                for (int o = 0; o < NOUT; ++o) v[o][i][e] = s7[o];
            }
        } else {
            const float4 x = load4(X, ld, n, r, c0, bounded);
            v[0][i][0] = x.x; v[0][i][1] = x.y; v[0][i][2] = x.z; v[0][i][3] = x.w;
        }
    }
}

// Split 4 values into P planes: planes[p] holds 4 16-bit terms packed in 8
// bytes -- bfloat16, or (fp16) binary16 of the values times `scale` (a power
// of two, so the scaling is exact).
template <int P, int N>
__device__ __forceinline__ void splitN(const float (&x)[N], uint32_t (&planes)[P][N / 2], bool fp16, float scale) {
    float r[N];
#pragma unroll
    for (int e = 0; e < N; ++e) r[e] = fp16 ? x[e] * scale : x[e];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        uint16_t b[N];
#pragma unroll
        for (int e = 0; e < N; ++e) {
            b[e] = fp16 ? f16_bits(r[e]) : bf16_bits(r[e]);
            r[e] = r[e] - (fp16 ? f16_value(b[e]) : bf16_value(b[e]));
        }
#pragma unroll
        for (int e = 0; e < N / 2; ++e) planes[p][e] = (uint32_t)b[2 * e] | ((uint32_t)b[2 * e + 1] << 16);
    }
}

// 4 or 2 consecutive 16-bit terms (8 or 4 bytes) at p.
template <int N>
__device__ __forceinline__ void store_terms(uint16_t* p, const uint32_t (&w)[N / 2]) {
    if (N == 4) *reinterpret_cast<uint2*>(p) = make_uint2(w[0], w[N / 2 - 1]);
    else *reinterpret_cast<uint32_t*>(p) = w[0];
}

// `node`: the level-(depth-1) node whose seven children's operands are
// written (FUSED: formed from its parent's operand, node / 7 at level
// depth-2, as child node % 7).
template <int NOUT, int P, bool FUSED, int W, int C1>
__device__ __forceinline__ void split_body(const ProbDesc& d, int side, int64_t node, int64_t tile, bool bounded,
                                           uint16_t* lds) {
    const int64_t L = d.leaf;
    const int64_t tiles_row = L / kSplitTile;
    const int64_t R0 = (tile / tiles_row) * kSplitRows, C0 = (tile % tiles_row) * kSplitTile;
    const int tid = threadIdx.x;
    const int ri = kSplitRPT * (tid >> 4), ci = 4 * (tid & 15);
    const int plevel = FUSED ? d.depth - 2 : (NOUT == 7) ? d.depth - 1 : 0;
    const float* X;
    int64_t ld;
    resolve(d, side, plevel, FUSED ? node / 7 : node, X, ld);
    uint16_t* base = reinterpret_cast<uint16_t*>(d.ws) + (side ? d.leaf_b : d.leaf_a) +
                     node * (int64_t)NOUT * P * L * L;
    const int64_t LL = L * L;

    float v[NOUT][kSplitRPT][4];
    split_values<NOUT, FUSED, W, C1>(X, ld, d.n, L, R0 + ri, C0 + ci, side, bounded, v);
    const bool fp16 = d.fp16 != 0;
    const float scale =
        fp16 ? ldexpf(1.0f, reinterpret_cast<const int*>(reinterpret_cast<const float*>(d.ws) + d.scale)[2 * kScaleParts + side])
             : 1.0f;

    constexpr int R = NOUT == 1 ? 1 : SplitRound<P>::R;
    if (side == 0) {
        // staged through LDS (rows of 64 + 8 16-bit terms) so that each
        // wave store writes one whole 1 KB block of the blocked layout:
        // lane l of a block takes row 16 rb + l / 4 and chunk 4 kb + l % 4
        constexpr int ROWA = kSplitTile + 8;
        constexpr int TILE_A = kSplitRows * ROWA;
        static_assert(TILE_A <= kSplitTile * kSplitLdsRow, "A tile fits the LDS of a B tile");
        constexpr int BLOCKS = (kSplitRows / 16) * (kSplitTile / 32);   // 1 KB blocks per output and plane
#pragma unroll
        for (int o0 = 0; o0 < NOUT; o0 += R) {
#pragma unroll
            for (int oo = 0; oo < R; ++oo) {
                if (o0 + oo >= NOUT) break;
#pragma unroll
                for (int i = 0; i < kSplitRPT; ++i) {
                    uint32_t pl[P][2];
                    splitN<P, 4>(v[o0 + oo][i], pl, fp16, scale);
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        store_terms<4>(lds + (oo * P + p) * TILE_A + (ri + i) * ROWA + ci, pl[p]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int oo = 0; oo < R; ++oo) {
                if (o0 + oo >= NOUT) break;
#pragma unroll
                for (int p = 0; p < P; ++p)
#pragma unroll
                    for (int h = 0; h < BLOCKS * 64 / kStreamThreads; ++h) {
                        const int id = tid + kStreamThreads * h;
                        const int blk = id >> 6, l = id & 63;
                        const int row = 16 * (blk >> 1) + (l >> 2), chunk = 4 * (blk & 1) + (l & 3);
                        const uint4 val = *reinterpret_cast<const uint4*>(lds + (oo * P + p) * TILE_A + row * ROWA + 8 * chunk);
                        *reinterpret_cast<uint4*>(base + ((int64_t)(o0 + oo) * P + p) * LL +
                                                  blk_offset(R0 + row, C0 + 8 * chunk, L)) = val;
                    }
            }
            __syncthreads();
        }
        return;
    }
    constexpr int TILE_U16 = kSplitTile * kSplitLdsRow;     // 64 rows of T^T
#pragma unroll
    for (int o0 = 0; o0 < NOUT; o0 += R) {
        // transpose into LDS: column ci + e of T becomes row ci + e of T^T
#pragma unroll
        for (int oo = 0; oo < R; ++oo) {
            if (o0 + oo >= NOUT) break;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float col[kSplitRPT];
#pragma unroll
                for (int i = 0; i < kSplitRPT; ++i) col[i] = v[o0 + oo][i][e];
                uint32_t pl[P][kSplitRPT / 2];
                splitN<P, kSplitRPT>(col, pl, fp16, scale);
#pragma unroll
                for (int p = 0; p < P; ++p)
                    store_terms<kSplitRPT>(lds + (oo * P + p) * TILE_U16 + (ci + e) * kSplitLdsRow + ri, pl[p]);
            }
        }
        __syncthreads();
        // write back whole rows of T^T: kSplitRows / 8 chunks of 16 bytes per row
        constexpr int CPR = kSplitRows / 8;
#pragma unroll
        for (int oo = 0; oo < R; ++oo) {
            if (o0 + oo >= NOUT) break;
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int h = 0; h < kSplitTile * CPR / kStreamThreads; ++h) {
                    const int id = tid + kStreamThreads * h;
                    const int j = id / CPR, q = id % CPR;
                    const uint4 val = *reinterpret_cast<const uint4*>(lds + (oo * P + p) * TILE_U16 + j * kSplitLdsRow + 8 * q);
                    *reinterpret_cast<uint4*>(base + ((int64_t)(o0 + oo) * P + p) * LL + blk_offset(C0 + j, R0 + 8 * q, L)) =
                        val;
                }
        }
        __syncthreads();
    }
}

// grid.y = side.  From depth 2 on, the last two divide levels run here (the
// level-(depth-2) sums are formed on the fly and never stored): the seven
// siblings of one tile position are consecutive logical blocks, placed on
// one XCD, so the grandparent tiles they share are re-read from its L2.  The
// source is read with bounds when it is the unpadded user matrix.
template <class Src, int P, int W>
__global__ __launch_bounds__(kStreamThreads) void k_split(Src src) {
    constexpr int R = SplitRound<P>::R;
    __shared__ __attribute__((aligned(16))) uint16_t lds[R * P * kSplitTile * kSplitLdsRow];
    int64_t local;
    const ProbDesc& d = src.get(src.locate(xcd_slot(blockIdx.x, gridDim.x), local));
    const int side = blockIdx.y;
    const int64_t L = d.leaf;
    const int64_t tiles = (L / kSplitRows) * (L / kSplitTile);
    if (d.depth >= 2) {
        const int64_t c1 = local % 7, rest = local / 7;
        const int64_t tile = rest % tiles, node = 7 * (rest / tiles) + c1;
        with_child((int)c1, [&](auto C1) {
            split_body<7, P, true, W, C1>(d, side, node, tile, d.bounded0 && d.depth == 2, lds);
        });
        return;
    }
    const int64_t node = local / tiles, tile = local - node * tiles;
    const bool bounded = d.bounded0 != 0;
    if (d.depth == 0) split_body<1, P, false, W, 0>(d, side, node, tile, bounded, lds);
    else split_body<7, P, false, W, 0>(d, side, node, tile, bounded, lds);
}

// ---------------------------------------------------------------------------
// FP16X3 scaling.  k_absmax: kScaleParts blocks per matrix take the largest
// magnitude of a contiguous chunk of A (grid.y = 0) or B (1).  k_scale_exp:
// one block per problem reduces the partial maxima and stores the exponents
// e = 14 - depth - E, with max = m 2^E (m in [0.5, 1)): multiplying by 2^e
// keeps every leaf operand (at most 2^depth max) below 2^14; Winograd's
// variant sums up to 4 blocks per level, so there e = 14 - 2 depth - E.
// e is capped at 127 so that 2^e is a finite binary32 (matrices whose largest
// magnitude is below about 2^-113 are scaled by 2^127 only).
// ---------------------------------------------------------------------------
constexpr int kAbsThreads = 1024;   // 16 waves per part: 2 x 256 parts fill the chip

template <class Src>
__global__ __launch_bounds__(kAbsThreads) void k_absmax(Src src) {
    __shared__ float part[kAbsThreads];
    int64_t local;
    const ProbDesc& d = src.get(src.locate(blockIdx.x, local));
    const int side = blockIdx.y;
    const float* X = side ? d.B : d.A;
    // the whole user matrix (for a peeled plan a superset of the core, so
    // the exponent still keeps every leaf operand in range)
    const int64_t count = d.ldu * d.ldu;
    // chunks of a multiple of 4 elements, so every chunk starts 16-byte aligned
    const int64_t chunk = ((count + kScaleParts - 1) / kScaleParts + 3) & ~int64_t(3);
    const int64_t lo = local * chunk < count ? local * chunk : count;
    const int64_t hi = lo + chunk < count ? lo + chunk : count;
    const int64_t nv = (hi - lo) >> 2;
    const float4* X4 = reinterpret_cast<const float4*>(X + lo);
    static_assert(kStreamUnroll == 4, "the final reduction below folds four partial maxima");
    float m[kStreamUnroll] = {};
    for (int64_t i = threadIdx.x; i < nv; i += kStreamUnroll * kAbsThreads) {
        float4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const int64_t j = i + u * kAbsThreads;
            v[u] = j < nv ? X4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u)
            m[u] = fmaxf(m[u], fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)), fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
    }
    for (int64_t i = lo + 4 * nv + threadIdx.x; i < hi; i += kAbsThreads) m[0] = fmaxf(m[0], fabsf(X[i]));
    part[threadIdx.x] = fmaxf(fmaxf(m[0], m[1]), fmaxf(m[2], m[3]));
    __syncthreads();
    for (int w = kAbsThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = fmaxf(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) reinterpret_cast<float*>(d.ws)[d.scale + side * kScaleParts + local] = part[0];
}

template <class Src>
__global__ __launch_bounds__(kScaleParts) void k_scale_exp(Src src) {
    __shared__ float part[2][kScaleParts];
    int64_t local;
    const ProbDesc& d = src.get(src.locate(blockIdx.x, local));
    const float* pm = reinterpret_cast<const float*>(d.ws) + d.scale;
    part[0][threadIdx.x] = pm[threadIdx.x];
    part[1][threadIdx.x] = pm[kScaleParts + threadIdx.x];
    __syncthreads();
    for (int w = kScaleParts / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            part[0][threadIdx.x] = fmaxf(part[0][threadIdx.x], part[0][threadIdx.x + w]);
            part[1][threadIdx.x] = fmaxf(part[1][threadIdx.x], part[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) {
        const float m = part[threadIdx.x][0];
        int E = 0;
        if (m > 0.0f) frexpf(m, &E);
        // a leaf operand sums at most 2 blocks per level (4 in Winograd's variant)
        const int growth = d.variant ? 2 * d.depth : d.depth;
        const int e = m > 0.0f ? 14 - growth - E : 0;
        reinterpret_cast<int*>(reinterpret_cast<float*>(d.ws) + d.scale)[2 * kScaleParts + threadIdx.x] =
            e < 127 ? e : 127;
    }
}

// ---------------------------------------------------------------------------
// Combine, level l: node's C quadrants from its children's products M1..M7
// (Algorithm 1 with C22 = M1 - M2 + M3 + M6), additions left to right.
// Level 0 writes the user's C, cropping to n x n when padded.
// ---------------------------------------------------------------------------
// The four quadrants of a node from its seven products, in the fixed order
// of Algorithm 1 (W = 0; C22 with +M3) or of Winograd's variant (W = 1:
// U2 = M1 + M6, U3 = U2 + M7, C11 = M1 + M2, C12 = (U2 + M5) + M3,
// C21 = U3 - M4, C22 = U3 + M5).
template <int W>
__device__ __forceinline__ void combine_quads(float4 m1, float4 m2, float4 m3, float4 m4, float4 m5, float4 m6,
                                              float4 m7, float4 (&c)[4]) {
    if (W) {
        const float4 u2 = f4add(m1, m6), u3 = f4add(u2, m7);
        c[0] = f4add(m1, m2);
        c[1] = f4add(f4add(u2, m5), m3);
        c[2] = f4sub(u3, m4);
        c[3] = f4add(u3, m5);
    } else {
        c[0] = f4add(f4sub(f4add(m1, m4), m5), m7);
        c[1] = f4add(m3, m5);
        c[2] = f4add(m2, m4);
        c[3] = f4add(f4add(f4sub(m1, m2), m3), m6);
    }
}

// Peeled plans (d.peel = r > 0): the recursion covers the leading d.n x d.n
// core of A, B and C (leading dimension d.ldu = d.n + r); each core output
// also takes the products through the r peeled columns of A and rows of B,
// C[i][j] += A[i][d.n + t] B[d.n + t][j] for t = 0 .. r-1 in order, one
// fused multiply-add per term, added when level 0 writes C.  v[a][b] holds
// the four outputs C[rows[a]][cols[b] .. cols[b] + 3].
template <int NR, int NC>
__device__ __forceinline__ void peel_fix(const ProbDesc& d, const int64_t (&rows)[NR], const int64_t (&cols)[NC],
                                         float4 (&v)[NR][NC]) {
    const int64_t ld = d.ldu, nc = d.n;
#pragma unroll 4
    for (int t = 0; t < d.peel; ++t) {
        float a[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) a[i] = d.A[rows[i] * ld + nc + t];
        const float* brow = d.B + (nc + t) * ld;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const float b0 = brow[cols[j]], b1 = brow[cols[j] + 1], b2 = brow[cols[j] + 2], b3 = brow[cols[j] + 3];
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                v[i][j].x = fmaf(a[i], b0, v[i][j].x);
                v[i][j].y = fmaf(a[i], b1, v[i][j].y);
                v[i][j].z = fmaf(a[i], b2, v[i][j].z);
                v[i][j].w = fmaf(a[i], b3, v[i][j].w);
            }
        }
    }
}

// PEEL: the variant launched for level 0 of peeled plans (with the fix-up;
// the plain variant keeps its registers free of it).
template <class Src, int W, bool PEEL>
__global__ __launch_bounds__(kStreamThreads) void k_combine(Src src, int level) {
    int64_t local;
    const ProbDesc& d = src.get(src.locate(blockIdx.x, local));
    const bool crop = (level == 0) && d.bounded0;
    const int64_t m = d.np >> level, h = m >> 1;
    const int64_t hq = h >> 2;
    const int64_t q4 = h * hq;
    const int64_t bpn = (q4 + kStreamPerBlock - 1) / kStreamPerBlock;
    const int64_t node = local / bpn, chunk = local - node * bpn;

    const float* wsf = reinterpret_cast<const float*>(d.ws);
    const float4* in = reinterpret_cast<const float4*>(
        wsf + ((level + 1 == d.depth) ? d.leaf_m : d.comb[level + 1]) + node * 7 * h * h);
    float* out;
    int64_t ldo;
    if (level == 0) {
        out = d.C;
        ldo = d.ldu;
    } else {
        out = reinterpret_cast<float*>(d.ws) + d.comb[level] + node * m * m;
        ldo = m;
    }
    const bool peel = PEEL && level == 0 && d.peel > 0;
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t f = chunk * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
        if (f >= q4) continue;
        const float4 m1 = in[f], m2 = in[q4 + f], m3 = in[2 * q4 + f], m4 = in[3 * q4 + f];
        const float4 m5 = in[4 * q4 + f], m6 = in[5 * q4 + f], m7 = in[6 * q4 + f];
        float4 cq[4];
        combine_quads<W>(m1, m2, m3, m4, m5, m6, m7, cq);
        const int64_t r = f / hq, c = (f - r * hq) * 4;
        if (peel) {
            const int64_t rows[2] = {r, r + h}, cols[2] = {c, c + h};
            float4 v[2][2] = {{cq[0], cq[1]}, {cq[2], cq[3]}};
            peel_fix<2, 2>(d, rows, cols, v);
            cq[0] = v[0][0]; cq[1] = v[0][1]; cq[2] = v[1][0]; cq[3] = v[1][1];
        }
        const float4 c11 = cq[0], c12 = cq[1], c21 = cq[2], c22 = cq[3];
        if (crop) {
            store4_bounded(out, ldo, d.n, r, c, c11);
            store4_bounded(out, ldo, d.n, r, c + h, c12);
            store4_bounded(out, ldo, d.n, r + h, c, c21);
            store4_bounded(out, ldo, d.n, r + h, c + h, c22);
        } else {
            float* p = out + r * ldo + c;
            *reinterpret_cast<float4*>(p) = c11;
            *reinterpret_cast<float4*>(p + h) = c12;
            *reinterpret_cast<float4*>(p + h * ldo) = c21;
            *reinterpret_cast<float4*>(p + h * ldo + h) = c22;
        }
    }
}

// Two combine levels in one pass: node P of level l (output m x m) from its
// 49 grandchildren (g x g, g = m/4) without writing the level-(l+1) outputs.
// A thread owns one float4 position (r, c) of the grandchild grid: for each
// child j it forms the child's four quadrant values at (r, c) from its seven
// products, exactly as k_combine does, and folds them into the parent's
// sixteen g x g sub-blocks as the children arrive.  Algorithm 1's order one
// level up (C11 = ((N1 + N4) - N5) + N7, ...) is child order, so running
// sums suffice; Winograd's (U2 = N1 + N6, ...) keeps N3, N4, N5 until N7.
// Either way the additions are those of two k_combine launches, in the same
// order, so the result equals them bit for bit.
template <class Src, int W, bool PEEL>
__global__ __launch_bounds__(kStreamThreads) void k_combine2(Src src, int level) {
    int64_t local;
    const ProbDesc& d = src.get(src.locate(blockIdx.x, local));
    const bool crop = (level == 0) && d.bounded0;
    const int64_t m = d.np >> level, g = m >> 2;
    const int64_t gq = g >> 2;                 // float4 per grandchild row
    const int64_t q4 = g * gq;                 // float4 per grandchild
    const int64_t bpn = (q4 + kStreamThreads - 1) / kStreamThreads;
    const int64_t node = local / bpn;
    const int64_t f = (local - node * bpn) * kStreamThreads + threadIdx.x;
    if (f >= q4) return;

    const float* wsf = reinterpret_cast<const float*>(d.ws);
    const float4* in = reinterpret_cast<const float4*>(
        wsf + ((level + 2 == d.depth) ? d.leaf_m : d.comb[level + 2]) + node * 49 * g * g);
    float* out;
    int64_t ldo;
    if (level == 0) {
        out = d.C;
        ldo = d.ldu;
    } else {
        out = reinterpret_cast<float*>(d.ws) + d.comb[level] + node * m * m;
        ldo = m;
    }
    // acc[Q][s]: parent quadrant Q (11, 12, 21, 22), sub-block s = 2 qa + qb
    float4 acc[4][4];
    float4 keep[3][4];   // Winograd: N3, N4, N5 (Algorithm 1 leaves it unused)
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const float4* mj = in + (int64_t)j * 7 * q4 + f;
        float4 nq[4];
        combine_quads<W>(mj[0], mj[q4], mj[2 * q4], mj[3 * q4], mj[4 * q4], mj[5 * q4], mj[6 * q4], nq);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float4 v = nq[s];
            if (W) {       // acc[1] holds U2 until the end
                switch (j) {
                    case 0: acc[0][s] = v; acc[1][s] = v; break;
                    case 1: acc[0][s] = f4add(acc[0][s], v); break;
                    case 2: keep[0][s] = v; break;
                    case 3: keep[1][s] = v; break;
                    case 4: keep[2][s] = v; break;
                    case 5: acc[1][s] = f4add(acc[1][s], v); break;
                    default: {
                        const float4 u3 = f4add(acc[1][s], v);
                        acc[1][s] = f4add(f4add(acc[1][s], keep[2][s]), keep[0][s]);
                        acc[2][s] = f4sub(u3, keep[1][s]);
                        acc[3][s] = f4add(u3, keep[2][s]);
                        break;
                    }
                }
                continue;
            }
            switch (j) {   // child j = N_{j+1}
                case 0: acc[0][s] = v; acc[3][s] = v; break;
                case 1: acc[2][s] = v; acc[3][s] = f4sub(acc[3][s], v); break;
                case 2: acc[1][s] = v; acc[3][s] = f4add(acc[3][s], v); break;
                case 3: acc[0][s] = f4add(acc[0][s], v); acc[2][s] = f4add(acc[2][s], v); break;
                case 4: acc[0][s] = f4sub(acc[0][s], v); acc[1][s] = f4add(acc[1][s], v); break;
                case 5: acc[3][s] = f4add(acc[3][s], v); break;
                default: acc[0][s] = f4add(acc[0][s], v); break;
            }
        }
    }
    const int64_t r = f / gq, c = (f - r * gq) * 4;
    if (PEEL && level == 0 && d.peel > 0) {
        // output rows r + a g and columns c + b g, a, b = 0..3: quadrant Q =
        // 2 (a / 2) + b / 2, sub-block 2 (a % 2) + b % 2
        const int64_t rows[4] = {r, r + g, r + 2 * g, r + 3 * g}, cols[4] = {c, c + g, c + 2 * g, c + 3 * g};
        float4 v[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[a][b] = acc[2 * (a >> 1) + (b >> 1)][2 * (a & 1) + (b & 1)];
        peel_fix<4, 4>(d, rows, cols, v);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[2 * (a >> 1) + (b >> 1)][2 * (a & 1) + (b & 1)] = v[a][b];
    }
#pragma unroll
    for (int Q = 0; Q < 4; ++Q)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const int64_t row = (Q >> 1) * 2 * g + (sb >> 1) * g + r;
            const int64_t col = (Q & 1) * 2 * g + (sb & 1) * g + c;
            if (crop) {
                store4_bounded(out, ldo, d.n, row, col, acc[Q][sb]);
            } else {
                *reinterpret_cast<float4*>(out + row * ldo + col) = acc[Q][sb];
            }
        }
}

// ---------------------------------------------------------------------------
// Rectangular products by square partition (the paper defers shapes other
// than n = 2^p to partitioning, Section III-A).
//   k_pack_blocks    rows x cols of X (leading dimension ld) into nbr x nbc
//                    contiguous s x s blocks, block (bi, bj) at
//                    (bi * nbc + bj) s^2, zero outside the matrix;
//   k_reduce_blocks  C (m x n, leading dimension n) from the block products
//                    P[(i NB + j) KB + p] (s x s each): C_ij = sum over p in
//                    ascending order, in binary32, cropped.
// The user matrices need not have 16-byte-aligned rows (k, n arbitrary), so
// they are read and written element by element; the blocks are float4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kStreamThreads) void k_pack_blocks(const float* X, int64_t rows, int64_t cols,
                                                                int64_t ld, float* dst, int64_t s, int64_t nblocks) {
    const int64_t per = s * s / 4;                // float4 per block
    const int64_t nbc = (cols + s - 1) / s;
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t f = (int64_t)blockIdx.x * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
        if (f >= nblocks * per) continue;
        const int64_t b = f / per, e = f - b * per;
        const int64_t r = e / (s / 4), c = (e - r * (s / 4)) * 4;
        const int64_t R = (b / nbc) * s + r, Cc = (b % nbc) * s + c;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (R < rows && Cc + q < cols) ? X[R * ld + Cc + q] : 0.0f;
        reinterpret_cast<float4*>(dst)[f] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

__global__ __launch_bounds__(kStreamThreads) void k_reduce_blocks(const float* P, float* C, int64_t m, int64_t n,
                                                                  int64_t s, int64_t MB, int64_t NB, int64_t KB) {
    const int64_t per = s * s / 4;
    const float4* P4 = reinterpret_cast<const float4*>(P);
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t f = (int64_t)blockIdx.x * kStreamPerBlock + u * kStreamThreads + threadIdx.x;
        if (f >= MB * NB * per) continue;
        const int64_t b = f / per, e = f - b * per;     // b = i NB + j
        const int64_t r = e / (s / 4), c = (e - r * (s / 4)) * 4;
        const int64_t R = (b / NB) * s + r, Cc = (b % NB) * s + c;
        if (R >= m || Cc >= n) continue;
        float4 acc = P4[(b * KB) * per + e];
        for (int64_t p = 1; p < KB; ++p) acc = f4add(acc, P4[(b * KB + p) * per + e]);
        const float* v = &acc.x;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (Cc + q < n) C[R * n + Cc + q] = v[q];
    }
}

// ---------------------------------------------------------------------------
// Border of a peeled plan (n = d.ldu, core nc = d.n, r = d.peel rows and
// columns peeled):
//   right:  C[i][nc + y] for i < nc, y < r
//   bottom: C[nc + y][j] for y < r, j < n
// each the whole inner product over t = 0 .. n-1 in binary32 (exact for
// integers): for r <= 4 in ascending order, one fused multiply-add per term;
// for larger r on the matrix cores (16 x 16 x 4 binary32 MFMAs, K ascending
// in steps of four).  A block
// owns 64 indices along the long side (right: rows i; bottom: columns j) and
// every short-side index y < r (RB >= r of them, the rest zero).  K runs in
// chunks of 64: the long side's 64 x 64 operand chunk and the short side's
// RB x 64 chunk sit in LDS (rows padded to 68 floats, so 16-byte reads of 16
// consecutive rows hit distinct banks) while the loads of the next chunk are
// in flight in registers.  With RB = 4 a thread owns one output (vector
// fused multiply-adds); with RB = 16 or 64 a wave owns 16 long x RB short
// outputs on the matrix cores (the vector path read 2 LDS bytes per
// multiply-add and was bound by LDS bandwidth: 2.6 ms for r = 64 at
// n = 16448).
// ---------------------------------------------------------------------------
constexpr int kPeelStrip = 64, kPeelK = 64, kPeelLd = kPeelK + 4;

template <int RB> struct PeelTile;   // thread tile of the vector path
template <> struct PeelTile<4> { static constexpr int TX = 1, TY = 1; };
template <> struct PeelTile<16> { static constexpr int TX = 1, TY = 4; };
template <> struct PeelTile<64> { static constexpr int TX = 4, TY = 4; };
typedef float peel_f32x4 __attribute__((ext_vector_type(4)));

template <class Src, int RB>
__global__ __launch_bounds__(kStreamThreads) void k_peel(Src src) {
    static_assert(RB <= kPeelMaxResidue, "short-side block");
    constexpr int TX = PeelTile<RB>::TX, TY = PeelTile<RB>::TY;
    constexpr int XS = kPeelStrip / TX, YS = RB / TY;      // thread grid XS x YS
    static_assert(XS * YS == kStreamThreads, "one output block per thread");
    int64_t local;
    const ProbDesc& d = src.get(src.locate(blockIdx.x, local));
    const int64_t n = d.ldu, nc = d.n;
    const int r = d.peel;
    const int64_t right_blocks = (nc + kPeelStrip - 1) / kPeelStrip;
    const bool right = local < right_blocks;
    const int64_t s0 = (right ? local : local - right_blocks) * kPeelStrip;
    const int64_t slen = right ? nc : n;
    __shared__ __attribute__((aligned(16))) float big[2][kPeelStrip][kPeelLd];   // [long index][t]
    __shared__ __attribute__((aligned(16))) float sm[2][RB][kPeelLd];           // [short index][t]
    const int tid = threadIdx.x;
    constexpr int BPT = kPeelStrip * kPeelK / kStreamThreads;   // long-side elements per thread
    constexpr int SPT = RB * kPeelK / kStreamThreads;           // short-side elements per thread
    float rb[BPT], rs[SPT];
    // long-side element u of this thread: lanes run along a matrix row (A row
    // s0 + x for the right border, B row k0 + t for the bottom one), so each
    // wave load reads 256 contiguous bytes whatever the row alignment
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int NWV = kStreamThreads / 64;
    auto big_at = [&](int u, int& x, int& t) {
        if (right) { t = lane; x = wv + NWV * u; }
        else { x = lane; t = wv + NWV * u; }
    };
    auto sm_at = [&](int u, int& y, int& t) {
        const int e = tid + kStreamThreads * u;
        if (right) { y = e % RB; t = e / RB; }      // B row k0 + t, column nc + y
        else { t = e % kPeelK; y = e / kPeelK; }    // A row nc + y, column k0 + t
    };
    // 16-byte loads where every row start and the border column nc are
    // 16-byte aligned (n and r multiples of 4, A and B 16-byte aligned): a
    // thread moves BPT / 4 and SPT / 4 float4, a wave four 256-byte row
    // segments (or 16 rows of the 64-float column strip) per load
    const bool vec = RB >= 16 && (n & 3) == 0 && (r & 3) == 0 && ((uintptr_t)d.A & 15) == 0 &&
                     ((uintptr_t)d.B & 15) == 0;
    constexpr int SQ = (SPT >= 4) ? RB / 4 : 1;     // float4 per short-side k-row
    auto fetch4 = [&](int64_t k0) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < BPT / 4; ++u) {
            const int e = tid + kStreamThreads * u, c4 = e & 15, ln = e >> 4;
            float4 v = z;
            if (right) {   // A row s0 + ln, columns k0 + 4 c4 ..
                const int64_t gx = s0 + ln, gt = k0 + 4 * c4;
                if (gx < slen && gt < n) v = *reinterpret_cast<const float4*>(d.A + gx * n + gt);
            } else {       // B row k0 + ln, columns s0 + 4 c4 ..
                const int64_t gt = k0 + ln, gx = s0 + 4 * c4;
                if (gx < slen && gt < n) v = *reinterpret_cast<const float4*>(d.B + gt * n + gx);
            }
            rb[4 * u] = v.x; rb[4 * u + 1] = v.y; rb[4 * u + 2] = v.z; rb[4 * u + 3] = v.w;
        }
#pragma unroll
        for (int u = 0; u < SPT / 4; ++u) {
            const int e = tid + kStreamThreads * u;
            float4 v = z;
            if (right) {   // B row k0 + t, columns nc + 4 y4 ..
                const int y4 = e % SQ, t = e / SQ;
                const int64_t gt = k0 + t;
                if (4 * y4 < r && gt < n) v = *reinterpret_cast<const float4*>(d.B + gt * n + nc + 4 * y4);
            } else {       // A row nc + y, columns k0 + 4 c4 ..
                const int c4 = e & 15, y = e >> 4;
                const int64_t gt = k0 + 4 * c4;
                if (y < r && gt < n) v = *reinterpret_cast<const float4*>(d.A + (nc + y) * n + gt);
            }
            rs[4 * u] = v.x; rs[4 * u + 1] = v.y; rs[4 * u + 2] = v.z; rs[4 * u + 3] = v.w;
        }
    };
    auto stash4 = [&](int buf) {
#pragma unroll
        for (int u = 0; u < BPT / 4; ++u) {
            const int e = tid + kStreamThreads * u, c4 = e & 15, ln = e >> 4;
            if (right) {
                *reinterpret_cast<float4*>(&big[buf][ln][4 * c4]) =
                    make_float4(rb[4 * u], rb[4 * u + 1], rb[4 * u + 2], rb[4 * u + 3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) big[buf][4 * c4 + q][ln] = rb[4 * u + q];
            }
        }
#pragma unroll
        for (int u = 0; u < SPT / 4; ++u) {
            const int e = tid + kStreamThreads * u;
            if (right) {
                const int y4 = e % SQ, t = e / SQ;
#pragma unroll
                for (int q = 0; q < 4; ++q) sm[buf][4 * y4 + q][t] = rs[4 * u + q];
            } else {
                const int c4 = e & 15, y = e >> 4;
                *reinterpret_cast<float4*>(&sm[buf][y][4 * c4]) =
                    make_float4(rs[4 * u], rs[4 * u + 1], rs[4 * u + 2], rs[4 * u + 3]);
            }
        }
    };
    auto fetch = [&](int64_t k0) {
        if constexpr (RB >= 16) {
            if (vec) {
                fetch4(k0);
                return;
            }
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            int x, t;
            big_at(u, x, t);
            const int64_t gx = s0 + x, gt = k0 + t;
            rb[u] = (gx < slen && gt < n) ? (right ? d.A[gx * n + gt] : d.B[gt * n + gx]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            int y, t;
            sm_at(u, y, t);
            const int64_t gt = k0 + t;
            rs[u] = (y < r && gt < n) ? (right ? d.B[gt * n + nc + y] : d.A[(nc + y) * n + gt]) : 0.0f;
        }
    };
    auto stash = [&](int buf) {
        if constexpr (RB >= 16) {
            if (vec) {
                stash4(buf);
                return;
            }
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            int x, t;
            big_at(u, x, t);
            big[buf][x][t] = rb[u];
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            int y, t;
            sm_at(u, y, t);
            sm[buf][y][t] = rs[u];
        }
    };

    const int64_t KC = (n + kPeelK - 1) / kPeelK;
    if constexpr (RB >= 16) {
        // Matrix cores: out[x][y] = sum_t big[x][t] sm[y][t] as 16 x 16 x 4
        // binary32 MFMAs; wave wv owns long indices 16 wv .. 16 wv + 15 and
        // every short index (RB / 16 tiles).  Lane (li, lg) supplies k = t +
        // lg of row li of each operand (conflict-free: row stride 68 words).
        constexpr int NTY = RB / 16;
        const int li = lane & 15, lg = lane >> 4;
        peel_f32x4 acc[NTY];
#pragma unroll
        for (int j = 0; j < NTY; ++j) acc[j] = peel_f32x4{0.f, 0.f, 0.f, 0.f};
        fetch(0);
        stash(0);
        __syncthreads();
        for (int64_t kc = 0; kc < KC; ++kc) {
            const int buf = (int)(kc & 1);
            if (kc + 1 < KC) fetch((kc + 1) * kPeelK);
#pragma unroll 4
            for (int t = 0; t < kPeelK; t += 4) {
                const float av = big[buf][16 * wv + li][t + lg];
#pragma unroll
                for (int j = 0; j < NTY; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sm[buf][16 * j + li][t + lg], acc[j], 0, 0, 0);
            }
            // the other buffer was last read in the previous chunk, before the
            // barrier that ended it
            if (kc + 1 < KC) stash(buf ^ 1);
            __syncthreads();
        }
        // lane (li, lg) holds out[16 wv + 4 lg + v][16 j + li], v = 0..3
#pragma unroll
        for (int j = 0; j < NTY; ++j) {
            const int y = 16 * j + li;
            if (y >= r) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gx = s0 + 16 * wv + 4 * lg + v;
                if (gx >= slen) continue;
                if (right) d.C[gx * n + nc + y] = acc[j][v];
                else d.C[(nc + y) * n + gx] = acc[j][v];
            }
        }
    } else {
        // outputs of this thread: long indices xa + XS i, short indices ya + YS j
        const int xa = tid % XS, ya = tid / XS;
        float acc[TX][TY];
#pragma unroll
        for (int i = 0; i < TX; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j) acc[i][j] = 0.0f;
        fetch(0);
        stash(0);
        __syncthreads();
        for (int64_t kc = 0; kc < KC; ++kc) {
            const int buf = (int)(kc & 1);
            if (kc + 1 < KC) fetch((kc + 1) * kPeelK);
#pragma unroll 2
            for (int t = 0; t < kPeelK; t += 4) {
                float4 a[TX], b[TY];
#pragma unroll
                for (int i = 0; i < TX; ++i) a[i] = *reinterpret_cast<const float4*>(&big[buf][xa + XS * i][t]);
#pragma unroll
                for (int j = 0; j < TY; ++j) b[j] = *reinterpret_cast<const float4*>(&sm[buf][ya + YS * j][t]);
#pragma unroll
                for (int i = 0; i < TX; ++i)
#pragma unroll
                    for (int j = 0; j < TY; ++j) {
                        acc[i][j] = fmaf(a[i].x, b[j].x, acc[i][j]);
                        acc[i][j] = fmaf(a[i].y, b[j].y, acc[i][j]);
                        acc[i][j] = fmaf(a[i].z, b[j].z, acc[i][j]);
                        acc[i][j] = fmaf(a[i].w, b[j].w, acc[i][j]);
                    }
            }
            if (kc + 1 < KC) stash(buf ^ 1);
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int64_t gx = s0 + xa + XS * i;
            if (gx >= slen) continue;
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int y = ya + YS * j;
                if (y >= r) continue;
                if (right) d.C[gx * n + nc + y] = acc[i][j];
                else d.C[(nc + y) * n + gx] = acc[i][j];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static int64_t pow7(int l) {
    int64_t p = 1;
    for (int i = 0; i < l; ++i) p *= 7;
    return p;
}

int64_t blocks_pad(const ProbDesc& d) {
    return (d.np * (d.np / 4) + kStreamPerBlock - 1) / kStreamPerBlock;
}
int64_t blocks_divide(const ProbDesc& d, int level) {
    const int64_t h = (d.np >> level) >> 1;
    const int64_t q4 = h * (h / 4);
    return pow7(level) * ((q4 + kStreamPerBlock - 1) / kStreamPerBlock);
}
int64_t blocks_split(const ProbDesc& d) {
    const int64_t tiles = (d.leaf / kSplitRows) * (d.leaf / kSplitTile);
    const int64_t nodes = d.depth > 0 ? pow7(d.depth - 1) : 1;
    return nodes * tiles;
}
int64_t blocks_combine(const ProbDesc& d, int level) { return blocks_divide(d, level); }
int64_t blocks_peel(const ProbDesc& d) {
    if (d.peel <= 0) return 0;
    return (d.n + kPeelStrip - 1) / kPeelStrip + (d.ldu + kPeelStrip - 1) / kPeelStrip;
}
int64_t blocks_combine2(const ProbDesc& d, int level) {
    const int64_t g = (d.np >> level) >> 2;
    const int64_t q4 = g * (g / 4);
    return pow7(level) * ((q4 + kStreamThreads - 1) / kStreamThreads);
}

template <class Src>
hipError_t launch_pad(const Src& s, int64_t blocks, hipStream_t st) {
    hipLaunchKernelGGL((k_pad<Src>), dim3((unsigned)blocks, 2), dim3(kStreamThreads), 0, st, s);
    return hipGetLastError();
}
template <class Src>
hipError_t launch_absmax(const Src& s, int64_t blocks, hipStream_t st) {
    hipLaunchKernelGGL((k_absmax<Src>), dim3((unsigned)blocks, 2), dim3(kAbsThreads), 0, st, s);
    return hipGetLastError();
}
template <class Src>
hipError_t launch_scale_exp(const Src& s, int64_t blocks, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_exp<Src>), dim3((unsigned)blocks), dim3(kScaleParts), 0, st, s);
    return hipGetLastError();
}
template <class Src>
hipError_t launch_divide(const Src& s, int level, int variant, int64_t blocks, hipStream_t st) {
    if (variant)
        hipLaunchKernelGGL((k_divide<Src, 1>), dim3((unsigned)blocks, 2), dim3(kStreamThreads), 0, st, s, level);
    else
        hipLaunchKernelGGL((k_divide<Src, 0>), dim3((unsigned)blocks, 2), dim3(kStreamThreads), 0, st, s, level);
    return hipGetLastError();
}
template <class Src>
hipError_t launch_split(const Src& s, int planes, int variant, int64_t blocks, hipStream_t st) {
    const dim3 grid((unsigned)blocks, 2), block(kStreamThreads);
    if (planes == 2 && !variant) hipLaunchKernelGGL((k_split<Src, 2, 0>), grid, block, 0, st, s);
    else if (planes == 2) hipLaunchKernelGGL((k_split<Src, 2, 1>), grid, block, 0, st, s);
    else if (!variant) hipLaunchKernelGGL((k_split<Src, 3, 0>), grid, block, 0, st, s);
    else hipLaunchKernelGGL((k_split<Src, 3, 1>), grid, block, 0, st, s);
    return hipGetLastError();
}
template <class Src>
hipError_t launch_combine2(const Src& s, int level, int variant, int64_t blocks, hipStream_t st, bool peel) {
    const dim3 grid((unsigned)blocks), block(kStreamThreads);
    if (peel && variant) hipLaunchKernelGGL((k_combine2<Src, 1, true>), grid, block, 0, st, s, level);
    else if (peel) hipLaunchKernelGGL((k_combine2<Src, 0, true>), grid, block, 0, st, s, level);
    else if (variant) hipLaunchKernelGGL((k_combine2<Src, 1, false>), grid, block, 0, st, s, level);
    else hipLaunchKernelGGL((k_combine2<Src, 0, false>), grid, block, 0, st, s, level);
    return hipGetLastError();
}
template <class Src>
hipError_t launch_combine(const Src& s, int level, int variant, int64_t blocks, hipStream_t st, bool peel) {
    const dim3 grid((unsigned)blocks), block(kStreamThreads);
    if (peel && variant) hipLaunchKernelGGL((k_combine<Src, 1, true>), grid, block, 0, st, s, level);
    else if (peel) hipLaunchKernelGGL((k_combine<Src, 0, true>), grid, block, 0, st, s, level);
    else if (variant) hipLaunchKernelGGL((k_combine<Src, 1, false>), grid, block, 0, st, s, level);
    else hipLaunchKernelGGL((k_combine<Src, 0, false>), grid, block, 0, st, s, level);
    return hipGetLastError();
}

template <class Src>
hipError_t launch_peel(const Src& s, int max_peel, int64_t blocks, hipStream_t st) {
    if (max_peel < 1 || max_peel > kPeelMaxResidue) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(kStreamThreads);
    if (max_peel <= 4) hipLaunchKernelGGL((k_peel<Src, 4>), grid, block, 0, st, s);
    else if (max_peel <= 16) hipLaunchKernelGGL((k_peel<Src, 16>), grid, block, 0, st, s);
    else hipLaunchKernelGGL((k_peel<Src, 64>), grid, block, 0, st, s);
    return hipGetLastError();
}

hipError_t launch_pack_blocks(const float* X, int64_t rows, int64_t cols, int64_t ld, float* dst, int64_t s,
                              hipStream_t st) {
    const int64_t nblocks = ((rows + s - 1) / s) * ((cols + s - 1) / s);
    const int64_t grid = (nblocks * (s * s / 4) + kStreamPerBlock - 1) / kStreamPerBlock;
    hipLaunchKernelGGL(k_pack_blocks, dim3((unsigned)grid), dim3(kStreamThreads), 0, st, X, rows, cols, ld, dst, s,
                       nblocks);
    return hipGetLastError();
}
hipError_t launch_reduce_blocks(const float* P, float* C, int64_t m, int64_t n, int64_t s, int64_t MB, int64_t NB,
                                int64_t KB, hipStream_t st) {
    const int64_t grid = (MB * NB * (s * s / 4) + kStreamPerBlock - 1) / kStreamPerBlock;
    hipLaunchKernelGGL(k_reduce_blocks, dim3((unsigned)grid), dim3(kStreamThreads), 0, st, P, C, m, n, s, MB, NB, KB);
    return hipGetLastError();
}

template hipError_t launch_pad<OneProb>(const OneProb&, int64_t, hipStream_t);
template hipError_t launch_pad<TableProb>(const TableProb&, int64_t, hipStream_t);
template hipError_t launch_absmax<OneProb>(const OneProb&, int64_t, hipStream_t);
template hipError_t launch_absmax<TableProb>(const TableProb&, int64_t, hipStream_t);
template hipError_t launch_scale_exp<OneProb>(const OneProb&, int64_t, hipStream_t);
template hipError_t launch_scale_exp<TableProb>(const TableProb&, int64_t, hipStream_t);
template hipError_t launch_divide<OneProb>(const OneProb&, int, int, int64_t, hipStream_t);
template hipError_t launch_divide<TableProb>(const TableProb&, int, int, int64_t, hipStream_t);
template hipError_t launch_split<OneProb>(const OneProb&, int, int, int64_t, hipStream_t);
template hipError_t launch_split<TableProb>(const TableProb&, int, int, int64_t, hipStream_t);
template hipError_t launch_combine<OneProb>(const OneProb&, int, int, int64_t, hipStream_t, bool);
template hipError_t launch_combine<TableProb>(const TableProb&, int, int, int64_t, hipStream_t, bool);
template hipError_t launch_combine2<OneProb>(const OneProb&, int, int, int64_t, hipStream_t, bool);
template hipError_t launch_combine2<TableProb>(const TableProb&, int, int, int64_t, hipStream_t, bool);
template hipError_t launch_peel<OneProb>(const OneProb&, int, int64_t, hipStream_t);
template hipError_t launch_peel<TableProb>(const TableProb&, int, int64_t, hipStream_t);

}  // namespace stk
