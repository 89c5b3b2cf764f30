// Device-side descriptors shared by every kernel of the Strassen hot path.
//
// One multiply ("problem") is described by a ProbDesc: user pointers, sizes
// and the element offsets of every workspace region.  Recursion nodes are
// numbered the way the paper tags blocks with an M-index (Section III-B,
// Algorithm 5): the children of node `id` at level l are 7*id + c at level
// l+1, c = 0..6 standing for M1..M7, so a node's parent is id / 7 and its
// base-7 digits spell the path from the root.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define STK_MAXD 8

namespace stk {

struct ProbDesc {
    const float* A;     // user operands (row-major, leading dimension n)
    const float* B;
    float* C;
    char* ws;           // workspace base
    int64_t n;          // user size
    int64_t np;         // padded size (multiple of 2^depth * 64)
    int64_t leaf;       // np >> depth
    int depth;
    int planes;         // 0: binary32 leaves; 2 or 3: bf16 split planes
    int bounded0;       // level 0 reads A/B with bounds (n != np)
    int gemm_tile;      // leaf tile edge (64 or 128)
    int64_t div_a[STK_MAXD], div_b[STK_MAXD];  // float offsets of divide outputs
    int div_slots[STK_MAXD];                   // 5 (views kept) or 7
    int64_t leaf_a, leaf_b;                    // uint16 offsets of split leaf operands
    int64_t leaf_m;                            // float offset of leaf products (-1: C)
    int64_t comb[STK_MAXD];                    // float offsets of combine outputs
    int64_t pad_a, pad_b;                      // float offsets of padded copies (-1)
    int fp16;                                  // leaf planes are binary16 (FP16X3)
    int64_t scale;                             // float offset of the FP16X3 scale region (-1)
};

constexpr int kScaleParts = 256;               // partial maxima per matrix (FP16X3)

// Where the operand blocks of the seven products live after one divide step
// (Algorithm 1): a materialised slot index, or a view of the parent's
// quadrant X11 (-1) / X22 (-2).  A side: S1=X11+X22, S2=X21+X22, S3=X11,
// S4=X22, S5=X11+X12, S6=X21-X11, S7=X12-X22 stored as slots [S1,S2,S5,S6,S7].
// B side: T1=Y11+Y22, T2=Y11, T3=Y12-Y22, T4=Y21-Y11, T5=Y22, T6=Y11+Y12,
// T7=Y21+Y22 stored as slots [T1,T3,T4,T6,T7].
__device__ __forceinline__ int slot_of(int side, int c) {
    // packed 3-bit fields: value+2 so views -2,-1 map to 0,1
    const uint32_t a = (2u) | (3u << 3) | (1u << 6) | (0u << 9) | (4u << 12) | (5u << 15) | (6u << 18);
    const uint32_t b = (2u) | (1u << 3) | (3u << 6) | (4u << 9) | (0u << 12) | (5u << 15) | (6u << 18);
    const uint32_t t = side ? b : a;
    return (int)((t >> (3 * c)) & 7u) - 2;
}

// Resolve the binary32 operand (pointer, leading dimension) of node `id` at
// recursion level `level` on side 0 (A) or 1 (B) by walking its base-7 digits
// from the root.
__device__ __forceinline__ void resolve(const ProbDesc& d, int side, int level, int64_t id,
                                        const float*& ptr, int64_t& ld) {
    const float* wsf = reinterpret_cast<const float*>(d.ws);
    if (d.pad_a >= 0) {
        ptr = wsf + (side ? d.pad_b : d.pad_a);
        ld = d.np;
    } else {
        ptr = side ? d.B : d.A;
        ld = d.n;
    }
    int64_t pw = 1;
    for (int j = 1; j < level; ++j) pw *= 7;
    int64_t prefix = 0;
    int64_t m = d.np;
    for (int j = 0; j < level; ++j) {
        const int c = (int)((id / pw) % 7);
        pw /= 7;
        const int64_t h = m >> 1;
        const int slots = d.div_slots[j];
        if (slots == 0) {   // level j is not stored: level j+1 stores all seven operands
            prefix = prefix * 7 + c;
            m = h;
            continue;
        }
        const int s = (slots == 7) ? c : slot_of(side, c);
        if (s >= 0) {
            ptr = wsf + (side ? d.div_b[j] : d.div_a[j]) + (prefix * slots + s) * h * h;
            ld = h;
        } else if (s == -2) {
            ptr += h * ld + h;
        }
        prefix = prefix * 7 + c;
        m = h;
    }
}

// Layout of a bf16 leaf-operand plane (edge L, "rows" = the A rows or the B
// columns, "k" = the contraction index).  The plane is cut into 1 KB blocks
// of kBlkRows rows x kBlkK k, stored block-row-major: block (r/kBlkRows,
// k/kBlkK) at ((r/kBlkRows) * (L/kBlkK) + k/kBlkK) * 512 elements.  Inside a
// block, row r holds kBlkK/8 chunks of 8 k; chunk c is stored at position
// c ^ blk_swz(r) of the row.  The swizzle makes the LDS reads of MFMA
// operands (one chunk of consecutive rows) hit distinct bank groups for both
// 8- and 16-lane LDS phases, and a block is copied to LDS unchanged, so one
// 64-lane 16-byte load moves one contiguous block.
constexpr int kBlkRows = 16;
constexpr int kBlkK = 512 / kBlkRows;    // 32
constexpr int kBlkChunks = kBlkK / 8;     // 4

__device__ __forceinline__ int blk_swz(int row) { return ((row >> 1) & 3) ^ ((row >> 3) & 1); }

__device__ __forceinline__ int64_t blk_offset(int64_t r, int64_t k, int64_t L) {
    const int rr = (int)(r % kBlkRows);
    const int c = (int)((k >> 3) % kBlkChunks);
    return ((r / kBlkRows) * (L / kBlkK) + k / kBlkK) * 512 + ((rr * kBlkChunks + (c ^ blk_swz(rr))) << 3) + (k & 7);
}

// Block b of a G-block grid -> its logical index.  Consecutive blocks go to
// different XCDs (b mod 8); when G is a multiple of 8 the remap gives the G/8
// blocks of XCD x the logical indices [x*G/8, (x+1)*G/8), so work items with
// neighbouring logical indices share that XCD's L2.
__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t G) {
    if (G % 8) return b;
    return (b % 8) * (G / 8) + b / 8;
}

// A launch covers one problem (kernel-argument descriptor) or many (device
// table).  `first_block` holds, per problem, the first block index of this
// launch that belongs to it (ascending, first_block[0] == 0).
struct OneProb {
    ProbDesc d;
    __device__ __forceinline__ const ProbDesc& get(int) const { return d; }
    // Problem owning block `blk` of this launch and the block's index within it.
    __device__ __forceinline__ int locate(int64_t blk, int64_t& local) const {
        local = blk;
        return 0;
    }
};

struct TableProb {
    const ProbDesc* table;
    const int64_t* first_block;  // per-launch prefix, nprob + 1 entries
    int nprob;
    __device__ __forceinline__ const ProbDesc& get(int p) const { return table[p]; }
    __device__ __forceinline__ int locate(int64_t blk, int64_t& local) const {
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first_block[mid] <= blk) lo = mid; else hi = mid - 1;
        }
        local = blk - first_block[lo];
        return lo;
    }
};

}  // namespace stk
