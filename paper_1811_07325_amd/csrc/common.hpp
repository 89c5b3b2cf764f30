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
    int64_t n;          // edge of the recursion's input: the user size, or
                        // the core of a peeled plan (n - peel)
    int64_t ldu;        // leading dimension of A, B and C (the user size)
    int peel;           // rows and columns peeled off the core (0: none)
    int64_t np;         // padded size (multiple of 2^depth * 64)
    int64_t leaf;       // np >> depth
    int depth;
    int planes;         // 0: binary32 leaves; 2 or 3: bf16 split planes
    int bounded0;       // level 0 reads A/B element by element with bounds
                        // (n != np, or a peeled plan: rows need not be
                        // 16-byte aligned)
    int gemm_tile;      // leaf tile edge (64 or 128)
    int64_t div_a[STK_MAXD], div_b[STK_MAXD];  // float offsets of divide outputs
    int div_slots[STK_MAXD];                   // 5 (views kept) or 7
    int64_t leaf_a, leaf_b;                    // uint16 offsets of split leaf operands
    int64_t leaf_m;                            // float offset of leaf products (-1: C)
    int64_t comb[STK_MAXD];                    // float offsets of combine outputs
    int64_t pad_a, pad_b;                      // float offsets of padded copies (-1)
    int fp16;                                  // leaf planes are binary16 (FP16X3)
    int64_t scale;                             // float offset of the FP16X3 scale region (-1)
    int variant;                               // 0: Algorithm 1, 1: Winograd's variant
};

constexpr int kScaleParts = 256;               // partial maxima per matrix (FP16X3)
constexpr int kPeelMaxResidue = 64;            // largest residue a plan peels

// Where the operand blocks of the seven products live after one divide step:
// a materialised slot index, or a view of the parent's quadrant X11 (-1),
// X22 (-2), X12 (-3) or X21 (-4).
// Algorithm 1, A side: S1=X11+X22, S2=X21+X22, S3=X11, S4=X22, S5=X11+X12,
// S6=X21-X11, S7=X12-X22 stored as slots [S1,S2,S5,S6,S7]; B side:
// T1=Y11+Y22, T2=Y11, T3=Y12-Y22, T4=Y21-Y11, T5=Y22, T6=Y11+Y12, T7=Y21+Y22
// stored as slots [T1,T3,T4,T6,T7].
// Winograd's variant, products M1..M7 = X11 Y11, X12 Y21, S4 Y22, X22 T4,
// S1 T1, S2 T2, S3 T3 with S1=X21+X22, S2=S1-X11, S3=X11-X21, S4=X12-S2,
// T1=Y12-Y11, T2=Y22-T1, T3=Y22-Y12, T4=T2-Y21, stored as slots
// [S1,S2,S3,S4] and [T1,T2,T3,T4].
__device__ __forceinline__ int slot_of(int side, int c, int variant) {
    // 4-bit field c holds the value + 4:
    //   A [0, 1, -1, -2, 2, 3, 4], B [0, -1, 1, 2, -2, 3, 4] (Algorithm 1),
    //   A [-1, -3, 3, -2, 0, 1, 2], B [-1, -4, -2, 3, 0, 1, 2] (Winograd)
    const uint32_t t = variant ? (side ? 0x6547203u : 0x6542713u) : (side ? 0x8726534u : 0x8762354u);
    return (int)((t >> (4 * c)) & 15u) - 4;
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
        ld = d.ldu;
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
        const int s = (slots == 7) ? c : slot_of(side, c, d.variant);
        if (s >= 0) {
            ptr = wsf + (side ? d.div_b[j] : d.div_a[j]) + (prefix * slots + s) * h * h;
            ld = h;
        } else if (s == -2) {
            ptr += h * ld + h;
        } else if (s == -3) {
            ptr += h;
        } else if (s == -4) {
            ptr += h * ld;
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
