// Leaf products of the Strassen recursion (Section III-C-2, Algorithm 4):
// one persistent, grouped launch multiplies every leaf pair M_id = S_id T_id
// (7^depth of them per problem, all problems of a batch) on the matrix cores.
//
//  k_gemm_f32_big / _mid / _small
//                    binary32 operands read in place (views included), MFMA
//                    v_mfma_f32_16x16x4_f32, binary32 accumulation; one
//                    kernel body (gemm32_lds) with 256-, 128- and 64-wide
//                    tiles, operand tiles copied from global memory straight
//                    into LDS.
//  k_gemm_bf16_big / _mid / _small
//                    operands pre-split into P 16-bit planes (blocked layout
//                    of blk_offset; B transposed so both are k-contiguous),
//                    MFMA v_mfma_f32_16x16x32_bf16 (or _f16) over the cross
//                    products of the planes whose magnitude matters, binary32
//                    accumulation; one kernel body (gemm16_lds) with 256-,
//                    128- and 64-wide tiles, operand tiles copied from global
//                    memory straight into LDS.
// Tile order is static (no atomics, no split-K): tile t of the grid-stride
// loop is remapped so that the blocks of one XCD (blockIdx mod 8) work on
// consecutive tiles, and tiles inside a leaf are visited in groups of 8 tile
// rows so the A and B panels in flight are shared through that XCD's L2.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace stk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// 16-bit operand flavour of the split leaf GEMMs: bfloat16 (BF16X3/X6) or
// binary16 (FP16X3), both on the 16x16x32 matrix-core instruction.
template <bool F16> struct Op16;
template <> struct Op16<false> {
    using T = bf16x8;
    static __device__ __forceinline__ f32x4 mfma(T a, T b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Op16<true> {
    using T = f16x8;
    static __device__ __forceinline__ f32x4 mfma(T a, T b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Factors 2^-e_A and 2^-e_B that undo the FP16X3 operand scaling (exact
// powers of two; applied one after the other, so each stays a finite binary32
// whatever the sum e_A + e_B).
struct Unscale {
    float a, b;
    __device__ __forceinline__ float operator()(float x) const { return x * a * b; }
};
__device__ __forceinline__ Unscale unscale_of(const ProbDesc& d) {
    if (!d.fp16) return Unscale{1.0f, 1.0f};
    const int* ex = reinterpret_cast<const int*>(reinterpret_cast<const float*>(d.ws) + d.scale) + 2 * kScaleParts;
    return Unscale{ldexpf(1.0f, -ex[0]), ldexpf(1.0f, -ex[1])};
}

constexpr int kGroupRows = 8;

// Tile coordinates of logical tile `r` of a leaf with tm_cnt x tn_cnt tiles,
// visiting groups of kGroupRows tile rows column by column.
__device__ __forceinline__ void tile_coords(int64_t r, int64_t tm_cnt, int64_t tn_cnt, int64_t& tm,
                                            int64_t& tn) {
    const int64_t per_group = (int64_t)kGroupRows * tn_cnt;
    const int64_t g = r / per_group;
    const int64_t first = g * kGroupRows;
    const int64_t rows = (tm_cnt - first) < kGroupRows ? (tm_cnt - first) : kGroupRows;
    const int64_t in = r - g * per_group;
    tm = first + in % rows;
    tn = in / rows;
}

// ---------------------------------------------------------------------------
// binary32 leaf GEMM.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// bf16-split leaf GEMM.  Planes p = 0 (hi), 1 (mid), 2 (lo).  The products
// kept are those of magnitude >= 2^-16 relative to hi*hi; they are issued
// smallest first into one binary32 accumulator.
// ---------------------------------------------------------------------------
template <int P>
struct SplitProducts;
template <>
struct SplitProducts<2> {
    static constexpr int count = 3;
    __device__ static constexpr int a(int q) { return q == 0 ? 1 : 0; }
    __device__ static constexpr int b(int q) { return q == 1 ? 1 : 0; }
};
template <>
struct SplitProducts<3> {
    // (mid,mid), (lo,hi), (hi,lo), (mid,hi), (hi,mid), (hi,hi)
    static constexpr int count = 6;
    __device__ static constexpr int a(int q) {
        return q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 0 : q == 3 ? 1 : 0;
    }
    __device__ static constexpr int b(int q) {
        return q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0;
    }
};

// LDS address space pointer of the direct global->LDS loads.
typedef __attribute__((address_space(3))) void lds_void_t;

// Configuration of the large-leaf kernel: block tile, wave grid and LDS
// stages per precision.  Measured alternatives (same kernel): 4 waves of
// 128 x 128, 256 x 128 or 128 x 128 tiles with 3-4 stages, and a 32 x 32 x 16
// MFMA variant with 16-wide K steps and 3-5 stages were all slower for P = 2.
template <int BM_, int BN_, int WAVES_M_, int WAVES_N_, int STAGES_>
struct BigCfgT {
    static constexpr int BM = BM_, BN = BN_, WAVES_M = WAVES_M_, WAVES_N = WAVES_N_, STAGES = STAGES_;
    static constexpr int NW = WAVES_M * WAVES_N, NT = 64 * NW;
};
template <int P> struct BigCfg;
template <> struct BigCfg<2> : BigCfgT<256, 256, 2, 4, 2> {};   // 8 waves of 128 x 64, 128 KB LDS
template <> struct BigCfg<3> : BigCfgT<256, 128, 4, 2, 2> {};   // 8 waves of 64 x 64, 144 KB LDS
// 128 x 128 and 64 x 64 tiles (leaves too small to fill the chip with
// 256-wide tiles): 4 waves of 64 x 64 / 32 x 32, two stages (64 / 32 KB for
// P = 2), two or more blocks per CU.  Three stages were slower for 128 x 128.
template <int P> struct MidCfg : BigCfgT<128, 128, 2, 2, 2> {};
template <int P> struct SmallCfg : BigCfgT<64, 64, 2, 2, 2> {};

// Wait until at most N of this wave's vector-memory operations are pending.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// LDS stages of step k and of step k + STAGES - 1 (the one refilled while
// step k is read).  With two stages the indices are k & 1 and (k & 1) ^ 1,
// a form the compiler's alias analysis can tell apart: it then does not make
// the LDS reads of step k wait for the copies into the other stage it has
// just issued (with k % 3 and (k + 2) % 3 it cannot, and waits for them --
// the whole load latency, every step).
template <int STAGES>
__device__ __forceinline__ int stage_of(int64_t k) {
    if constexpr (STAGES == 2) return (int)(k & 1);
    else return (int)(k % STAGES);
}
template <int STAGES>
__device__ __forceinline__ int refill_stage_of(int64_t k) {
    if constexpr (STAGES == 2) return (int)(k & 1) ^ 1;
    else return (int)((k + STAGES - 1) % STAGES);
}

// Workgroup barrier between LDS stages of a pipelined K loop: this wave's
// LDS reads have completed, then a bare s_barrier.  __syncthreads() would add
// a workgroup memory fence, which waits for every vector-memory operation of
// the wave -- the direct copies of the later stages, still in flight, too --
// and so shortens the pipeline to one stage of look-ahead.  The caller waits
// for the copies of the stage about to be read (wait_vmcnt) before this.
// The memory clobbers and scheduling barriers keep every LDS access on its
// side of the barrier.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// bf16-split leaf GEMM for large leaves.  Operand tiles go from global
// memory straight into LDS (global_load_lds_dwordx4: each lane deposits 16
// bytes at LDS base + 16 * lane), STAGES deep: while step k runs on the
// matrix cores the loads of steps k+1 .. k+STAGES-1 are in flight, with no
// register staging.  The LDS image of a stage is [plane][row][4 chunks of 8
// bf16], A rows first, then B rows, chunks swizzled by blk_swz -- the same image
// as the operands' blocked layout in HBM (blk_offset), so each load copies a
// contiguous 1 KB block.
// ---------------------------------------------------------------------------
template <class Cfg, class Src, int P, bool F16>
__device__ __forceinline__ void gemm16_lds(Src src, int64_t total_tiles) {
    using VT = typename Op16<F16>::T;
    constexpr int BM = Cfg::BM, BN = Cfg::BN, NW = Cfg::NW, STAGES = Cfg::STAGES;
    constexpr int WAVES_N = Cfg::WAVES_N;
    constexpr int BK = 32, KC = BK / 8;                 // 16-byte chunks per row and plane
    constexpr int ROWS = BM + BN;                       // LDS rows per plane (A rows, then B rows)
    constexpr int UNITS = P * ROWS * KC;                // 16-byte units per stage
    constexpr int GA = BM / 16, GB = BN / 16;           // 16-row groups per side
    static_assert(GA % NW == 0 && GB % NW == 0, "groups must split evenly over the waves");
    static_assert(kBlkRows == 16 && kBlkK == BK, "operand layout must match the K step");
    constexpr int LPS = P * (GA + GB) / NW;             // direct loads per lane per stage
    constexpr int WM = BM / Cfg::WAVES_M, WN = BN / WAVES_N, TM = WM / 16, TN = WN / 16;
    __shared__ __attribute__((aligned(16))) uint4 lds[STAGES][UNITS];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WAVES_N, wn = w % WAVES_N;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t G = gridDim.x;
    const int64_t slot = xcd_slot(blockIdx.x, G);

    for (int64_t t = slot; t < total_tiles; t += G) {
        int64_t local;
        const ProbDesc& d = src.get(src.locate(t, local));
        const int64_t L = d.leaf, LL = L * L;
        const int64_t tm_cnt = L / BM, tn_cnt = L / BN, tpl = tm_cnt * tn_cnt;
        const int64_t leaf = local / tpl;
        int64_t tm, tn;
        tile_coords(local - leaf * tpl, tm_cnt, tn_cnt, tm, tn);
        const uint16_t* Ah = reinterpret_cast<const uint16_t*>(d.ws) + d.leaf_a + leaf * P * LL;
        const uint16_t* Bh = reinterpret_cast<const uint16_t*>(d.ws) + d.leaf_b + leaf * P * LL;
        float* Cp;
        int64_t ldc;
        if (d.depth == 0) { Cp = d.C; ldc = d.ldu; }
        else { Cp = reinterpret_cast<float*>(d.ws) + d.leaf_m + leaf * LL; ldc = L; }
        const bool crop = d.depth == 0 && d.bounded0;
        const Unscale unscale = unscale_of(d);
        const int64_t m0 = tm * BM, n0 = tn * BN;

        // One direct load of a wave moves one 1 KB block of the blocked
        // operand layout (16 rows x 32 k, chunks already swizzled) into 64
        // consecutive LDS units.  Block row g of a side (rows 16g..16g+15) of
        // plane p is loaded by wave g % NW; lane l moves bytes 16l..16l+15.
        const int64_t blocks_k = L >> 5;                  // blocks per block row
        const uint16_t* a_src = Ah + ((m0 >> 4) * blocks_k << 9) + 8 * lane;
        const uint16_t* b_src = Bh + ((n0 >> 4) * blocks_k << 9) + 8 * lane;
        auto issue = [&](int stage, int64_t k0) {
            const int64_t kb = (k0 >> 5) << 9;
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int r = 0; r < GA / NW; ++r) {
                    const int g = w + NW * r;
                    __builtin_amdgcn_global_load_lds(a_src + p * LL + ((int64_t)g * blocks_k << 9) + kb,
                                                     (lds_void_t*)&lds[stage][(p * ROWS + 16 * g) * KC], 16, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < GB / NW; ++r) {
                    const int g = w + NW * r;
                    __builtin_amdgcn_global_load_lds(b_src + p * LL + ((int64_t)g * blocks_k << 9) + kb,
                                                     (lds_void_t*)&lds[stage][(p * ROWS + BM + 16 * g) * KC], 16, 0,
                                                     0);
                }
            }
        };

        f32x4 acc[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

        const int64_t KT = L / BK;
#pragma unroll
        for (int s = 0; s < STAGES - 1; ++s)
            if (s < KT) issue(s, s * BK);
        for (int64_t kt = 0; kt < KT; ++kt) {
            // step kt has landed once at most the loads of the later steps
            // already issued (up to STAGES-2 of them) are pending
            if (kt + STAGES - 2 < KT) wait_vmcnt<LPS * (STAGES - 2)>();
            else wait_vmcnt<0>();
            __syncthreads();     // every wave's part of step kt landed; step kt-1's reads are done
            // three planes: the compiler's DS / MFMA interleaving strategy 1
            // (measured 4 % faster there, 3 % slower with two planes)
            if constexpr (P == 3) __builtin_amdgcn_iglp_opt(1);
            // Every fragment of the step is read before the copies of a later
            // step are issued: the compiler cannot tell the stages apart and
            // makes LDS reads wait for every copy issued before them, which
            // would stall each step for the whole latency of its new copies.
            const uint4* sl = lds[stage_of<STAGES>(kt)];
            VT b[P][TN], a[TM][P];
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int row = BM + wn * WN + 16 * j + li;
                    b[p][j] = __builtin_bit_cast(VT, sl[(p * ROWS + row) * KC + (lg ^ blk_swz(row))]);
                }
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = wm * WM + 16 * i + li;
#pragma unroll
                for (int p = 0; p < P; ++p)
                    a[i][p] = __builtin_bit_cast(VT, sl[(p * ROWS + row) * KC + (lg ^ blk_swz(row))]);
            }
            if (kt + STAGES - 1 < KT) issue(refill_stage_of<STAGES>(kt), (kt + STAGES - 1) * BK);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int q = 0; q < SplitProducts<P>::count; ++q)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = Op16<F16>::mfma(a[i][SplitProducts<P>::a(q)], b[SplitProducts<P>::b(q)][j],
                                                    acc[i][j]);
        }
        __syncthreads();         // the next tile's first loads overwrite the stages

#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + wm * WM + 16 * i + 4 * lg + r;
                    const int64_t col = n0 + wn * WN + 16 * j + li;
                    if (!crop || (row < d.n && col < d.n)) Cp[row * ldc + col] = unscale(acc[i][j][r]);
                }
    }
}


// ---------------------------------------------------------------------------
// Two-plane, 256 x 256 leaf GEMM with the eight waves in two groups that
// take turns on the matrix cores ("ping-pong").  Group g = w / 4 owns output
// rows 128 g .. 128 g + 127 and holds one wave on each SIMD (waves w and
// w + 4 share a SIMD).  A K step of a group is two phases separated by
// workgroup barriers: a read phase (all operand fragments of the step from
// LDS into registers) and a compute phase (its 96 MFMAs from registers).
// Group 1 runs one phase behind group 0, so while one wave of a SIMD issues
// MFMAs the other reads LDS and issues the global->LDS copies: the matrix
// core does not wait for LDS reads at step boundaries.  LDS holds two
// stages; stage s of step k is read in phases 2k (group 0) and 2k + 1
// (group 1), so the copies of step k + 1 are issued in phase 2k, when its
// stage (that of step k - 1) is free, and waited for before phase 2k + 2;
// group 0 issues all of them, so both groups run the same loop.
// Each output accumulates the same MFMAs in the same order as gemm16_lds, so
// both give identical results.
// ---------------------------------------------------------------------------
// A wave-uniform address held in scalar registers: readfirstlane is opaque
// to the compiler, so a per-lane offset added afterwards stays a 32-bit
// vector offset (the load's scalar-base form) instead of the compiler
// hoisting (uniform part + lane part) of every load into vector registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ const char* scalar_ptr(const void* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const char*>(((uint64_t)hi << 32) | lo);
}

#ifndef STK_PINGPONG
#define STK_PINGPONG 1
#endif

template <class Src, int P, bool F16>
__device__ __forceinline__ void gemm16_pingpong(Src src, int64_t total_tiles) {
    using VT = typename Op16<F16>::T;
    using Cfg = BigCfg<P>;
    constexpr int BM = Cfg::BM, BN = Cfg::BN, NW = Cfg::NW, WAVES_N = Cfg::WAVES_N;
    static_assert(Cfg::STAGES == 2 && NW == 8 && Cfg::WAVES_M % 2 == 0, "two groups of four waves, two stages");
    constexpr int BK = 32, KC = BK / 8;
    constexpr int ROWS = BM + BN;
    constexpr int UNITS = P * ROWS * KC;
    constexpr int GA = BM / 16, GB = BN / 16;
    static_assert(kBlkRows == 16 && kBlkK == BK, "operand layout must match the K step");
    constexpr int WM = BM / Cfg::WAVES_M, WN = BN / WAVES_N, TM = WM / 16, TN = WN / 16;
    __shared__ __attribute__((aligned(16))) uint4 lds[2][UNITS];

    // the wave index is uniform across a wave: readfirstlane lets the
    // compiler keep it, and the copies' base addresses, in scalar registers
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // group = upper or lower half of the tile's wave rows; waves w and
    // w + 4 share a SIMD and sit in different groups
    const int wm = w / WAVES_N, wn = w % WAVES_N, grp = w / (NW / 2);
    const int li = lane & 15, lg = lane >> 4;
    const int64_t G = gridDim.x;
    const int64_t slot = xcd_slot(blockIdx.x, G);

    for (int64_t t = slot; t < total_tiles; t += G) {
        // Everything a tile's K loop needs is uniform across the workgroup.
        // Read from a device problem table it would land in vector
        // registers, beside the accumulators and fragments, so there it is
        // moved to scalar registers first and the epilogue's values are
        // read after the loop (a kernel-argument descriptor is scalar
        // already).
        constexpr bool kTable = !std::is_same<Src, OneProb>::value;
        auto uni = [](int64_t v) { return kTable ? uniform64(v) : v; };
        int64_t local;
        int pi = src.locate(t, local);
        if constexpr (kTable) pi = __builtin_amdgcn_readfirstlane(pi);
        local = uni(local);
        const ProbDesc& d = src.get(pi);
        const int64_t L = uni(d.leaf), LL = L * L;
        const int64_t tm_cnt = L / BM, tn_cnt = L / BN, tpl = tm_cnt * tn_cnt;
        const int64_t leaf = local / tpl;
        int64_t tm, tn;
        tile_coords(local - leaf * tpl, tm_cnt, tn_cnt, tm, tn);
        const uint16_t* ws16 = reinterpret_cast<const uint16_t*>(kTable ? scalar_ptr(d.ws) : d.ws);
        const uint16_t* Ah = ws16 + uni(d.leaf_a) + leaf * P * LL;
        const uint16_t* Bh = ws16 + uni(d.leaf_b) + leaf * P * LL;
        const int64_t m0 = tm * BM, n0 = tn * BN;
        float* Cp;
        int64_t ldc;
        bool crop;
        Unscale unscale;
        auto epilogue_args = [&] {
            if (d.depth == 0) { Cp = d.C; ldc = d.ldu; }
            else { Cp = reinterpret_cast<float*>(d.ws) + d.leaf_m + leaf * LL; ldc = L; }
            crop = d.depth == 0 && d.bounded0;
            unscale = unscale_of(d);
        };
        if constexpr (!kTable) epilogue_args();

        // direct copies, as in gemm16_lds, by the four waves of group 0:
        // block row g of a side of plane p (one contiguous 1 KB block per K
        // step) is moved by wave g % 4
        constexpr int NL = NW / 2;
        const int64_t blocks_k = L >> 5;
        const uint16_t* a_blk = Ah + ((m0 >> 4) * blocks_k << 9);
        const uint16_t* b_blk = Bh + ((n0 >> 4) * blocks_k << 9);
        const uint32_t lane_bytes = 16 * lane;
        auto issue = [&](int stage, int64_t k0) {
            const int64_t kb = (k0 >> 5) << 9;
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int r = 0; r < GA / NL; ++r) {
                    const int g = w + NL * r;
                    __builtin_amdgcn_global_load_lds(
                        scalar_ptr(a_blk + p * LL + ((int64_t)g * blocks_k << 9) + kb) + lane_bytes,
                        (lds_void_t*)&lds[stage][(p * ROWS + 16 * g) * KC], 16, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < GB / NL; ++r) {
                    const int g = w + NL * r;
                    __builtin_amdgcn_global_load_lds(
                        scalar_ptr(b_blk + p * LL + ((int64_t)g * blocks_k << 9) + kb) + lane_bytes,
                        (lds_void_t*)&lds[stage][(p * ROWS + BM + 16 * g) * KC], 16, 0, 0);
                }
            }
        };


        f32x4 acc[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        VT a[TM][P], b[TN][P];

        // read phase: every fragment of step kt into registers
        auto read_frags = [&](int64_t kt) {
            const uint4* sl = lds[kt & 1];
#pragma unroll
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int row = BM + wn * WN + 16 * j + li;
                    b[j][p] = __builtin_bit_cast(VT, sl[(p * ROWS + row) * KC + (lg ^ blk_swz(row))]);
                }
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int row = wm * WM + 16 * i + li;
                    a[i][p] = __builtin_bit_cast(VT, sl[(p * ROWS + row) * KC + (lg ^ blk_swz(row))]);
                }
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the stage may be refilled two phases on
        };
        // compute phase: the step's MFMAs, in the order of gemm16_lds
        auto compute = [&] {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int q = 0; q < SplitProducts<P>::count; ++q)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = Op16<F16>::mfma(a[i][SplitProducts<P>::a(q)], b[j][SplitProducts<P>::b(q)],
                                                    acc[i][j]);
        };
        // Phase boundary: a bare workgroup barrier (no memory fence, which
        // would wait for the copies in flight), nothing scheduled across it.
        // Every LDS read before it has completed (read_frags waits), and a
        // stage's copies are waited for explicitly before the barrier that
        // precedes its first read.
        auto boundary = [] {
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
        };

        const int64_t KT = L / BK;
        // Group 0 moves every operand block (16 copies per wave and step),
        // group 1 none, so the two groups run the same loop; group 1 enters
        // it one phase later (one extra barrier before, one fewer after).
        if (grp == 0) {
            issue(0, 0);
            wait_vmcnt<0>();
        }
        boundary();
        if (grp == 1) boundary();
        for (int64_t kt = 0; kt < KT; ++kt) {
            // group 0: phase 2 kt (group 1 computes step kt - 1 meanwhile)
            if (grp == 0 && kt + 1 < KT) issue((int)((kt + 1) & 1), (kt + 1) * BK);
            read_frags(kt);
            boundary();
            // group 0: phase 2 kt + 1 (group 1 reads step kt meanwhile)
            compute();
            if (grp == 0) wait_vmcnt<0>();                     // step kt + 1 is in LDS
            boundary();
        }
        if (grp == 0) boundary();                               // phase 2 KT: group 1 computes step KT - 1

        if constexpr (kTable) epilogue_args();
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + wm * WM + 16 * i + 4 * lg + r;
                    const int64_t col = n0 + wn * WN + 16 * j + li;
                    if (!crop || (row < d.n && col < d.n)) Cp[row * ldc + col] = unscale(acc[i][j][r]);
                }
    }
}


template <class Src, int P, bool F16>
__global__ __launch_bounds__(BigCfg<P>::NT) void k_gemm_bf16_big(Src src, int64_t total_tiles) {
    // the ping-pong kernel for single problems and problem tables alike
    // (its tile set-up lives in scalar registers)
    if constexpr (STK_PINGPONG)
        gemm16_pingpong<Src, P, F16>(src, total_tiles);
    else
        gemm16_lds<BigCfg<P>, Src, P, F16>(src, total_tiles);
}
template <class Src, int P, bool F16>
__global__ __launch_bounds__(MidCfg<P>::NT) void k_gemm_bf16_mid(Src src, int64_t total_tiles) {
    gemm16_lds<MidCfg<P>, Src, P, F16>(src, total_tiles);
}
template <class Src, int P, bool F16>
__global__ __launch_bounds__(SmallCfg<P>::NT) void k_gemm_bf16_small(Src src, int64_t total_tiles) {
    gemm16_lds<SmallCfg<P>, Src, P, F16>(src, total_tiles);
}

// ---------------------------------------------------------------------------
// binary32 leaf GEMM: BM x BN block tile (256 x 256 with 8 waves of 128 x 64
// for large leaves; 128 x 128 or 64 x 64 with 4 waves otherwise), K steps of
// 16, LDS stages filled by direct global->LDS loads straight from the
// binary32 operands (views included: leading dimension from the recursion),
// no register staging.  The 256-wide tile meets its waves at one barrier
// per two K steps (four stages of 32 KB, two groups of two); the smaller
// tiles at one per step (two stages).  Measured for the 256-wide tile at
// n = 16384: two steps per barrier 41.9 ms (depth 3) and 62.3 ms (depth 0);
// one step per barrier with two stages 43.0 / 62.7, three 45.1 / 65.7,
// four 44.1 / 64.5; for the 128-wide tile at n = 2048, depth 1: two stages
// 0.154 ms, three 0.164, four 0.153.
//   A stage image: [BM rows][4 chunks of 4 k], chunk position c ^ blk_swz(row
//     mod 16) (as the 16-bit blocked layout), one load = one 16-row block.
//   B stage image: [16 k][BN/4 chunks of 4 n], chunk position c ^ f32_bswz(k),
//     one load = 256 / BN consecutive k-rows.
// The permutation is applied on the global side (lane l fetches the chunk
// that belongs at LDS unit l), so both MFMA operand reads are bank-conflict
// free.  MFMA s of a step gives lane group g the k = 4g + s, so every tile
// size accumulates each output in the same order (ascending k) and gives the
// same result.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int f32_bswz(int k) { return ((k >> 2) & 1) << 2; }

constexpr int kF32BigThreads = 512;

template <int BM_, int BN_, int WAVES_M_, int WAVES_N_, int STAGES_, int SPB_ = 1>
struct F32CfgT {
    static constexpr int BM = BM_, BN = BN_, WAVES_M = WAVES_M_, WAVES_N = WAVES_N_, STAGES = STAGES_;
    static constexpr int SPB = SPB_;                   // K steps per barrier
    static constexpr int NW = WAVES_M * WAVES_N, NT = 64 * NW;
};
#ifndef STK_F32_STAGES
#define STK_F32_STAGES 2
#endif
#ifndef STK_F32_SMALL_STAGES
#define STK_F32_SMALL_STAGES 2
#endif
#ifndef STK_F32_SPB
#define STK_F32_SPB 2
#endif
#ifndef STK_F32_MID_SPB
#define STK_F32_MID_SPB 1
#endif
using F32BigCfg = F32CfgT<256, 256, 2, 4, STK_F32_SPB == 1 ? STK_F32_STAGES : 2 * STK_F32_SPB,
                          STK_F32_SPB>;   // 8 waves of 128 x 64, 32 KB LDS per stage
using F32FusedCfg = F32CfgT<256, 256, 2, 4, 2>;  // the same with fused leaf operands, 128 KB LDS
using F32MidCfg = F32CfgT<128, 128, 2, 2, STK_F32_MID_SPB == 1 ? STK_F32_SMALL_STAGES : 2 * STK_F32_MID_SPB,
                          STK_F32_MID_SPB>;    // 4 waves of 64 x 64, 16 KB per stage
using F32SmallCfg = F32CfgT<64, 64, 2, 2, STK_F32_SMALL_STAGES>;    // 4 waves of 32 x 32, 8 KB per stage
static_assert(F32BigCfg::NT == kF32BigThreads, "thread count of the 256-wide kernel");

// Leaf operand of leaf `leaf` formed inside the binary32 leaf GEMM (plans
// with fused leaves): the leaf is child c = leaf mod 7 of the level-(depth-1)
// node leaf / 7, whose operand X (edge 2L, stored by the divide or a view)
// has quadrants X11, X12, X21, X22 at offsets 0, L, L ld, L ld + L.  The
// operand is X_q1 (views S3, S4, T2, T5) or X_q1 + X_q2 or X_q1 - X_q2 -- the
// sums of Algorithm 1 in the order k_divide forms them, so each element is
// the same binary32 add and the product is bit-identical to the one of the
// materialised operand.  p2 = nullptr for a view; neg is the sign bit to
// flip on the second term (x + (-y) is x - y exactly).
__device__ __forceinline__ void fused_operand(const ProbDesc& d, int side, int64_t leaf, const float*& p1,
                                              const float*& p2, int64_t& ld, uint32_t& neg) {
    const float* X;
    resolve(d, side, d.depth - 1, leaf / 7, X, ld);
    const int c = (int)(leaf % 7);
    // per child: 4-bit fields q1 | q2 << 2 | two << 4 | minus << 5 (quadrant q: 0 X11, 1 X12, 2 X21, 3 X22)
    //   A: S1 = X11+X22, S2 = X21+X22, S3 = X11, S4 = X22, S5 = X11+X12, S6 = X21-X11, S7 = X12-X22
    //   B: T1 = Y11+Y22, T2 = Y11, T3 = Y12-Y22, T4 = Y21-Y11, T5 = Y22, T6 = Y11+Y12, T7 = Y21+Y22
    constexpr uint8_t kA[7] = {0 | 3 << 2 | 16, 2 | 3 << 2 | 16, 0, 3, 0 | 1 << 2 | 16, 2 | 0 << 2 | 48,
                               1 | 3 << 2 | 48};
    constexpr uint8_t kB[7] = {0 | 3 << 2 | 16, 0, 1 | 3 << 2 | 48, 2 | 0 << 2 | 48, 3, 0 | 1 << 2 | 16,
                               2 | 3 << 2 | 16};
    const int code = side ? kB[c] : kA[c];
    const int64_t L = d.leaf;
    auto quad = [&](int q) { return X + (q >> 1) * L * ld + (q & 1) * L; };
    p1 = quad(code & 3);
    p2 = (code & 16) ? quad((code >> 2) & 3) : nullptr;
    neg = (code & 32) ? 0x80000000u : 0u;
}

__device__ __forceinline__ float flip_add(float a, float b, uint32_t neg) {
    return a + __uint_as_float(__float_as_uint(b) ^ neg);
}
__device__ __forceinline__ float4 flip_add(float4 a, float4 b, uint32_t neg) {
    return make_float4(flip_add(a.x, b.x, neg), flip_add(a.y, b.y, neg), flip_add(a.z, b.z, neg),
                       flip_add(a.w, b.w, neg));
}

// One B load of a wave moves 256 consecutive floats of the stage image: 256 /
// BN k-rows (lane l: k-row l / (BN / 4), chunk l % (BN / 4)).
// FUSE: the leaf operands are formed from the level above (fused_operand):
// a stage holds both terms of each side, [A1][A2][B1][B2], both copied by
// direct loads, and the operand reads add them -- once per fragment read, a
// few adds per matrix-core instruction (16x16x4 binary32 MFMAs are long).
template <class Cfg, class Src, bool FUSE>
__device__ __forceinline__ void gemm32_lds(Src src, int64_t total_tiles) {
    constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = 16, NW = Cfg::NW, WAVES_N = Cfg::WAVES_N;
    constexpr int STAGES = Cfg::STAGES, SPB = Cfg::SPB;
    constexpr int WM = BM / Cfg::WAVES_M, WN = BN / WAVES_N, TM = WM / 16, TN = WN / 16;
    constexpr int AU = BM * BK / 4;                    // 16-byte units of one A term per stage
    constexpr int BU = BK * BN / 4;                    // of one B term
    constexpr int A2_OFF = AU;                         // second A term (FUSE)
    constexpr int B1_OFF = FUSE ? 2 * AU : AU;
    constexpr int B2_OFF = B1_OFF + BU;
    constexpr int UNITS = FUSE ? 2 * (AU + BU) : AU + BU;
    constexpr int GA = BM / 16;                        // A blocks of 16 rows per stage
    constexpr int CPR = BN / 4;                        // 16-byte chunks per B k-row
    constexpr int RPL = 64 / CPR;                      // B k-rows per wave load
    constexpr int GB = BK / RPL;                       // B loads per stage
    static_assert(BN >= 64 && GA % NW == 0 && GB % NW == 0, "loads must split evenly over the waves");
    __shared__ __attribute__((aligned(16))) uint4 lds[STAGES][UNITS];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WAVES_N, wn = w % WAVES_N;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t G = gridDim.x;
    const int64_t slot = xcd_slot(blockIdx.x, G);

    for (int64_t t = slot; t < total_tiles; t += G) {
        int64_t local;
        const ProbDesc& d = src.get(src.locate(t, local));
        const int64_t L = d.leaf;
        const int64_t tm_cnt = L / BM, tn_cnt = L / BN, tpl = tm_cnt * tn_cnt;
        const int64_t leaf = local / tpl;
        int64_t tm, tn;
        tile_coords(local - leaf * tpl, tm_cnt, tn_cnt, tm, tn);
        const float *Ap, *Bp, *Ap2 = nullptr, *Bp2 = nullptr;
        int64_t lda, ldb;
        uint32_t nega = 0, negb = 0;
        if constexpr (FUSE) {
            fused_operand(d, 0, leaf, Ap, Ap2, lda, nega);
            fused_operand(d, 1, leaf, Bp, Bp2, ldb, negb);
        } else {
            resolve(d, 0, d.depth, leaf, Ap, lda);
            resolve(d, 1, d.depth, leaf, Bp, ldb);
        }
        float* Cp;
        int64_t ldc;
        if (d.depth == 0) { Cp = d.C; ldc = d.ldu; }
        else { Cp = reinterpret_cast<float*>(d.ws) + d.leaf_m + leaf * L * L; ldc = L; }
        const bool crop = d.depth == 0 && d.bounded0;
        const int64_t m0 = tm * BM, n0 = tn * BN;

        // Per-lane sources.  A block g (rows 16g..16g+15) goes to wave g % NW;
        // lane l fills unit 4*(l/4) + l%4 of the block: row l/4, position
        // l%4, holding chunk (l%4) ^ blk_swz(l/4).  B load q (k-rows RPL q ..)
        // goes to wave q % NW; lane l fills position l % CPR of k-row
        // RPL q + l / CPR, holding chunk (l % CPR) ^ f32_bswz(k-row).
        const int arow = lane >> 2;
        const int64_t a_lane = (m0 + arow) * lda + 4 * ((lane & 3) ^ blk_swz(arow));
        const int bsub = lane / CPR, bpos = lane % CPR;

        // The K loop; TA / TB: the A / B operand has a second term.
        auto run = [&](auto TA, auto TB) {
            constexpr bool kTA = decltype(TA)::value, kTB = decltype(TB)::value;
            constexpr int LPS = (kTA ? 2 : 1) * GA / NW + (kTB ? 2 : 1) * GB / NW;   // loads per lane per stage
            auto issue = [&](int stage, int64_t k0) {
#pragma unroll
                for (int r = 0; r < GA / NW; ++r) {
                    const int g = w + NW * r;
                    __builtin_amdgcn_global_load_lds(Ap + a_lane + (int64_t)(16 * g) * lda + k0,
                                                     (lds_void_t*)&lds[stage][64 * g], 16, 0, 0);
                    if constexpr (kTA)
                        __builtin_amdgcn_global_load_lds(Ap2 + a_lane + (int64_t)(16 * g) * lda + k0,
                                                         (lds_void_t*)&lds[stage][A2_OFF + 64 * g], 16, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < GB / NW; ++r) {
                    const int q = w + NW * r, kr = RPL * q + bsub;
                    const int64_t off = (k0 + kr) * ldb + n0 + 4 * (bpos ^ f32_bswz(kr));
                    __builtin_amdgcn_global_load_lds(Bp + off, (lds_void_t*)&lds[stage][B1_OFF + 64 * q], 16, 0, 0);
                    if constexpr (kTB)
                        __builtin_amdgcn_global_load_lds(Bp2 + off, (lds_void_t*)&lds[stage][B2_OFF + 64 * q], 16,
                                                         0, 0);
                }
            };

            f32x4 acc[TM][TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

            const int64_t KT = L / BK;
            // Fragments of one K step from a stage image, and its MFMAs.
            auto read_step = [&](const uint4* sl, float (&b)[TN][4], float4 (&a)[TM]) {
                const float* sb = reinterpret_cast<const float*>(sl + B1_OFF);
                const float* sb2 = reinterpret_cast<const float*>(sl + B2_OFF);
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int col = wn * WN + 16 * j + li;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k = 4 * lg + s;
                        const int e = k * BN + 4 * ((col >> 2) ^ f32_bswz(k)) + (col & 3);
                        b[j][s] = sb[e];
                        if constexpr (kTB) b[j][s] = flip_add(b[j][s], sb2[e], negb);
                    }
                }
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int row = wm * WM + 16 * i + li;
                    const int e = 4 * row + (lg ^ blk_swz(row & 15));
                    a[i] = __builtin_bit_cast(float4, sl[e]);
                    if constexpr (kTA) a[i] = flip_add(a[i], __builtin_bit_cast(float4, sl[A2_OFF + e]), nega);
                }
            };
            auto mfma_step = [&](const float (&b)[TN][4], const float4 (&a)[TM]) {
#pragma unroll
                for (int i = 0; i < TM; ++i) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float av = s == 0 ? a[i].x : s == 1 ? a[i].y : s == 2 ? a[i].z : a[i].w;
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[j][s], acc[i][j], 0, 0, 0);
                    }
                }
            };
            if constexpr (SPB == 1) {
#pragma unroll
                for (int s = 0; s < STAGES - 1; ++s)
                    if (s < KT) issue(s, s * BK);
                for (int64_t kt = 0; kt < KT; ++kt) {
                    if (kt + STAGES - 2 < KT) wait_vmcnt<LPS * (STAGES - 2)>();
                    else wait_vmcnt<0>();
                    lds_barrier();       // step kt landed for every wave; step kt-1's reads are done
                    // Every fragment of the step is read before the copies of a
                    // later step are issued: the compiler cannot tell the stages
                    // apart and makes LDS reads wait for every copy issued before
                    // them, which would stall each step for the whole latency of
                    // its new copies.
                    float b[TN][4];
                    float4 a[TM];
                    read_step(lds[stage_of<STAGES>(kt)], b, a);
                    if (kt + STAGES - 1 < KT) issue(refill_stage_of<STAGES>(kt), (kt + STAGES - 1) * BK);
                    mfma_step(b, a);
                }
            } else {
                // SPB K steps per barrier over a ring of 2 SPB stages: the
                // steps of group g sit in stages SPB (g & 1) .. SPB (g & 1) +
                // SPB - 1; after the barrier every wave runs the group's
                // steps (the fragments of a step read during the MFMAs of the
                // one before), issuing the copies of group g + 1 into the
                // stages of group g - 1 (read by every wave before this
                // barrier) once its last step's fragments are read.  KT is a
                // multiple of SPB (the leaf edge is a multiple of BM).
                static_assert(STAGES == 2 * SPB, "a ring of two groups");
#pragma unroll
                for (int h = 0; h < SPB; ++h) issue(h, h * BK);
                for (int64_t kt = 0; kt < KT; kt += SPB) {
                    wait_vmcnt<0>();
                    lds_barrier();
                    const int g0 = (int)((kt / SPB) & 1) * SPB;
                    float b[TN][4];
                    float4 a[TM];
                    read_step(lds[g0], b, a);
#pragma unroll
                    for (int h = 1; h < SPB; ++h) {
                        mfma_step(b, a);
                        read_step(lds[g0 + h], b, a);
                    }
                    if (kt + SPB < KT) {
#pragma unroll
                        for (int h = 0; h < SPB; ++h) issue(SPB - g0 + h, (kt + SPB + h) * BK);
                    }
                    mfma_step(b, a);
                }
            }
            __syncthreads();         // the next tile's first loads overwrite the stages

#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = m0 + wm * WM + 16 * i + 4 * lg + r;
                        const int64_t col = n0 + wn * WN + 16 * j + li;
                        if (!crop || (row < d.n && col < d.n)) Cp[row * ldc + col] = acc[i][j][r];
                    }
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        if constexpr (!FUSE) {
            run(F_{}, F_{});
        } else {
            // (Algorithm 1 never has a view on both sides of one product)
            if (Ap2 && Bp2) run(T_{}, T_{});
            else if (Ap2) run(T_{}, F_{});
            else if (Bp2) run(F_{}, T_{});
            else run(F_{}, F_{});
        }
    }
}

template <class Src>
__global__ __launch_bounds__(F32BigCfg::NT) void k_gemm_f32_big(Src src, int64_t total_tiles) {
    gemm32_lds<F32BigCfg, Src, false>(src, total_tiles);
}
// Fused leaves: two terms per side make a stage 64 KB, so two stages.
template <class Src>
__global__ __launch_bounds__(F32FusedCfg::NT) void k_gemm_f32_fused(Src src, int64_t total_tiles) {
    gemm32_lds<F32FusedCfg, Src, true>(src, total_tiles);
}
template <class Src>
__global__ __launch_bounds__(F32MidCfg::NT) void k_gemm_f32_mid(Src src, int64_t total_tiles) {
    gemm32_lds<F32MidCfg, Src, false>(src, total_tiles);
}
template <class Src>
__global__ __launch_bounds__(F32SmallCfg::NT) void k_gemm_f32_small(Src src, int64_t total_tiles) {
    gemm32_lds<F32SmallCfg, Src, false>(src, total_tiles);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
template <class Src>
static hipError_t launch_f32_tile_t(const Src& s, int tile, int64_t tiles, int grid, hipStream_t st) {
    if (tile == 128) {
        hipLaunchKernelGGL((k_gemm_f32_mid<Src>), dim3(grid), dim3(F32MidCfg::NT), 0, st, s, tiles);
    } else {
        hipLaunchKernelGGL((k_gemm_f32_small<Src>), dim3(grid), dim3(F32SmallCfg::NT), 0, st, s, tiles);
    }
    return hipGetLastError();
}
template <class Src>
static hipError_t launch_f32_big_t(const Src& s, int64_t tiles, int grid, bool fused, hipStream_t st) {
    if (fused)
        hipLaunchKernelGGL((k_gemm_f32_fused<Src>), dim3(grid), dim3(F32FusedCfg::NT), 0, st, s, tiles);
    else
        hipLaunchKernelGGL((k_gemm_f32_big<Src>), dim3(grid), dim3(kF32BigThreads), 0, st, s, tiles);
    return hipGetLastError();
}
template <class Src, int P, bool F16>
static hipError_t launch_bf16_big_t(const Src& s, int64_t tiles, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_gemm_bf16_big<Src, P, F16>), dim3(grid), dim3(BigCfg<P>::NT), 0, st, s, tiles);
    return hipGetLastError();
}
// 16-bit leaf GEMM with a 128- or 64-wide tile
template <class Src, int P, bool F16>
static hipError_t launch_bf16_tile_t(const Src& s, int tile, int64_t tiles, int grid, hipStream_t st) {
    if (tile == 128)
        hipLaunchKernelGGL((k_gemm_bf16_mid<Src, P, F16>), dim3(grid), dim3(MidCfg<P>::NT), 0, st, s, tiles);
    else
        hipLaunchKernelGGL((k_gemm_bf16_small<Src, P, F16>), dim3(grid), dim3(SmallCfg<P>::NT), 0, st, s, tiles);
    return hipGetLastError();
}

template <class K>
static int occupancy(K kernel, int threads) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess) return 1;
    return n > 0 ? n : 1;
}

int64_t gemm_tiles_per_leaf(int planes, int tile, int64_t leaf) {
    if (tile == 256)   // 256 x 128 for three bf16 planes, else 256 x 256 (binary32 and two planes)
        return planes == 3 ? (leaf / BigCfg<3>::BM) * (leaf / BigCfg<3>::BN)
                           : (leaf / BigCfg<2>::BM) * (leaf / BigCfg<2>::BN);
    return (leaf / tile) * (leaf / tile);
}

int gemm_blocks_per_cu(int planes, int tile) {
    // Occupancy does not depend on the descriptor source or the 16-bit flavour.
    if (planes == 0)
        return tile == 256   ? occupancy(k_gemm_f32_big<OneProb>, kF32BigThreads)
               : tile == 128 ? occupancy(k_gemm_f32_mid<OneProb>, F32MidCfg::NT)
                             : occupancy(k_gemm_f32_small<OneProb>, F32SmallCfg::NT);
    if (tile == 256)
        return planes == 2 ? occupancy(k_gemm_bf16_big<OneProb, 2, false>, BigCfg<2>::NT)
                           : occupancy(k_gemm_bf16_big<OneProb, 3, false>, BigCfg<3>::NT);
    if (planes == 2)
        return tile == 128 ? occupancy(k_gemm_bf16_mid<OneProb, 2, false>, MidCfg<2>::NT)
                           : occupancy(k_gemm_bf16_small<OneProb, 2, false>, SmallCfg<2>::NT);
    return tile == 128 ? occupancy(k_gemm_bf16_mid<OneProb, 3, false>, MidCfg<3>::NT)
                       : occupancy(k_gemm_bf16_small<OneProb, 3, false>, SmallCfg<3>::NT);
}

template <class Src>
hipError_t launch_gemm(const Src& s, int planes, int tile, bool f16, int64_t tiles, int grid, hipStream_t st,
                       bool fused) {
    if (fused && (planes != 0 || tile != 256)) return hipErrorInvalidValue;
    if (planes == 0) return tile == 256 ? launch_f32_big_t<Src>(s, tiles, grid, fused, st)
                                        : launch_f32_tile_t<Src>(s, tile, tiles, grid, st);
    if (f16) {   // FP16X3: two binary16 planes
        if (tile == 256) return launch_bf16_big_t<Src, 2, true>(s, tiles, grid, st);
        return launch_bf16_tile_t<Src, 2, true>(s, tile, tiles, grid, st);
    }
    if (tile == 256) return planes == 2 ? launch_bf16_big_t<Src, 2, false>(s, tiles, grid, st)
                                        : launch_bf16_big_t<Src, 3, false>(s, tiles, grid, st);
    return planes == 2 ? launch_bf16_tile_t<Src, 2, false>(s, tile, tiles, grid, st)
                       : launch_bf16_tile_t<Src, 3, false>(s, tile, tiles, grid, st);
}

template hipError_t launch_gemm<OneProb>(const OneProb&, int, int, bool, int64_t, int, hipStream_t, bool);
template hipError_t launch_gemm<TableProb>(const TableProb&, int, int, bool, int64_t, int, hipStream_t, bool);

}  // namespace stk
