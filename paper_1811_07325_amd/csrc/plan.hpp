// Planner: padded size, leaf size, workspace layout and launch sequence of one
// multiply.  Pure host arithmetic (no HIP calls), so it is testable anywhere.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "common.hpp"

namespace stk {

constexpr int64_t kLeafGranule = 64;   // leaf edge is a multiple of this
constexpr double kPeelRate = 60e12;     // border and fix-up flops per second (model)

struct Plan {
    int64_t n = 0, np = 0, leaf = 0;
    int depth = 0;
    int precision = 0;   // stark_precision as passed (may carry STARK_WINOGRAD)
    int variant = 0;     // 0: Algorithm 1, 1: Winograd's variant
    int planes = 0;      // 0, 2, 3
    int tile = 128;      // leaf GEMM tile edge
    bool padded = false;  // level 0 reads A, B element by element (n != np,
                          // except a peeled plan with 16-byte-aligned rows)
    // Byte offsets (-1 = region absent).
    int64_t div_a[STK_MAXD], div_b[STK_MAXD];
    int div_slots[STK_MAXD];
    int64_t leaf_a = -1, leaf_b = -1, leaf_m = -1;
    int64_t comb[STK_MAXD];
    int64_t pad_a = -1, pad_b = -1;
    int64_t scale = -1;   // FP16X3 scale region
    size_t bytes = 0;
    int fp32_levels = 0;  // binary32 divide levels launched (0 .. depth)
    // binary32 leaves formed inside the leaf GEMM from the level above
    // (the divide stops one level early); see make_plan
    bool fuse = false;
    // residue peeled off: the recursion runs on the leading np x np core
    // (np = n - peel) in place; the border and the core's fix-up are
    // classical (see make_plan)
    int peel = 0;
};

int64_t pow7(int l);
int64_t padded_size(int64_t n, int depth);
int max_depth_for(int64_t n);
int planes_for(int precision);  // -1 if unknown (STARK_WINOGRAD may be set)

// Returns "" on success, else the reason the plan is invalid.  tile = 0
// takes the rule's leaf-GEMM tile class; 64, 128 or 256 (dividing the leaf)
// forces one (the autotuner's choice).
std::string make_plan(int64_t n, int depth, int precision, Plan& out, int tile = 0);

// Tile classes the autotuner measures for a plan: its own and the valid
// neighbouring classes (64, 128, 256 that divide the leaf).
int tile_candidates(const Plan& p, int out[3]);

// Descriptor of the plan with user/workspace pointers filled in.
ProbDesc make_desc(const Plan& p, const float* A, const float* B, float* C, void* ws);

// Algorithmic work of one multiply (stark_plan_info): leaf flops (useful,
// 2 L^3 per leaf; matrix-core flops count every split product) and the bytes
// the divide / split / combine phases must move.
struct Work {
    double leaf_flops, mfma_flops;
    double divide_bytes, split_bytes, combine_bytes, pad_bytes;
    // peeled plans: border and fix-up flops; bytes the border kernel must
    // read (A and B once)
    double peel_flops, peel_bytes;
};
Work plan_work(const Plan& p);

// Parts of the modelled time of a plan on one MI355X: the leaf GEMM on full
// waves of tiles (matrix-core work at the measured rate of its tile class,
// scaled for short K by leaf / (leaf + 128)), its tile count, the streaming
// passes (bytes at 3.5 TB/s on the 16-bit paths, 5 TB/s on binary32, plus the
// peeled border's vector flops) and the launch count.
struct ModelParts {
    double gemm_s, tiles, stream_s;
    int launches;
};
ModelParts model_parts(const Plan& p);

// Share of the CUs a launch of `tiles` tiles keeps busy over its waves of
// 256 (the last wave partly empty).
double wave_fill(double tiles);

// Rough time of one plan alone (seconds): gemm_s / wave_fill(tiles) +
// stream_s + 10 us per launch.  Only used to choose a depth where nothing
// has been measured.
double model_seconds(const Plan& p);

// Deepest level model_depth considers for (n, precision): 3, BF16X3 1.
int model_max_depth(int64_t n, int precision);

// Depth (0..3) of least model_seconds for (n, precision); BF16X3 at most 1.
int model_depth(int64_t n, int precision);

// Plans of a batch whose problems share every launch (grouped multiplies
// at the automatic depth).  Problems with fixed[i] keep plans[i]; each of
// the others takes, for a given tile class, its depth (0 ..
// model_max_depth) and padding of least gemm_s + stream_s: in a batch the
// other problems' tiles fill the waves, so a problem's own fill does not
// count.  The batch takes the cheaper of: every problem on one tile class
// (a single leaf GEMM launch), or each on its own best class; a choice
// costs, per class, the summed GEMM time over its launch's wave fill, plus
// every streaming pass, plus 10 us per GEMM launch.  Returns "" or the
// first problem's error.
std::string plan_batch(int count, const int64_t* n, int precision, std::vector<Plan>& plans,
                       const std::vector<char>& fixed);

}  // namespace stk
