// Host-side launchers of the device kernels (implemented next to the kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace stk {

// Block counts of one launch for one problem.
int64_t blocks_pad(const ProbDesc& d);
int64_t blocks_divide(const ProbDesc& d, int level);
int64_t blocks_split(const ProbDesc& d);
int64_t blocks_combine(const ProbDesc& d, int level);
int64_t blocks_combine2(const ProbDesc& d, int level);
int64_t blocks_peel(const ProbDesc& d);   // 0 unless the plan peels

template <class Src> hipError_t launch_pad(const Src& s, int64_t blocks, hipStream_t st);
// FP16X3 scaling: partial maxima (kScaleParts blocks per problem), then the
// exponents (1 block per problem).
template <class Src> hipError_t launch_absmax(const Src& s, int64_t blocks, hipStream_t st);
template <class Src> hipError_t launch_scale_exp(const Src& s, int64_t blocks, hipStream_t st);
// variant: 0 Algorithm 1, 1 Winograd's variant (same for every problem of
// a launch).
template <class Src> hipError_t launch_divide(const Src& s, int level, int variant, int64_t blocks, hipStream_t st);
template <class Src> hipError_t launch_split(const Src& s, int planes, int variant, int64_t blocks, hipStream_t st);
// peel: level 0 of a launch with peeled problems (adds their core fix-up).
template <class Src> hipError_t launch_combine(const Src& s, int level, int variant, int64_t blocks, hipStream_t st,
                                               bool peel = false);
// Combine levels `level` + 1 and `level` in one pass (depth >= level + 2).
template <class Src> hipError_t launch_combine2(const Src& s, int level, int variant, int64_t blocks, hipStream_t st,
                                                bool peel = false);
// Border rows and columns of peeled plans (max_peel: the largest residue
// among the launch's problems, 1 .. kPeelMaxResidue).
template <class Src> hipError_t launch_peel(const Src& s, int max_peel, int64_t blocks, hipStream_t st);
// f16: the two planes are binary16 (FP16X3) rather than bfloat16.  fused:
// binary32 leaves formed from the level above inside the GEMM (plans with
// fused leaves; 256-wide tiles only).
template <class Src> hipError_t launch_gemm(const Src& s, int planes, int tile, bool f16, int64_t tiles, int grid,
                                            hipStream_t st, bool fused = false);

// Tiles of one leaf of edge `leaf` for the GEMM variant (planes, tile class).
int64_t gemm_tiles_per_leaf(int planes, int tile, int64_t leaf);

// Resident blocks per CU of the leaf GEMM for (planes, tile).
int gemm_blocks_per_cu(int planes, int tile);

// Rectangular products: pack rows x cols of X (leading dimension ld) into
// zero-padded s x s blocks (row-major block order), and sum the block
// products P[(i NB + j) KB + p] over p into C (m x n, leading dimension n).
hipError_t launch_pack_blocks(const float* X, int64_t rows, int64_t cols, int64_t ld, float* dst, int64_t s,
                              hipStream_t st);
hipError_t launch_reduce_blocks(const float* P, float* C, int64_t m, int64_t n, int64_t s, int64_t MB, int64_t NB,
                                int64_t KB, hipStream_t st);

// Measurement helpers (k_check.hip).
hipError_t launch_matvec_f64(const float* M, const double* x, double* y, int64_t n, hipStream_t st);
hipError_t launch_row_errors(const float* C, int64_t n, const int64_t* rows, int64_t nrows,
                             const double* ref, double* out, hipStream_t st);
hipError_t launch_generate_normal(float* X, int64_t count, uint64_t seed, hipStream_t st);
// Binary64 sum of count floats; partials must hold 256 doubles.
hipError_t launch_sum_f64(const float* X, int64_t count, double* partials, double* out, hipStream_t st);

}  // namespace stk
