// Measurement-side kernels: the only binary64 arithmetic on the GPU (error
// checks; no Strassen step needs it), and the seeded operand generator of the
// serving path.
#include "common.hpp"
#include "launch.hpp"

namespace stk {

// y = M x, M binary32 (n x n row-major), x and y binary64.  One block per
// row; fixed per-thread strides and a fixed reduction tree (deterministic).
__global__ __launch_bounds__(256) void k_matvec_f64(const float* __restrict__ M, const double* __restrict__ x,
                                                    double* __restrict__ y, int64_t n) {
    __shared__ double part[256];
    const int64_t i = blockIdx.x;
    const float* row = M + i * n;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) s += (double)row[j] * x[j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) y[i] = part[0];
}

// Errors of sampled rows against a binary64 reference: max |d|, sum d^2,
// sum ref^2.  A single block of 1024 threads (deterministic reduction).
__global__ __launch_bounds__(1024) void k_row_errors(const float* __restrict__ C, int64_t n,
                                                     const int64_t* __restrict__ rows, int64_t nrows,
                                                     const double* __restrict__ ref, double* __restrict__ out) {
    __shared__ double smax[1024], sd2[1024], sr2[1024];
    double mx = 0.0, d2 = 0.0, r2 = 0.0;
    const int64_t total = nrows * n;
    for (int64_t f = threadIdx.x; f < total; f += 1024) {
        const int64_t i = f / n, j = f - i * n;
        const double rv = ref[f];
        const double dv = (double)C[rows[i] * n + j] - rv;
        mx = fmax(mx, fabs(dv));
        d2 += dv * dv;
        r2 += rv * rv;
    }
    smax[threadIdx.x] = mx;
    sd2[threadIdx.x] = d2;
    sr2[threadIdx.x] = r2;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            sd2[threadIdx.x] += sd2[threadIdx.x + w];
            sr2[threadIdx.x] += sr2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = sd2[0];
        out[2] = sr2[0];
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of the 4x32 bijection with the published
// multipliers and Weyl key increments.
struct Philox4 {
    uint32_t v[4];
};
__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Elements 4m .. 4m + 3: two Box-Muller pairs (Box and Muller, 1958) from
// one Philox call, counters (m_lo, m_hi, 0, 0), key (seed_lo, seed_hi).
// Pair j (words w_2j, w_2j+1): u1 = (w_2j + 1) 2^-32 in (0, 1] and
// u2 = w_2j+1 2^-32 (each rounded to binary32; the scaling is exact),
// radius sqrt(-2 ln u1), angle 2 pi u2; element 4m + 2j takes radius x
// cos(angle), element 4m + 2j + 1 radius x sin(angle): independent normal(0,
// 1) variates, at most 6.7 in magnitude.  Binary32 arithmetic throughout
// (the library's logf, sincosf and sqrtf, within a few ulps): a host
// repeating the steps in binary64 from the same binary32 u1, u2 agrees to a
// few binary32 ulps of the radius.
__device__ __forceinline__ void box_muller(uint32_t w1, uint32_t w2, float& z0, float& z1) {
    const float u1 = (float)((uint64_t)w1 + 1) * 0x1p-32f, u2 = (float)w2 * 0x1p-32f;
    const float radius = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincosf(6.28318530717958647692f * u2, &sn, &cs);
    z0 = radius * cs;
    z1 = radius * sn;
}

__global__ __launch_bounds__(256) void k_generate_normal(float* __restrict__ X, int64_t count, uint64_t seed) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (4 * m >= count) return;
    const Philox4 r = philox4x32_10((uint32_t)m, (uint32_t)((uint64_t)m >> 32), 0u, 0u, (uint32_t)seed,
                                    (uint32_t)(seed >> 32));
    float z[4];
    box_muller(r.v[0], r.v[1], z[0], z[1]);
    box_muller(r.v[2], r.v[3], z[2], z[3]);
    if (4 * m + 4 <= count) {
        *reinterpret_cast<float4*>(X + 4 * m) = make_float4(z[0], z[1], z[2], z[3]);
    } else {
        for (int j = 0; j < 4 && 4 * m + j < count; ++j) X[4 * m + j] = z[j];
    }
}

// Deterministic binary64 sum of X: kSumBlocks blocks sum contiguous chunks
// (a multiple of 4 elements each) with a fixed tree into partials, then one
// block sums the partials.  With X 16-byte aligned a thread reads float4,
// four of them in flight per step (one load at a time left the sum of an
// 8192^2 result at about 2 ms, bound by load latency); the order of the
// additions depends only on count and the alignment of X.
constexpr int kSumBlocks = 256;
__device__ __forceinline__ double sum4(float4 v) {
    return ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
}
__global__ __launch_bounds__(256) void k_sum_stage1(const float* __restrict__ X, int64_t count,
                                                    double* __restrict__ partials) {
    __shared__ double part[256];
    const int64_t chunk = (count + 4 * kSumBlocks - 1) / (4 * kSumBlocks) * 4;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < count ? lo + chunk : count;
    double s = 0.0;
    if (lo < hi && ((uintptr_t)X & 15) == 0) {
        const float4* X4 = reinterpret_cast<const float4*>(X + lo);   // lo is a multiple of 4
        const int64_t n4 = (hi - lo) >> 2;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t j = threadIdx.x;
        for (; j + 768 < n4; j += 1024) {
            const float4 a = X4[j], b = X4[j + 256], c = X4[j + 512], d = X4[j + 768];
            s0 += sum4(a);
            s1 += sum4(b);
            s2 += sum4(c);
            s3 += sum4(d);
        }
        for (; j < n4; j += 256) s0 += sum4(X4[j]);
        s = (s0 + s1) + (s2 + s3);
        for (int64_t i = lo + 4 * n4 + threadIdx.x; i < hi; i += 256) s += (double)X[i];
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += (double)X[i];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = part[0];
}
__global__ __launch_bounds__(256) void k_sum_stage2(const double* __restrict__ partials, double* __restrict__ out) {
    __shared__ double part[256];
    part[threadIdx.x] = partials[threadIdx.x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

hipError_t launch_sum_f64(const float* X, int64_t count, double* partials, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_stage1, dim3(kSumBlocks), dim3(256), 0, st, X, count, partials);
    hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(256), 0, st, partials, out);
    return hipGetLastError();
}

hipError_t launch_matvec_f64(const float* M, const double* x, double* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_matvec_f64, dim3((unsigned)n), dim3(256), 0, st, M, x, y, n);
    return hipGetLastError();
}
hipError_t launch_row_errors(const float* C, int64_t n, const int64_t* rows, int64_t nrows, const double* ref,
                             double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_row_errors, dim3(1), dim3(1024), 0, st, C, n, rows, nrows, ref, out);
    return hipGetLastError();
}
hipError_t launch_generate_normal(float* X, int64_t count, uint64_t seed, hipStream_t st) {
    const int64_t blocks = ((count + 3) / 4 + 255) / 256;   // one thread per four elements
    hipLaunchKernelGGL(k_generate_normal, dim3((unsigned)blocks), dim3(256), 0, st, X, count, seed);
    return hipGetLastError();
}

}  // namespace stk
