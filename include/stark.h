/*
 * stark.h -- C ABI of the MI355X (gfx950) Strassen hot path.
 *
 * The library computes C = A * B for square dense binary32 matrices with
 * `depth` levels of Strassen's seven-product recursion (Algorithm 1,
 * Section III-A of Misra, Bhattacharya and Ghosh, "Stark: Fast and Scalable
 * Strassen's Matrix Multiplication using Apache Spark").  The three phases of
 * the paper's distributed method (Section III-C) become GPU launches:
 *   divide   (Section III-C-1, Algorithms 2-3): one launch per recursion level
 *            forms the operand sums S_i, T_i of every node of that level;
 *   leaf     (Section III-C-2, Algorithm 4): one grouped launch multiplies all
 *            7^depth leaf pairs;
 *   combine  (Section III-C-3, Algorithm 5): one launch per level folds
 *            M1..M7 of every node back into its four quadrants.
 * Sizes that are not a multiple of 2^depth * 64 are zero-padded (the paper
 * treats n = 2^p and defers other sizes to partitioning, Section III-A).
 *
 * Conventions for every call:
 *   - Matrices are device pointers to row-major binary32 with leading
 *     dimension n (n x n, contiguous), 16-byte aligned (EINVAL otherwise;
 *     allocator results always are).  The caller owns them; the library
 *     never frees caller memory.  A, B, C must stay valid until the work
 *     enqueued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work and return; they do not synchronise.
 *   - A context's workspace holds one call's intermediates at a time, so the
 *     calls that use it (stark_gemm, stark_gemm_phases, stark_gemm_batched,
 *     stark_gemm_rect, stark_tune) run one after another on the device
 *     whatever streams they are given: each waits for the previous one's
 *     work.  Multiplies meant to overlap on the device go through the
 *     serving calls (stark_submit) or separate contexts.  Contexts are
 *     thread-safe; calls from several threads are serialised.
 *   - Status codes are returned; no exception crosses the ABI.  On failure
 *     stark_last_error() returns a message (thread-local, valid until the
 *     next failing call on that thread).
 */
#ifndef STARK_H
#define STARK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int stark_status;
#define STARK_OK 0
#define STARK_PENDING 1          /* stark_poll: request not finished yet      */
#define STARK_EINVAL (-1)        /* bad argument                              */
#define STARK_ENOMEM (-2)        /* workspace or HBM budget too small         */
#define STARK_EDEVICE (-3)       /* a HIP call failed (message kept)          */
#define STARK_EBUSY (-4)         /* serving queue full                        */
#define STARK_ENOTFOUND (-5)     /* unknown ticket                            */
#define STARK_EUNSUPPORTED (-6)  /* valid but not supported (e.g. precision)  */

/* Arithmetic of the leaf products.  Divide and combine are binary32 in all
 * modes.  BF16X3: each leaf operand x is split as hi = bf16(x),
 * lo = bf16(x - hi) (round to nearest even) and the product is formed from
 * hi*hi + hi*lo + lo*hi on bf16 matrix cores with binary32 accumulation.
 * BF16X6: three terms (hi, mid, lo) and the six products whose order of
 * magnitude is at least 2^-16 of hi*hi.
 * FP16X3: each matrix is scaled by a power of two 2^e (from its largest
 * magnitude, so every leaf operand stays below 2^14), each leaf operand split
 * into two binary16 terms hi + lo (22 significant bits), hi*hi + hi*lo +
 * lo*hi on fp16 matrix cores with binary32 accumulation, and the product
 * scaled back exactly (the exponent is capped at 127 for matrices whose
 * largest magnitude is below about 2^-113).  An entry 2^-k times the largest
 * magnitude of its matrix keeps about min(22, 38 - depth - k) significant
 * bits (binary16 subnormals below that): at depth 0 every row and column
 * down to 2^-20 of the largest keeps binary32-level accuracy.  At depth >= 1
 * Strassen's operand sums add rows (and columns) of different scales, so in
 * every leaf precision, FP32 included, a row much smaller than the rows it
 * is added to loses accuracy; the error bound of the recursion is normwise. */
typedef enum {
    STARK_FP32 = 0,
    STARK_BF16X3 = 1,
    STARK_BF16X6 = 2,
    STARK_FP16X3 = 3,
    /* Flag, OR-ed into any of the above wherever a precision is passed:
     * Winograd's variant of the recursion (the same seven products at every
     * level, formed with 15 block additions per node instead of 18:
     * S1 = A21+A22, S2 = S1-A11, S3 = A11-A21, S4 = A12-S2, T1 = B12-B11,
     * T2 = B22-T1, T3 = B22-B12, T4 = T2-B21; M1..M7 = A11 B11, A12 B21,
     * S4 B22, A22 T4, S1 T1, S2 T2, S3 T3; C11 = M1+M2, U2 = M1+M6,
     * U3 = U2+M7, C12 = (U2+M5)+M3, C21 = U3-M4, C22 = U3+M5). */
    STARK_WINOGRAD = 16,
    /* Flag: binary32 leaves formed inside the leaf GEMM.  With Algorithm 1,
     * binary32 leaves on the 256-wide leaf-GEMM tiles, depth >= 1 (and not
     * depth 1 of a padded size) the leaf GEMM forms the last level's operand
     * sums itself from the quadrants of the level above while it copies its
     * tiles into LDS (the fusion of "Strassen's Algorithm Reloaded", Huang et
     * al., SC'16), so the divide stops one level early and the workspace
     * shrinks by the last level's operand blocks; the result is the same bit
     * for bit.  Elsewhere the flag is ignored (stark_plan_info reports
     * whether it applies).  Off by default: the leaf GEMM then moves twice
     * the operand bytes for five of the seven products and runs slower than
     * the stored-operand path plus the divide it saves. */
    STARK_FUSED = 32,
    /* Sizes that are not a multiple of 64 * 2^depth (Section III-A treats
     * n = 2^p only and leaves other sizes to partitioning).  Either the
     * residue r = n mod (64 * 2^depth) is peeled (possible for
     * 1 <= r <= 64, depth >= 1 and n - r >= 64 * 2^depth): the recursion
     * runs on the leading (n - r) x (n - r) core of A and B in place, the r
     * border rows and columns of C are classical binary32 inner products,
     * and every core output takes the r products through A's peeled columns
     * and B's peeled rows when the last combine level writes it.  Or A and B
     * are zero-padded to a multiple of 64, 128 or 256 times 2^depth (on the
     * fly: level 0 reads them with bounds) and C is cropped.  By default the
     * planner takes the candidate its time model finds fastest; STARK_PEEL
     * peels whenever possible, STARK_PAD always pads, and giving both is an
     * error.  stark_plan_info reports the residue a plan peels and the
     * padded (or core) edge n_pad. */
    STARK_PEEL = 64,
    STARK_PAD = 128
} stark_precision;
#define STARK_PRECISION_MASK 15

#define STARK_DEPTH_AUTO (-1)    /* let the autotuner choose the depth        */
#define STARK_MAX_DEPTH 8

typedef struct stark_ctx stark_ctx;

typedef struct {
    int device;               /* HIP device ordinal                               */
    void* workspace;          /* optional caller-owned device buffer lent to the
                                 context until stark_destroy; NULL = the library
                                 allocates (and grows) its own                    */
    size_t workspace_bytes;   /* size of `workspace`                              */
    size_t hbm_budget_bytes;  /* serving: device bytes the engine may hold
                                 (0 = 3/4 of free memory at create time), taken
                                 in segments of at least 4 GiB as admissions
                                 need them                                        */
    int max_slots;            /* serving: concurrent requests (0 = 4)             */
    const char* tuner_cache;  /* autotuner cache file (NULL = none)               */
} stark_config;

/* Create a context on cfg->device.  cfg may be NULL (device 0, library-owned
 * workspace).  *out receives the context.  Errors: EINVAL, EDEVICE. */
stark_status stark_create(stark_ctx** out, const stark_config* cfg);

/* Wait for work the context enqueued (serving included) and free everything
 * the context owns.  NULL is accepted. */
stark_status stark_destroy(stark_ctx* ctx);

/* Bytes of workspace one multiply of size n needs at this depth and
 * precision (pure function, no context).  depth must be >= 0. */
stark_status stark_workspace_size(int64_t n, int depth, stark_precision p, size_t* bytes);

/* Largest depth usable for n (leaf size >= 64 after padding). */
int stark_max_depth(int64_t n);

/* Depth (0..3) the library uses for a STARK_DEPTH_AUTO request that no
 * autotuner record covers (served requests): the one of least modelled time,
 * from the plan's matrix-core work at the measured rate of its leaf-GEMM tile
 * class, its streaming bytes and its launch count; at most 1 for BF16X3,
 * whose error roughly doubles per level.  -1 for n <= 0 or an unknown
 * precision. */
int stark_model_depth(int64_t n, stark_precision p);

/* C = A * B with `depth` Strassen levels (Algorithm 1; depth 0 is the
 * classical product on the same leaf kernels).  depth = STARK_DEPTH_AUTO asks
 * the autotuner (which may also run measurements on `stream` the first time a
 * size is seen).  C must not overlap A or B.  Errors: EINVAL (null or
 * misaligned pointer, n <= 0, depth out of range, overlap), ENOMEM (caller workspace too small),
 * EUNSUPPORTED, EDEVICE. */
stark_status stark_gemm(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n,
                        int depth, stark_precision p, void* stream);

/* For callers that cannot allocate device memory (work under stream capture,
 * serving loops or harnesses that forbid the allocator): stark_gemm without a
 * context.  Same arguments, layout, arithmetic and result as stark_gemm at
 * the same depth; depth = STARK_DEPTH_AUTO takes stark_model_depth(n, p).  It
 * calls no allocator: the intermediates of the multiply live in a fixed
 * device array of STARK_NOALLOC_SCRATCH_BYTES per GPU, part of the library's
 * device code (held by every GPU the library runs on until the process ends).
 * A plan needing more (see stark_workspace_size: e.g. n <= 1024 fits up to
 * depth 2, n = 2048 at depth 0) is refused with ENOMEM before anything is
 * enqueued.  Runs on the current device and enqueues on `stream`.  Every
 * call on one GPU shares that GPU's array: calls that overlap on the device
 * (other streams, other threads) race and corrupt each other's results --
 * order them (one stream, or events).  Nothing in the array needs clearing
 * between calls; it keeps the last call's intermediates.  Errors: EINVAL,
 * ENOMEM, EUNSUPPORTED, EDEVICE. */
#define STARK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
stark_status stark_gemm_noalloc(const float* A, const float* B, float* C, int64_t n, int depth,
                                stark_precision p, void* stream);

/* Rectangular product C (m x n) = A (m x k) B (k x n): row-major binary32
 * with leading dimensions k, n and n, 16-byte aligned base pointers (rows
 * need not be aligned).  depth = STARK_DEPTH_AUTO takes
 * stark_model_depth(min(m, k, n), p).  The paper treats n = 2^p and defers other shapes to
 * partitioning (Section III-A): A and B are packed into zero-padded square
 * s x s blocks, s = stark_rect_block_edge(m, k, n, depth); every block
 * product A_ip B_pj runs at `depth` as one problem of a grouped launch (as
 * stark_gemm_batched); C_ij = sum over p of the products in binary32, in
 * ascending p, cropped to m x n.  The context keeps the packed blocks and
 * products (grown on demand).  Errors: EINVAL (null or misaligned pointer,
 * m, k or n <= 0, depth out of range, C overlapping A or B, more than 4096
 * block products), EUNSUPPORTED, ENOMEM, EDEVICE. */
stark_status stark_gemm_rect(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t m, int64_t k,
                             int64_t n, int depth, stark_precision p, void* stream);

/* Block edge s of stark_gemm_rect: the smallest multiple of 64 * 2^depth not
 * below min(m, k, n); -1 for invalid arguments. */
int64_t stark_rect_block_edge(int64_t m, int64_t k, int64_t n, int depth);

/* One measured point of the autotuner: depth, median time of three runs
 * (ms), the relative error estimated by Freivalds' check in binary64, and the
 * leaf-GEMM tile class (64, 128 or 256: the edge of the square output tile one
 * workgroup computes). */
typedef struct {
    int depth;
    double ms;
    double err;
    int tile;
} stark_tune_point;

/* Autotune the depth and the leaf-GEMM tile class for (n, p): for every depth
 * in [min_depth, max_depth] (clamped to stark_max_depth(n)), run the planner's
 * tile class and its valid neighbours (64 / 128 / 256 dividing the leaf) on
 * the caller's A and B (C is overwritten), time each after a warm-up,
 * estimate its error as ||C x - A (B x)|| / ||A (B x)|| for a Gaussian x, and
 * record the fastest (depth, tile) whose error is <= tol (tol <= 0: 1e-5 or
 * STARK_TUNE_TOL).  If no point is within tol nothing is recorded (a record
 * made earlier stays) and the call still returns STARK_OK: the points carry
 * their errors.  Later calls with depth = STARK_DEPTH_AUTO (stark_gemm,
 * stark_submit, stark_gemm_batched) use the record; one with no record tunes
 * depths 0..5 first and, should none meet the tolerance, records the most
 * accurate point, marked as outside it in the cache file.  Up to `cap`
 * points are written to `points` (may be NULL) and their number to *count
 * (may be NULL).  Synchronises `stream`. */
stark_status stark_tune(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n,
                        stark_precision p, int min_depth, int max_depth, double tol,
                        stark_tune_point* points, int cap, int* count, void* stream);

/* `count` independent products C[i] = A[i] * B[i] of sizes n[i] (host arrays
 * of device pointers / sizes), all in one precision, at `depth` (clamped per
 * problem to stark_max_depth) or, with depth = STARK_DEPTH_AUTO, each problem
 * at its autotuner record (depth and tile class) if the context has one for
 * (n[i], p); the other problems are planned together (the autotuner itself is
 * not run): for each, the depth (up to 3; BF16X3 up to 1) and padding of
 * least modelled time on a tile class, where the other problems' tiles fill
 * the waves, and the batch takes one tile class for all of them (a single
 * leaf-GEMM launch) unless its model finds per-problem classes faster (see
 * stark_plan_batched).  Every recursion level of every problem is one
 * launch, and all leaf products of all problems form one grouped launch per
 * tile class, the problems with the longest leaves first; the sequence is
 * captured once into a hipGraph and replayed.  Errors as stark_gemm. */
stark_status stark_gemm_batched(stark_ctx* ctx, int count, const float* const* A,
                                const float* const* B, float* const* C, const int64_t* n,
                                int depth, stark_precision p, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent multiply requests.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;                /* matrix size                                       */
    stark_precision precision;
    int depth;                /* >= 0, or STARK_DEPTH_AUTO                         */
    const float* A;           /* device operands owned by the caller, or NULL to  */
    const float* B;           /* have the engine generate them on the device from */
    float* C;                 /* `seed` (normal(0,1), see stark_generate_normal); */
    uint64_t seed;            /* C NULL = library-owned result (freed at poll)    */
    uint64_t tag;             /* caller's tag, returned by poll                    */
} stark_request;

typedef struct {
    uint64_t tag;
    int depth;                /* depth actually used                               */
    stark_status status;
    double t_submit_us;       /* host steady-clock timestamps (microseconds)       */
    double t_admit_us;
    double t_done_us;         /* completion as observed by the engine              */
    double gpu_ms;            /* device time between the request's own events      */
    double checksum;          /* sum of the result in binary64 (library-owned C)   */
} stark_result;

/* Enqueue a request; returns at once with a ticket.  Thread-safe.  The
 * engine runs requests on streams of its own that do not wait for any stream
 * of the caller: caller-owned A, B and C must hold their final contents on the
 * device (e.g. the host synchronised after writing them) before the call, and
 * must stay valid, and C unread, until stark_poll returns STARK_OK.
 * Errors: EINVAL, EBUSY (queue full), ENOMEM (request alone exceeds the HBM
 * budget). */
stark_status stark_submit(stark_ctx* ctx, const stark_request* r, uint64_t* ticket);

/* STARK_PENDING while the request runs; STARK_OK (out filled, ticket
 * retired) or the request's error once done; ENOTFOUND for an unknown or
 * retired ticket.  Thread-safe. */
stark_status stark_poll(stark_ctx* ctx, uint64_t ticket, stark_result* out);

typedef struct {
    uint64_t completed;
    uint64_t failed;
    double throughput_tflops; /* effective 2n^3/t over the engine's busy span     */
    double p50_ms;            /* latency submit -> done, over the most recent
                                 2^20 completed requests                           */
    double p99_ms;
    double max_inflight_bytes;
    int max_concurrent;       /* most requests on the device at once               */
} stark_stats_t;

stark_status stark_stats(stark_ctx* ctx, stark_stats_t* out);

/* Start a new statistics window: counts, latencies, throughput span and
 * maxima restart from the requests completed after this call (requests in
 * flight are counted when they finish).  Thread-safe; no effect before the
 * first stark_submit. */
stark_status stark_stats_reset(stark_ctx* ctx);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* stark_last_error(void);

/* ------------------------------------------------------------------------ */
/* Measurement helpers (binary64 on the GPU, used by tests and benchmarks).  */
/* ------------------------------------------------------------------------ */

/* y = M x in binary64 for a device binary32 M (n x n, row-major) and device
 * binary64 x, y.  Freivalds' check (1977) compares C x with A (B x), both
 * formed with this call. */
stark_status stark_matvec_f64(const float* M, const double* x, double* y, int64_t n, void* stream);

/* Sums over the sampled rows: out[0] = max |C[r][j] - ref[i][j]|,
 * out[1] = sum (C - ref)^2, out[2] = sum ref^2, where r = rows[i]; rows is a
 * device int64 array, ref a device binary64 array (nrows x n), out a device
 * binary64 array of 3. */
stark_status stark_row_errors(const float* C, int64_t n, const int64_t* rows, int64_t nrows,
                              const double* ref, double* out, void* stream);

/* Fill X (n x n binary32, device) with normal(0,1) values from `seed`:
 * Philox4x32-10 (Salmon et al., SC'11) counter stream: elements 4m .. 4m+3
 * (row-major) take one Philox call (counters m_lo, m_hi, 0, 0; key = seed);
 * words (w0, w1) and (w2, w3) each give uniforms u1 = (w + 1) 2^-32 in
 * (0, 1] and u2 = w' 2^-32 and the Box-Muller pair sqrt(-2 ln u1) cos(2 pi
 * u2), sqrt(-2 ln u1) sin(2 pi u2) in binary32 (independent normal(0, 1);
 * magnitude at most 6.7).  A host repeating the steps in binary64 agrees to
 * a few binary32 ulps.  X: n x n device binary32, 16-byte aligned (EINVAL
 * otherwise, as for NULL X or n <= 0). */
stark_status stark_generate_normal(float* X, int64_t n, uint64_t seed, void* stream);

/* ------------------------------------------------------------------------ */
/* Introspection for tests and profiling.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, n_pad, leaf;   /* user size, padded size (a peeled plan: its core),
                                 leaf size n_pad/2^depth                           */
    int depth, precision, planes;
    int64_t div_a[STARK_MAX_DEPTH], div_b[STARK_MAX_DEPTH]; /* byte offsets of the
                                 binary32 divide outputs of level l (-1 = none)    */
    int div_slots[STARK_MAX_DEPTH]; /* blocks per node written at level l (5 or 7) */
    int64_t leaf_a, leaf_b;   /* byte offsets of the split bf16 leaf operands (-1) */
    int64_t leaf_m;           /* byte offset of the 7^depth leaf products (-1 when
                                 depth 0 writes C directly)                        */
    int64_t comb[STARK_MAX_DEPTH]; /* byte offset of level-l combine output (l>=1) */
    int64_t pad_a, pad_b;     /* byte offsets of padded copies (depth-0 FP32 only) */
    size_t bytes;             /* total workspace                                   */
    int gemm_tile;            /* leaf GEMM tile class (64, 128 or 256)             */
    int64_t scale;            /* FP16X3: byte offset of the scale region: 2 x 256
                                 binary32 partial maxima, then the two int32
                                 exponents e_A, e_B (-1 otherwise)                 */
    /* Algorithmic work of one multiply (what the method must move or compute;
     * views not counted): bytes of the binary32 divide levels, of the split
     * (16-bit paths; it forms the last one or two divide levels) and of the
     * combine; useful leaf flops (2 L^3 per leaf) and matrix-core flops
     * (times 1, 3, 6 or 3 products for FP32, BF16X3, BF16X6, FP16X3). */
    double divide_bytes, split_bytes, combine_bytes, leaf_flops, mfma_flops;
    int variant;              /* 0: Algorithm 1, 1: Winograd's variant           */
    int fused;                /* 1: the leaf GEMM forms the last level's operands
                                 (binary32; see STARK_FUSED)                       */
    int peel;                 /* residue r peeled off (n_pad = n - r is then the
                                 core the recursion runs on; see STARK_PEEL)       */
    double peel_flops;        /* border products plus the core's r-term fix-up     */
} stark_plan_desc;

stark_status stark_plan_info(int64_t n, int depth, stark_precision p, stark_plan_desc* out);

/* Plans stark_gemm_batched gives `count` problems of edges n[] (host array)
 * at `depth` (or STARK_DEPTH_AUTO) in precision p: out[i] (host array of
 * count) receives problem i's plan as stark_plan_info describes it.  ctx
 * supplies the autotuner records STARK_DEPTH_AUTO takes; it may be NULL (no
 * records).  Host work only.  Errors: EINVAL (count <= 0, NULL n or out, a
 * problem without a plan), EUNSUPPORTED (precision). */
stark_status stark_plan_batched(stark_ctx* ctx, int count, const int64_t* n, int depth, stark_precision p,
                                stark_plan_desc* out);

/* Phases for stark_gemm_phases. */
#define STARK_PHASE_DIVIDE 1u   /* pad, divide levels and the 16-bit split        */
#define STARK_PHASE_LEAF 2u     /* grouped leaf products                          */
#define STARK_PHASE_COMBINE 4u  /* combine levels (level 0 writes C)              */
#define STARK_PHASE_ALL 7u

/* As stark_gemm at a fixed depth, but only the phases in `mask` are launched
 * (eagerly, no graph); the workspace keeps its contents between calls, so a
 * test can run the phases one by one and inspect the regions described by
 * stark_plan_info. */
stark_status stark_gemm_phases(stark_ctx* ctx, const float* A, const float* B, float* C, int64_t n,
                               int depth, stark_precision p, unsigned mask, void* stream);

/* Device address of the context's workspace (NULL before first use) and its
 * size; lets tests read the regions of stark_plan_info. */
stark_status stark_workspace(stark_ctx* ctx, void** ptr, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* STARK_H */
