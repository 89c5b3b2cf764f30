/*
 * Stark CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statement of what the Strassen hot path
 * computes.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this file; the GPU library never does, and the two
 * share no code, headers or tables.
 *
 * Every floating-point routine works in IEEE binary64 on inputs that were
 * converted exactly from binary32 (the paper computes in double precision
 * throughout, Section V-A "Test Setup").  The FP32 step routines
 * (oracle_divide_f32 / oracle_combine_f32) exist so the GPU's divide and
 * combine kernels can be checked bit for bit: a single binary32 addition is
 * correctly rounded on both sides, and the order of the additions is fixed
 * below.
 *
 * Pins (what keeps this file honest; all run on the CPU):
 *   - brute force: on small-integer inputs the Strassen recursion, the
 *     classical triple loop, the int64 triple loop and numpy's integer matmul
 *     agree exactly, for every n <= 16 and every depth (odd n padded);
 *   - the 2x2 worked example of Algorithm 1 (golden file);
 *   - identities A*I = A, I*B = B, 0*B = 0, (-A)*B = -(A*B),
 *     (2^a A)(2^b B) = 2^(a+b) AB, which hold bit for bit;
 *   - structure: 7^k leaf products, 18 block additions per internal node,
 *     and each quadrant of A and B used 4/2/2/4 times per node (Section
 *     III-C-1, Fig. 3);
 *   - the classical loop against numpy/BLAS double matmul (library routine).
 *
 * Readings of the paper taken here (the paper is silent or misprinted):
 *   - Algorithm 1 prints C22 = M1 - M2 - M3 + M6; the product it must equal
 *     has +M3 (worked 2x2 example: the printed form gives 54, the product is
 *     50).  The oracle uses C22 = M1 - M2 + M3 + M6.
 *   - Algorithm 2 recurses on (A, B); the recursion must act on the divided
 *     pairs D.  The oracle recurses on the seven (S_i, T_i) pairs.
 *   - The base case (size equal to a threshold in Algorithm 1, a single
 *     block in Algorithm 2) is read as: recurse exactly `depth` times; the
 *     leaf size is n_pad / 2^depth.
 *   - Sizes that are not 2^p (the paper defers to partitioning) are
 *     zero-padded to n_pad, a multiple of 2^depth, and the product cropped.
 *     Padding is exact: the extra rows/columns contribute only zeros.
 *   - The order of the combine additions is left to right as printed:
 *     C11 = ((M1 + M4) - M5) + M7, C22 = ((M1 - M2) + M3) + M6.
 *
 * Winograd's variant (not in the paper; the "next" variant of the hot path):
 * the same seven-product recursion with 15 block additions per node instead
 * of 18, in the form published by S. Winograd (1971) and used by Douglas et
 * al. (1994) and Boyer et al. (2009):
 *   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
 *   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21,
 *   M1 = A11 B11, M2 = A12 B21, M3 = S4 B22, M4 = A22 T4,
 *   M5 = S1 T1, M6 = S2 T2, M7 = S3 T3,
 *   U2 = M1 + M6, U3 = U2 + M7,
 *   C11 = M1 + M2, C12 = (U2 + M5) + M3, C21 = U3 - M4, C22 = U3 + M5.
 * Its pins are the same kinds: brute force, a hand-computed 2x2 example,
 * 15 additions per node, planted mistakes.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math:
 * every operation below is a plain IEEE operation in the written order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Structural counters (pins for Algorithm 1 / Section III-C-1).            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t leaf_products;   /* base-case multiplications performed         */
    int64_t internal_nodes;  /* recursion nodes that divided                */
    int64_t block_additions; /* h x h additions/subtractions (divide+combine)*/
    int64_t uses_a[4];       /* uses of A11, A12, A21, A22 by the 7 products */
    int64_t uses_b[4];       /* uses of B11, B12, B21, B22                   */
} oracle_counts;

/* Deliberate-mistake switch, used only by the tests that prove the pins
 * catch plausible errors.  0 = the oracle as specified.  Never set by any
 * product path. */
static int g_mutation = 0;
void oracle_set_mutation(int m) { g_mutation = m; }

/* ------------------------------------------------------------------------ */
/* Classical product, the plain definition C[i][j] = sum_t A[i][t] B[t][j]. */
/* i-t-j loop order; rows are independent and split over OpenMP threads.    */
/* ------------------------------------------------------------------------ */
static void classical_f64(const double* A, int64_t lda, const double* B, int64_t ldb,
                          double* C, int64_t ldc, int64_t m, int parallel)
{
#pragma omp parallel for schedule(static) if (parallel)
    for (int64_t i = 0; i < m; ++i) {
        double* c = C + i * ldc;
        for (int64_t j = 0; j < m; ++j) c[j] = 0.0;
        for (int64_t t = 0; t < m; ++t) {
            const double a = A[i * lda + t];
            const double* b = B + t * ldb;
            for (int64_t j = 0; j < m; ++j) c[j] += a * b[j];
        }
    }
}

void oracle_gemm_f64(const double* A, const double* B, double* C, int64_t n)
{
    classical_f64(A, n, B, n, C, n, n, 1);
}

/* Rectangular classical product C (m x n) = A (m x k) B (k x n), row-major,
 * FP64, the same i-t-j order. */
void oracle_gemm_rect_f64(const double* A, const double* B, double* C, int64_t m, int64_t k, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double* c = C + i * n;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t t = 0; t < k; ++t) {
            const double a = A[i * k + t];
            const double* b = B + t * n;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

void oracle_gemm_i64(const int64_t* A, const int64_t* B, int64_t* C, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t s = 0;
            for (int64_t t = 0; t < n; ++t) s += A[i * n + t] * B[t * n + j];
            C[i * n + j] = s;
        }
}

/* Selected rows of the classical product: out[r][:] = A[rows[r]][:] * B,
 * in the same i-t-j order as classical_f64 (so a sampled row is bit-identical
 * to that row of the full product). */
void oracle_rows_f64(const double* A, const double* B, int64_t n,
                     const int64_t* rows, int64_t nrows, double* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        double* c = out + r * n;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t t = 0; t < n; ++t) {
            const double a = A[i * n + t];
            const double* b = B + t * n;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

/* y = M x in double (Freivalds' check: ||C x - A (B x)||, Freivalds 1977). */
void oracle_gemv_f64(const double* M, const double* x, double* y, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += M[i * n + j] * x[j];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Strassen recursion, Algorithm 1 (Section III-A), depth-limited.          */
/* ------------------------------------------------------------------------ */

/* out = P + sign*Q on h x h blocks (out contiguous, ld = h). */
static void block_addsub(double* out, const double* P, int64_t ldp, const double* Q, int64_t ldq,
                         double sign, int64_t h)
{
    for (int64_t i = 0; i < h; ++i)
        for (int64_t j = 0; j < h; ++j)
            out[i * h + j] = (sign > 0) ? P[i * ldp + j] + Q[i * ldq + j]
                                        : P[i * ldp + j] - Q[i * ldq + j];
}

static void block_copy(double* out, const double* P, int64_t ldp, int64_t h)
{
    for (int64_t i = 0; i < h; ++i) memcpy(out + i * h, P + i * ldp, (size_t)h * sizeof(double));
}

static void strassen_rec(const double* X, int64_t ldx, const double* Y, int64_t ldy,
                         double* Z, int64_t ldz, int64_t m, int levels, int top,
                         oracle_counts* cnt)
{
    if (levels == 0) {
        /* Base case: the classical product of the two leaf blocks. */
        classical_f64(X, ldx, Y, ldy, Z, ldz, m, top);
        cnt->leaf_products += 1;
        return;
    }
    const int64_t h = m / 2;
    const size_t hh = (size_t)h * (size_t)h;
    /* The four quadrants of each operand (views, no copies). */
    const double *A11 = X, *A12 = X + h, *A21 = X + h * ldx, *A22 = X + h * ldx + h;
    const double *B11 = Y, *B12 = Y + h, *B21 = Y + h * ldy, *B22 = Y + h * ldy + h;

    /* Two operand scratch blocks and the seven products M1..M7. */
    double* s = (double*)malloc(hh * sizeof(double));
    double* t = (double*)malloc(hh * sizeof(double));
    double* M = (double*)malloc(7 * hh * sizeof(double));
    double *M1 = M, *M2 = M + hh, *M3 = M + 2 * hh, *M4 = M + 3 * hh,
           *M5 = M + 4 * hh, *M6 = M + 5 * hh, *M7 = M + 6 * hh;
    const int lv = levels - 1;

    cnt->internal_nodes += 1;

    /* M1 = (A11 + A22)(B11 + B22) */
    block_addsub(s, A11, ldx, A22, ldx, +1, h);
    block_addsub(t, B11, ldy, B22, ldy, +1, h);
    cnt->uses_a[0]++; cnt->uses_a[3]++; cnt->uses_b[0]++; cnt->uses_b[3]++;
    strassen_rec(s, h, t, h, M1, h, h, lv, 0, cnt);

    /* M2 = (A21 + A22) B11 */
    block_addsub(s, A21, ldx, A22, ldx, +1, h);
    cnt->uses_a[2]++; cnt->uses_a[3]++; cnt->uses_b[0]++;
    strassen_rec(s, h, B11, ldy, M2, h, h, lv, 0, cnt);

    /* M3 = A11 (B12 - B22) */
    block_addsub(t, B12, ldy, B22, ldy, -1, h);
    cnt->uses_a[0]++; cnt->uses_b[1]++; cnt->uses_b[3]++;
    if (g_mutation == 2) /* mistake: operands of M3 exchanged */
        strassen_rec(t, h, A11, ldx, M3, h, h, lv, 0, cnt);
    else
        strassen_rec(A11, ldx, t, h, M3, h, h, lv, 0, cnt);

    /* M4 = A22 (B21 - B11) */
    block_addsub(t, B21, ldy, B11, ldy, -1, h);
    cnt->uses_a[3]++; cnt->uses_b[2]++; cnt->uses_b[0]++;
    strassen_rec(A22, ldx, t, h, M4, h, h, lv, 0, cnt);

    /* M5 = (A11 + A12) B22 */
    if (g_mutation == 3) /* mistake: A21 taken for A12 */
        block_addsub(s, A11, ldx, A21, ldx, +1, h);
    else
        block_addsub(s, A11, ldx, A12, ldx, +1, h);
    cnt->uses_a[0]++; cnt->uses_a[1]++; cnt->uses_b[3]++;
    strassen_rec(s, h, B22, ldy, M5, h, h, lv, 0, cnt);

    /* M6 = (A21 - A11)(B11 + B12) */
    block_addsub(s, A21, ldx, A11, ldx, -1, h);
    block_addsub(t, B11, ldy, B12, ldy, +1, h);
    cnt->uses_a[2]++; cnt->uses_a[0]++; cnt->uses_b[0]++; cnt->uses_b[1]++;
    strassen_rec(s, h, t, h, M6, h, h, lv, 0, cnt);

    /* M7 = (A12 - A22)(B21 + B22) */
    block_addsub(s, A12, ldx, A22, ldx, -1, h);
    block_addsub(t, B21, ldy, B22, ldy, +1, h);
    cnt->uses_a[1]++; cnt->uses_a[3]++; cnt->uses_b[2]++; cnt->uses_b[3]++;
    strassen_rec(s, h, t, h, M7, h, h, lv, 0, cnt);

    /* 10 operand additions above, 8 below: 18 per node. */
    cnt->block_additions += 18;

    /* Combine, left to right as printed (C22 with +M3, see header). */
    double *C11 = Z, *C12 = Z + h, *C21 = Z + h * ldz, *C22 = Z + h * ldz + h;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < h; ++j) {
            const size_t q = (size_t)i * h + j;
            double c11 = ((M1[q] + M4[q]) - M5[q]);
            if (g_mutation != 4) c11 = c11 + M7[q]; /* mistake 4: M7 dropped */
            C11[i * ldz + j] = c11;
            C12[i * ldz + j] = M3[q] + M5[q];
            C21[i * ldz + j] = M2[q] + M4[q];
            if (g_mutation == 1) /* mistake 1: C22 sign exactly as printed */
                C22[i * ldz + j] = ((M1[q] - M2[q]) - M3[q]) + M6[q];
            else
                C22[i * ldz + j] = ((M1[q] - M2[q]) + M3[q]) + M6[q];
        }
    }
    free(s); free(t); free(M);
}

/* C (n x n) = A (n x n) * B (n x n) by `depth` levels of Strassen on the
 * zero-padded n_pad x n_pad operands; n_pad must be >= n and a multiple of
 * 2^depth.  Returns 0, or -1 on bad arguments.  cnt may be NULL. */
int oracle_strassen_f64(const double* A, const double* B, double* C, int64_t n,
                        int depth, int64_t n_pad, oracle_counts* cnt)
{
    oracle_counts local;
    if (!cnt) cnt = &local;
    memset(cnt, 0, sizeof(*cnt));
    if (n <= 0 || depth < 0 || depth > 20 || n_pad < n || (n_pad % ((int64_t)1 << depth)) != 0)
        return -1;
    const size_t N = (size_t)n_pad * (size_t)n_pad;
    double* Ap = (double*)calloc(N, sizeof(double));
    double* Bp = (double*)calloc(N, sizeof(double));
    double* Cp = (double*)calloc(N, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        memcpy(Ap + i * n_pad, A + i * n, (size_t)n * sizeof(double));
        memcpy(Bp + i * n_pad, B + i * n, (size_t)n * sizeof(double));
    }
    strassen_rec(Ap, n_pad, Bp, n_pad, Cp, n_pad, n_pad, depth, 1, cnt);
    for (int64_t i = 0; i < n; ++i) memcpy(C + i * n, Cp + i * n_pad, (size_t)n * sizeof(double));
    free(Ap); free(Bp); free(Cp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Winograd's variant in binary64 (definitions in the header).              */
/* ------------------------------------------------------------------------ */
static void winograd_rec(const double* X, int64_t ldx, const double* Y, int64_t ldy,
                         double* Z, int64_t ldz, int64_t m, int levels, int top,
                         oracle_counts* cnt)
{
    if (levels == 0) {
        classical_f64(X, ldx, Y, ldy, Z, ldz, m, top);
        cnt->leaf_products += 1;
        return;
    }
    const int64_t h = m / 2;
    const size_t hh = (size_t)h * (size_t)h;
    const double *A11 = X, *A12 = X + h, *A21 = X + h * ldx, *A22 = X + h * ldx + h;
    const double *B11 = Y, *B12 = Y + h, *B21 = Y + h * ldy, *B22 = Y + h * ldy + h;
    double* S = (double*)malloc(4 * hh * sizeof(double));   /* S1..S4 */
    double* T = (double*)malloc(4 * hh * sizeof(double));   /* T1..T4 */
    double* M = (double*)malloc(7 * hh * sizeof(double));
    double *S1 = S, *S2 = S + hh, *S3 = S + 2 * hh, *S4 = S + 3 * hh;
    double *T1 = T, *T2 = T + hh, *T3 = T + 2 * hh, *T4 = T + 3 * hh;
    const int lv = levels - 1;
    cnt->internal_nodes += 1;

    block_addsub(S1, A21, ldx, A22, ldx, +1, h);
    block_addsub(S2, S1, h, A11, ldx, -1, h);
    block_addsub(S3, A11, ldx, A21, ldx, -1, h);
    if (g_mutation == 5) /* mistake: S4 taken from S1 instead of S2 */
        block_addsub(S4, A12, ldx, S1, h, -1, h);
    else
        block_addsub(S4, A12, ldx, S2, h, -1, h);
    block_addsub(T1, B12, ldy, B11, ldy, -1, h);
    block_addsub(T2, B22, ldy, T1, h, -1, h);
    block_addsub(T3, B22, ldy, B12, ldy, -1, h);
    block_addsub(T4, T2, h, B21, ldy, -1, h);

    winograd_rec(A11, ldx, B11, ldy, M, h, h, lv, 0, cnt);
    winograd_rec(A12, ldx, B21, ldy, M + hh, h, h, lv, 0, cnt);
    winograd_rec(S4, h, B22, ldy, M + 2 * hh, h, h, lv, 0, cnt);
    winograd_rec(A22, ldx, T4, h, M + 3 * hh, h, h, lv, 0, cnt);
    winograd_rec(S1, h, T1, h, M + 4 * hh, h, h, lv, 0, cnt);
    winograd_rec(S2, h, T2, h, M + 5 * hh, h, h, lv, 0, cnt);
    winograd_rec(S3, h, T3, h, M + 6 * hh, h, h, lv, 0, cnt);
    cnt->uses_a[0] += 1; cnt->uses_a[1] += 1; cnt->uses_a[3] += 1;   /* direct operands */
    cnt->uses_b[0] += 1; cnt->uses_b[2] += 1; cnt->uses_b[3] += 1;

    /* 8 operand additions above, 7 below: 15 per node. */
    cnt->block_additions += 15;
    double *C11 = Z, *C12 = Z + h, *C21 = Z + h * ldz, *C22 = Z + h * ldz + h;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < h; ++j) {
            const size_t q = (size_t)i * h + j;
            const double m1 = M[q], m2 = M[hh + q], m3 = M[2 * hh + q], m4 = M[3 * hh + q];
            const double m5 = M[4 * hh + q], m6 = M[5 * hh + q], m7 = M[6 * hh + q];
            const double u2 = m1 + m6, u3 = u2 + m7;
            C11[i * ldz + j] = m1 + m2;
            C12[i * ldz + j] = (u2 + m5) + m3;
            C21[i * ldz + j] = (g_mutation == 6) ? u3 + m4 : u3 - m4;   /* mistake 6: sign of M4 */
            C22[i * ldz + j] = u3 + m5;
        }
    }
    free(S); free(T); free(M);
}

/* As oracle_strassen_f64, with Winograd's variant at every level. */
int oracle_winograd_f64(const double* A, const double* B, double* C, int64_t n,
                        int depth, int64_t n_pad, oracle_counts* cnt)
{
    oracle_counts local;
    if (!cnt) cnt = &local;
    memset(cnt, 0, sizeof(*cnt));
    if (n <= 0 || depth < 0 || depth > 20 || n_pad < n || (n_pad % ((int64_t)1 << depth)) != 0)
        return -1;
    const size_t N = (size_t)n_pad * (size_t)n_pad;
    double* Ap = (double*)calloc(N, sizeof(double));
    double* Bp = (double*)calloc(N, sizeof(double));
    double* Cp = (double*)calloc(N, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        memcpy(Ap + i * n_pad, A + i * n, (size_t)n * sizeof(double));
        memcpy(Bp + i * n_pad, B + i * n, (size_t)n * sizeof(double));
    }
    winograd_rec(Ap, n_pad, Bp, n_pad, Cp, n_pad, n_pad, depth, 1, cnt);
    for (int64_t i = 0; i < n; ++i) memcpy(C + i * n, Cp + i * n_pad, (size_t)n * sizeof(double));
    free(Ap); free(Bp); free(Cp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One divide step and one combine step in binary32, for bit-exact checks    */
/* of the GPU's per-level kernels.                                           */
/* ------------------------------------------------------------------------ */

/* Operand pairs of the seven products of one node (Algorithm 1; replication
 * map of Section III-C-1 / Fig. 3).  X, Y: m x m with leading dims ldx, ldy.
 * S, T: 7 contiguous h x h blocks each (h = m/2), S[i], T[i] the operands of
 * M_{i+1}; the pass-through operands (S3 = A11, S4 = A22, T2 = B11, T5 = B22)
 * are copied so that every block is explicit. */
void oracle_divide_f32(const float* X, int64_t ldx, const float* Y, int64_t ldy, int64_t m,
                       float* S, float* T)
{
    const int64_t h = m / 2;
    const size_t hh = (size_t)h * (size_t)h;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < h; ++j) {
            const float a11 = X[i * ldx + j], a12 = X[i * ldx + j + h];
            const float a21 = X[(i + h) * ldx + j], a22 = X[(i + h) * ldx + j + h];
            const float b11 = Y[i * ldy + j], b12 = Y[i * ldy + j + h];
            const float b21 = Y[(i + h) * ldy + j], b22 = Y[(i + h) * ldy + j + h];
            const size_t q = (size_t)i * h + j;
            S[0 * hh + q] = a11 + a22;  T[0 * hh + q] = b11 + b22;  /* M1 */
            S[1 * hh + q] = a21 + a22;  T[1 * hh + q] = b11;        /* M2 */
            S[2 * hh + q] = a11;        T[2 * hh + q] = b12 - b22;  /* M3 */
            S[3 * hh + q] = a22;        T[3 * hh + q] = b21 - b11;  /* M4 */
            S[4 * hh + q] = a11 + a12;  T[4 * hh + q] = b22;        /* M5 */
            S[5 * hh + q] = a21 - a11;  T[5 * hh + q] = b11 + b12;  /* M6 */
            S[6 * hh + q] = a12 - a22;  T[6 * hh + q] = b21 + b22;  /* M7 */
        }
    }
}

/* C (m x m, leading dim ldc) from the seven h x h products M[0..6] = M1..M7
 * (Algorithm 1, C22 with +M3), additions left to right in binary32. */
void oracle_combine_f32(const float* M, int64_t h, float* C, int64_t ldc)
{
    const size_t hh = (size_t)h * (size_t)h;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < h; ++j) {
            const size_t q = (size_t)i * h + j;
            const float m1 = M[q], m2 = M[hh + q], m3 = M[2 * hh + q], m4 = M[3 * hh + q];
            const float m5 = M[4 * hh + q], m6 = M[5 * hh + q], m7 = M[6 * hh + q];
            C[i * ldc + j] = ((m1 + m4) - m5) + m7;
            C[i * ldc + j + h] = m3 + m5;
            C[(i + h) * ldc + j] = m2 + m4;
            C[(i + h) * ldc + j + h] = ((m1 - m2) + m3) + m6;
        }
    }
}

/* Winograd's variant, one divide step in binary32: S[i], T[i] the operands
 * of M_{i+1} in product order (A11, A12, S4, A22, S1, S2, S3 and B11, B21,
 * B22, T4, T1, T2, T3), each sum rounded once in the order of the header. */
void oracle_divide_f32_w(const float* X, int64_t ldx, const float* Y, int64_t ldy, int64_t m,
                         float* S, float* T)
{
    const int64_t h = m / 2;
    const size_t hh = (size_t)h * (size_t)h;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < h; ++j) {
            const float a11 = X[i * ldx + j], a12 = X[i * ldx + j + h];
            const float a21 = X[(i + h) * ldx + j], a22 = X[(i + h) * ldx + j + h];
            const float b11 = Y[i * ldy + j], b12 = Y[i * ldy + j + h];
            const float b21 = Y[(i + h) * ldy + j], b22 = Y[(i + h) * ldy + j + h];
            const float s1 = a21 + a22, s2 = s1 - a11, s3 = a11 - a21, s4 = a12 - s2;
            const float t1 = b12 - b11, t2 = b22 - t1, t3 = b22 - b12, t4 = t2 - b21;
            const size_t q = (size_t)i * h + j;
            S[0 * hh + q] = a11;  T[0 * hh + q] = b11;   /* M1 */
            S[1 * hh + q] = a12;  T[1 * hh + q] = b21;   /* M2 */
            S[2 * hh + q] = s4;   T[2 * hh + q] = b22;   /* M3 */
            S[3 * hh + q] = a22;  T[3 * hh + q] = t4;    /* M4 */
            S[4 * hh + q] = s1;   T[4 * hh + q] = t1;    /* M5 */
            S[5 * hh + q] = s2;   T[5 * hh + q] = t2;    /* M6 */
            S[6 * hh + q] = s3;   T[6 * hh + q] = t3;    /* M7 */
        }
    }
}

/* Winograd's variant, one combine step in binary32 (order of the header). */
void oracle_combine_f32_w(const float* M, int64_t h, float* C, int64_t ldc)
{
    const size_t hh = (size_t)h * (size_t)h;
    for (int64_t i = 0; i < h; ++i) {
        for (int64_t j = 0; j < h; ++j) {
            const size_t q = (size_t)i * h + j;
            const float m1 = M[q], m2 = M[hh + q], m3 = M[2 * hh + q], m4 = M[3 * hh + q];
            const float m5 = M[4 * hh + q], m6 = M[5 * hh + q], m7 = M[6 * hh + q];
            const float u2 = m1 + m6, u3 = u2 + m7;
            C[i * ldc + j] = m1 + m2;
            C[i * ldc + j + h] = (u2 + m5) + m3;
            C[(i + h) * ldc + j] = u3 - m4;
            C[(i + h) * ldc + j + h] = u3 + m5;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* bfloat16 split (not in the paper: the leaf-precision scheme of the GPU    */
/* path).  bfloat16 = the upper 16 bits of a binary32; rounding to nearest,  */
/* ties to even, on the 16 discarded bits.  Finite inputs only.             */
/* ------------------------------------------------------------------------ */
static uint16_t bf16_rne(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

static float bf16_to_f32(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
}

/* binary16 (IEEE 754 half): 1 sign, 5 exponent (bias 15), 10 fraction bits.
 * Round a binary32 to the nearest binary16 value, ties to even, with
 * subnormals (spacing 2^-24) and overflow to infinity; the result is
 * returned as its exact binary32 value (every binary16 is a binary32). */
static float f16_round(float x)
{
    if (x != x) return x;
    const double ax = fabs((double)x);
    if (ax == 0.0) return x;
    int e;
    frexp(ax, &e);                 /* ax = m * 2^e, m in [0.5, 1) */
    int ulp_exp = e - 11;          /* 11 significant bits */
    if (ulp_exp < -24) ulp_exp = -24;   /* subnormal spacing */
    const double ulp = ldexp(1.0, ulp_exp);
    double q = ax / ulp;           /* exact: ax is a binary32, ulp a power of two */
    double fl = floor(q);
    const double rem = q - fl;
    if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) != 0.0)) fl += 1.0;
    double r = fl * ulp;
    if (r >= 65520.0) r = INFINITY;     /* beyond the largest finite half after rounding */
    return (float)(x < 0 ? -r : r);
}

/* Power-of-two scale exponent of the FP16X3 leaf operands of one matrix:
 * with max|X| = m * 2^E (m in [0.5, 1)), the leaf operands after `depth`
 * levels are at most 2^depth max|X|, so scaling by 2^(14 - depth - E)
 * keeps them below 2^14 (binary16's largest finite value is 65504).  In
 * Winograd's variant an operand sums up to four blocks per level (S4, T4),
 * so its callers pass 2 * depth.  The exponent is capped at 127, the largest
 * for which 2^e is a finite binary32. */
int oracle_f16_scale_exp(const float* X, int64_t count, int depth)
{
    float m = 0.0f;
    for (int64_t i = 0; i < count; ++i) {
        const float a = fabsf(X[i]);
        if (a > m) m = a;
    }
    if (m == 0.0f) return 0;
    int E;
    frexp((double)m, &E);
    const int e = 14 - depth - E;
    return e < 127 ? e : 127;
}

/* x ~= hi + mid + lo with each term bfloat16: hi = rne(x), mid = rne(x - hi),
 * lo = rne(x - hi - mid).  The differences are exact in binary32. `terms` is
 * 2 (hi, mid) or 3; out has `terms` planes of count values each. */
void oracle_split_bf16(const float* x, int64_t count, int terms, uint16_t* out)
{
    for (int64_t i = 0; i < count; ++i) {
        float r = x[i];
        for (int p = 0; p < terms; ++p) {
            const uint16_t b = bf16_rne(r);
            out[(size_t)p * (size_t)count + (size_t)i] = b;
            r = r - bf16_to_f32(b);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Arithmetic model of the GPU path (error-model tool).                      */
/*                                                                            */
/* The same recursion as oracle_strassen_f64, but every operand sum and every */
/* combine addition is a binary32 operation (oracle_divide_f32 /              */
/* oracle_combine_f32 order), and each leaf product is formed exactly in     */
/* binary64 from the leaf operands as the leaf arithmetic sees them, then    */
/* rounded once to binary32:                                                  */
/*   mode 0 (FP32):   x*y                                                     */
/*   mode 2 (BF16X3): xh*yh + xh*yl + xl*yh           (2-term split)          */
/*   mode 3 (BF16X6): + xh*ym.. the six cross terms of the 3-term split whose */
/*                    plane indices sum to at most 2                          */
/*   mode 4 (FP16X3): x scaled by 2^ex, y by 2^ey (oracle_f16_scale_exp of  */
/*                    the whole A and B), split into two binary16 terms,     */
/*                    xh*yh + xh*yl + xl*yh, result scaled by 2^-ex, then  */
/*                    by 2^-ey (two exact steps, as the GPU epilogue)       */
/* The GPU accumulates the leaf sums in binary32 instead; the difference is  */
/* that accumulation's rounding only, so GPU results sit within a few units  */
/* of accumulation error of this model at any depth.                         */
/* ------------------------------------------------------------------------ */
static int g_model_ex = 0, g_model_ey = 0;   /* FP16X3 scale exponents of the current run */

static void leaf_model(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* Z, int64_t ldz,
                       int64_t m, int mode)
{
    const int terms = mode == 0 ? 1 : (mode == 2 || mode == 4) ? 2 : 3;
    const size_t mm = (size_t)m * (size_t)m;
    /* planes of X and Y as doubles (mode 0: the values themselves) */
    double* xp = (double*)malloc((size_t)terms * mm * sizeof(double));
    double* yp = (double*)malloc((size_t)terms * mm * sizeof(double));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < m; ++j) {
            float rx = X[i * ldx + j], ry = Y[i * ldy + j];
            if (mode == 4) { rx = ldexpf(rx, g_model_ex); ry = ldexpf(ry, g_model_ey); }
            for (int p = 0; p < terms; ++p) {
                float hx = rx, hy = ry;
                if (mode == 4) { hx = f16_round(rx); hy = f16_round(ry); }
                else if (mode != 0) { hx = bf16_to_f32(bf16_rne(rx)); hy = bf16_to_f32(bf16_rne(ry)); }
                xp[(size_t)p * mm + (size_t)i * m + j] = hx;
                yp[(size_t)p * mm + (size_t)i * m + j] = hy;
                rx = rx - hx;
                ry = ry - hy;
            }
        }
    double* acc = (double*)calloc(mm, sizeof(double));
    for (int pa = 0; pa < terms; ++pa)
        for (int pb = 0; pb < terms; ++pb) {
            if (pa + pb > terms - 1) continue;   /* keep hi*hi (+ hi*lo, lo*hi (+ ...)) */
            const double* xa = xp + (size_t)pa * mm;
            const double* yb = yp + (size_t)pb * mm;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < m; ++i)
                for (int64_t t = 0; t < m; ++t) {
                    const double a = xa[(size_t)i * m + t];
                    const double* y = yb + (size_t)t * m;
                    double* c = acc + (size_t)i * m;
                    for (int64_t j = 0; j < m; ++j) c[j] += a * y[j];
                }
        }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < m; ++j) {
            float z = (float)acc[(size_t)i * m + j];
            if (mode == 4) z = ldexpf(ldexpf(z, -g_model_ex), -g_model_ey);   /* one factor at a time */
            Z[i * ldz + j] = z;
        }
    free(xp); free(yp); free(acc);
}

static void model_rec(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* Z, int64_t ldz,
                      int64_t m, int levels, int mode, int variant)
{
    if (levels == 0) {
        leaf_model(X, ldx, Y, ldy, Z, ldz, m, mode);
        return;
    }
    const int64_t h = m / 2;
    const size_t hh = (size_t)h * (size_t)h;
    float* S = (float*)malloc(7 * hh * sizeof(float));
    float* T = (float*)malloc(7 * hh * sizeof(float));
    float* M = (float*)malloc(7 * hh * sizeof(float));
    if (variant) oracle_divide_f32_w(X, ldx, Y, ldy, m, S, T);
    else oracle_divide_f32(X, ldx, Y, ldy, m, S, T);
    for (int i = 0; i < 7; ++i)
        model_rec(S + i * hh, h, T + i * hh, h, M + i * hh, h, h, levels - 1, mode, variant);
    if (variant) oracle_combine_f32_w(M, h, Z, ldz);
    else oracle_combine_f32(M, h, Z, ldz);
    free(S); free(T); free(M);
}

/* C (n x n, binary32) from binary32 A, B: zero-pad to n_pad, `depth` levels
 * of Algorithm 1 (variant 0) or of Winograd's variant (1), leaf arithmetic
 * `mode` (0, 2, 3, 4), crop.  Returns 0 or -1. */
int oracle_model_f32(const float* A, const float* B, float* C, int64_t n, int depth, int64_t n_pad,
                     int mode, int variant)
{
    if (n <= 0 || depth < 0 || depth > 20 || n_pad < n || (n_pad % ((int64_t)1 << depth)) != 0 ||
        (mode != 0 && mode != 2 && mode != 3 && mode != 4) || (variant != 0 && variant != 1))
        return -1;
    if (mode == 4) {   /* growth per level: 2 blocks (Algorithm 1), 4 (Winograd) */
        g_model_ex = oracle_f16_scale_exp(A, n * n, variant ? 2 * depth : depth);
        g_model_ey = oracle_f16_scale_exp(B, n * n, variant ? 2 * depth : depth);
    }
    const size_t N = (size_t)n_pad * (size_t)n_pad;
    float* Ap = (float*)calloc(N, sizeof(float));
    float* Bp = (float*)calloc(N, sizeof(float));
    float* Cp = (float*)calloc(N, sizeof(float));
    for (int64_t i = 0; i < n; ++i) {
        memcpy(Ap + i * n_pad, A + i * n, (size_t)n * sizeof(float));
        memcpy(Bp + i * n_pad, B + i * n, (size_t)n * sizeof(float));
    }
    model_rec(Ap, n_pad, Bp, n_pad, Cp, n_pad, n_pad, depth, mode, variant);
    for (int64_t i = 0; i < n; ++i) memcpy(C + i * n, Cp + i * n_pad, (size_t)n * sizeof(float));
    free(Ap); free(Bp); free(Cp);
    return 0;
}

int oracle_strassen_model_f32(const float* A, const float* B, float* C, int64_t n, int depth, int64_t n_pad,
                              int mode)
{
    return oracle_model_f32(A, B, C, n, depth, n_pad, mode, 0);
}

/* Peeled sizes (not in the paper, which treats n = 2^p and leaves other
 * sizes to partitioning schemes of other work, Section III-A): with
 * nc = n - r, write A = [A11 A12; A21 A22] with A11 the leading nc x nc
 * block (likewise B).  Then
 *   C11 = A11 B11 + A12 B21        (the recursion on the core, plus r terms)
 *   C12 = A11 B12 + A12 B22        = rows 0..nc-1 of A times columns nc..n-1 of B
 *   C21, C22 = A21 B + A22 B2*     = rows nc..n-1 of A times all of B,
 * so only A11 B11 goes through Strassen's recursion (unpadded, nc a multiple
 * of 2^depth).  Arithmetic model of that scheme: the core by model_rec
 * (binary32 divide/combine, leaf `mode`; FP16X3 scale exponents from the
 * whole of A and B), every core output plus its r-term sum A12 B21 and every
 * border output (an inner product of length n) exact in binary64, each
 * rounded once to binary32.  Returns 0 or -1. */
int oracle_peel_model_f32(const float* A, const float* B, float* C, int64_t n, int64_t nc, int depth, int mode,
                          int variant)
{
    if (n <= 0 || nc <= 0 || nc > n || depth < 0 || depth > 20 || (nc % ((int64_t)1 << depth)) != 0 ||
        (mode != 0 && mode != 2 && mode != 3 && mode != 4) || (variant != 0 && variant != 1))
        return -1;
    if (mode == 4) {
        g_model_ex = oracle_f16_scale_exp(A, n * n, variant ? 2 * depth : depth);
        g_model_ey = oracle_f16_scale_exp(B, n * n, variant ? 2 * depth : depth);
    }
    model_rec(A, n, B, n, C, n, nc, depth, mode, variant);   /* core, in place (leading dimension n) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const int core = i < nc && j < nc;
            double acc = core ? (double)C[i * n + j] : 0.0;
            for (int64_t t = core ? nc : 0; t < n; ++t) acc += (double)A[i * n + t] * (double)B[t * n + j];
            C[i * n + j] = (float)acc;
        }
    return 0;
}

/* x * 2^e ~= hi + lo with binary16 terms (RNE), as binary32 values. */
void oracle_split_f16(const float* x, int64_t count, int e, float* out)
{
    for (int64_t i = 0; i < count; ++i) {
        const float v = ldexpf(x[i], e);
        const float hi = f16_round(v);
        out[i] = hi;
        out[count + i] = f16_round(v - hi);
    }
}

/* Threads the OpenMP loops above use (for reporting CPU timings). */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops from here on (CPU timings on 1 thread). */
void oracle_set_threads(int count)
{
#ifdef _OPENMP
    if (count > 0) omp_set_num_threads(count);
#else
    (void)count;
#endif
}
