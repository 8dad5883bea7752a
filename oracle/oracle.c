/*
 * CPU oracle for split-BF16 linear algebra (Henry, Tang & Heinecke,
 * "Leveraging the bfloat16 Artificial Intelligence Datatype For
 * Higher-Precision Computations", 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct statement of what the GPU library computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header or table with the HIP library and
 * must never be used to produce a product result.
 *
 * Arithmetic conventions (fixed by the paper, Sec. II-B/II-C/II-D):
 *   - every partial inner product is an FP32 FMA chain, one rounding per
 *     step, in increasing index order, starting from +0;
 *   - bin sums and the final combination are FP32 additions in the
 *     printed parenthesisation;
 *   - the build uses -ffp-contract=off and no fast-math, so an
 *     expression a*b+c is two roundings and fmaf() is one.
 *
 * Readings where the paper is silent (each is listed in the design doc):
 *   R-rne   FP32->BF16 conversion rounds to nearest, ties to even.
 *   R-sat   a finite value whose RNE result would overflow to Inf is
 *           saturated to the largest finite BF16 of that sign, so that
 *           the split stays exact up to the top of the FP32 range
 *           (the paper's usable exponent range extends to 127, Sec. II-F).
 *   R-nan   NaN converts to the canonical quiet NaN of its sign.
 *   R-nonfinite  for Inf/NaN inputs b1 = b2 = +0.
 *   R-bins  the 9-product result sums all five bins smallest first:
 *           Z0 + (Z1 + (Z2 + (Z3 + Z4))) (Sec. II-D prints Z_3 without
 *           Z4; Sec. II-G says bins are added smallest to largest).
 *   R-x7    the 7-product variant adds Z^(1,2) as bin 3, the product the
 *           worked example of Sec. II-G singles out.
 *   R-epi   C = alpha*X when beta == 0 (C not read), else
 *           C = fmaf(alpha, X, beta*C)  (BLAS convention).
 *   R-po    per-operand split counts (Sec. II-G): pa terms of A, pb of B,
 *           the products a_i b_j with i + j <= 2, bins as x6 (x3 when
 *           both counts are at most 2).
 *   R-fmt   the single-format (BF16, FP16) LU of the Sec. IV-B tables
 *           rounds the matrix and every multiplier and update to the
 *           format once (nearest even, gradual underflow, overflow to
 *           Inf); the paper does not say which operations it rounds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Bit views                                                           */
/* ------------------------------------------------------------------ */
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* ------------------------------------------------------------------ */
/* Sec. I / Sec. II-A: the (B16) conversion.                            */
/* A BF16 number is an FP32 number whose low 16 bits are zero.  For a  */
/* finite FP32 value, the two BF16 neighbours of |a| are its pattern   */
/* with the low 16 bits cleared (toward zero) and that plus one BF16   */
/* unit (away from zero).  Round to nearest, ties to the neighbour     */
/* whose last kept bit is 0 (R-rne).                                    */
/* ------------------------------------------------------------------ */
uint16_t orc_bf16_rne(float a)
{
    uint32_t u = f2u(a);
    uint32_t sign = u & 0x80000000u;
    uint32_t mag = u & 0x7FFFFFFFu;
    if (mag > 0x7F800000u)                 /* NaN (R-nan) */
        return (uint16_t)((sign >> 16) | 0x7FC0u);
    if (mag == 0x7F800000u)                /* +-Inf */
        return (uint16_t)(u >> 16);
    uint32_t toward_zero = mag & 0xFFFF0000u;
    uint32_t away = toward_zero + 0x10000u;
    uint32_t rest = mag & 0x0000FFFFu;
    uint32_t pick;
    if (rest > 0x8000u)
        pick = away;
    else if (rest < 0x8000u)
        pick = toward_zero;
    else
        pick = ((toward_zero >> 16) & 1u) ? away : toward_zero;
    if (pick == 0x7F800000u)               /* would overflow: R-sat */
        pick = 0x7F7F0000u;
    return (uint16_t)((sign | pick) >> 16);
}

float orc_bf16_to_f32(uint16_t h) { return u2f((uint32_t)h << 16); }

/* ------------------------------------------------------------------ */
/* Sec. II-A: split of one FP32 value into three BF16 terms            */
/*   b0 = (B16)a,  b1 = (B16)(a - b0),  b2 = (B16)(a - b0 - b1).       */
/* The subtractions are exact FP32 operations in the range the paper   */
/* calls usable; a - b0 - b1 is evaluated left to right.                */
/* ------------------------------------------------------------------ */
static void split_one(float a, uint16_t *h0, uint16_t *h1, uint16_t *h2)
{
    if (!isfinite(a)) {                    /* R-nonfinite */
        *h0 = orc_bf16_rne(a);
        *h1 = 0;
        *h2 = 0;
        return;
    }
    *h0 = orc_bf16_rne(a);
    float r1 = a - orc_bf16_to_f32(*h0);
    *h1 = orc_bf16_rne(r1);
    float r2 = r1 - orc_bf16_to_f32(*h1);
    *h2 = orc_bf16_rne(r2);
}

/* Split n values; b2 may be NULL (two-term split). */
void orc_split(const float *a, int64_t n, uint16_t *b0, uint16_t *b1,
               uint16_t *b2)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint16_t h0, h1, h2;
        split_one(a[i], &h0, &h1, &h2);
        b0[i] = h0;
        b1[i] = h1;
        if (b2) b2[i] = h2;
    }
}

/* ------------------------------------------------------------------ */
/* Split-product variants.                                              */
/* variant = number of BF16 products formed per scalar product:         */
/*   1: Z00                          (one BF16 term each, split table)  */
/*   3: Z0 + Z1                      (two terms, Sec. II-G)             */
/*   6: Z0 + (Z1 + Z2)               (Z_2 of Sec. II-D)                 */
/*   7: Z0 + (Z1 + (Z2 + Z12))       (R-x7, worked example Sec. II-G)   */
/*   8: Z0 + (Z1 + (Z2 + Z3))        (Z_3 of Sec. II-D)                 */
/*   9: Z0 + (Z1 + (Z2 + (Z3 + Z4))) (R-bins)                           */
/*  12, 13, 21, 23, 31, 32: per-operand split counts (see per_operand)   */
/* ------------------------------------------------------------------ */
/* Per-operand split counts (Sec. II-G, "a different number of splits"):  */
/* variant 10 pa + pb (pa != pb, both in 1..3) takes pa BF16 terms of A   */
/* and pb of B and the products a_i b_j with i < pa, j < pb and i + j <= 2 */
/* (bins 0-2); its bins and their order are those of x6 (x3 when both    */
/* counts are at most 2), an absent product being a +0 chain.             */
static int per_operand(int v)
{
    return v == 12 || v == 13 || v == 21 || v == 23 || v == 31 || v == 32;
}

static int variant_ok(int v)
{
    return v == 1 || v == 3 || v == 6 || v == 7 || v == 8 || v == 9 || per_operand(v);
}

/* Which (i,j) partial inner products a variant needs (Sec. II-D). */
static int needs(int v, int i, int j)
{
    int lvl = i + j;
    if (per_operand(v)) return i < v / 10 && j < v % 10 && lvl <= 2;
    if (v == 1) return lvl == 0;
    if (v == 3) return lvl <= 1 && i <= 1 && j <= 1;
    if (v == 6) return lvl <= 2;
    if (v == 7) return lvl <= 2 || (i == 1 && j == 2);
    if (v == 8) return lvl <= 3;
    return 1;
}

/* Sec. II-D: bins of equal level, then the final FP32 sum, smallest    */
/* first.  Z[i][j] holds the FP32 partial inner products.               */
static float combine_bins(int v, float Z[3][3])
{
    if (per_operand(v)) v = (v / 10 <= 2 && v % 10 <= 2) ? 3 : 6;
    float Z0 = Z[0][0];
    if (v == 1) return Z0;
    float Z1 = Z[0][1] + Z[1][0];
    if (v == 3) return Z0 + Z1;
    float Z2 = Z[0][2] + (Z[1][1] + Z[2][0]);
    if (v == 6) return Z0 + (Z1 + Z2);
    if (v == 7) return Z0 + (Z1 + (Z2 + Z[1][2]));
    float Z3 = Z[1][2] + Z[2][1];
    if (v == 8) return Z0 + (Z1 + (Z2 + Z3));
    float Z4 = Z[2][2];
    return Z0 + (Z1 + (Z2 + (Z3 + Z4)));
}

/* Same combination with every bin and the final sum in FP64 (the "d"  */
/* option of the Sec. IV-A GEMM); the partial products stay FP32 chains.*/
static double combine_bins_f64(int v, float Z[3][3])
{
    if (per_operand(v)) v = (v / 10 <= 2 && v % 10 <= 2) ? 3 : 6;
    double Z0 = Z[0][0];
    if (v == 1) return Z0;
    double Z1 = (double)Z[0][1] + (double)Z[1][0];
    if (v == 3) return Z0 + Z1;
    double Z2 = (double)Z[0][2] + ((double)Z[1][1] + (double)Z[2][0]);
    if (v == 6) return Z0 + (Z1 + Z2);
    if (v == 7) return Z0 + (Z1 + (Z2 + (double)Z[1][2]));
    double Z3 = (double)Z[1][2] + (double)Z[2][1];
    if (v == 8) return Z0 + (Z1 + (Z2 + Z3));
    double Z4 = Z[2][2];
    return Z0 + (Z1 + (Z2 + (Z3 + Z4)));
}

/* BLAS-style epilogue (R-epi). */
static float epilogue(float alpha, float X, float beta, float c)
{
    if (beta == 0.0f) return alpha * X;
    return fmaf(alpha, X, beta * c);
}

/* The split planes of an M x K row-major matrix, stored as floats      */
/* (each value is exactly a BF16 number), plane p at P + p*M*K.         */
static float *split_planes_rows(const float *A, int64_t M, int64_t K,
                                int64_t lda)
{
    float *P = (float *)malloc(sizeof(float) * 3 * (size_t)M * (size_t)K);
    if (!P) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k) {
            uint16_t h0, h1, h2;
            split_one(A[i * lda + k], &h0, &h1, &h2);
            size_t o = (size_t)i * K + k;
            P[o] = orc_bf16_to_f32(h0);
            P[(size_t)M * K + o] = orc_bf16_to_f32(h1);
            P[2 * (size_t)M * K + o] = orc_bf16_to_f32(h2);
        }
    return P;
}

/* Split planes of the columns of a K x N row-major matrix, stored     */
/* column by column (N x K) so that every inner product reads both      */
/* operands with unit stride.  Only the storage differs; the values and */
/* the order of operations are those of Sec. II-D.                      */
static float *split_planes_cols(const float *B, int64_t K, int64_t N,
                                int64_t ldb)
{
    float *P = (float *)malloc(sizeof(float) * 3 * (size_t)N * (size_t)K);
    if (!P) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        for (int64_t k = 0; k < K; ++k) {
            uint16_t h0, h1, h2;
            split_one(B[k * ldb + j], &h0, &h1, &h2);
            size_t o = (size_t)j * K + k;
            P[o] = orc_bf16_to_f32(h0);
            P[(size_t)N * K + o] = orc_bf16_to_f32(h1);
            P[2 * (size_t)N * K + o] = orc_bf16_to_f32(h2);
        }
    return P;
}

/* Sec. II-D: the partial inner products of one output entry.           */
/* x-planes: row of A (plane stride xs), y-planes: column of B.          */
static void partials(int v, int64_t K, const float *x, size_t xs,
                     const float *y, size_t ys, float Z[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Z[i][j] = 0.0f;
            if (!needs(v, i, j)) continue;
            const float *xi = x + (size_t)i * xs;
            const float *yj = y + (size_t)j * ys;
            float acc = 0.0f;
            for (int64_t l = 0; l < K; ++l)
                acc = fmaf(xi[l], yj[l], acc);
            Z[i][j] = acc;
        }
}

/* ------------------------------------------------------------------ */
/* Split GEMM (Sec. IV-A): C = alpha * (A x B) + beta * C, row-major.   */
/* fp64_sum != 0 selects the "d" option (bins summed in FP64).          */
/* Returns 0, or a negative argument index on invalid input.            */
/* ------------------------------------------------------------------ */
int orc_gemm_ex(int variant, int fp64_sum, int64_t M, int64_t N, int64_t K,
                float alpha, const float *A, int64_t lda, const float *B,
                int64_t ldb, float beta, float *C, int64_t ldc)
{
    if (!variant_ok(variant)) return -1;
    if (M < 0) return -3;
    if (N < 0) return -4;
    if (K < 0) return -5;
    if (M == 0 || N == 0) return 0;
    float *PA = split_planes_rows(A, M, K, lda);
    float *PB = split_planes_cols(B, K, N, ldb);
    if (!PA || !PB) { free(PA); free(PB); return -100; }
    size_t xs = (size_t)M * K, ys = (size_t)N * K;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            float Z[3][3];
            partials(variant, K, PA + (size_t)i * K, xs, PB + (size_t)j * K,
                     ys, Z);
            float X = fp64_sum ? (float)combine_bins_f64(variant, Z)
                               : combine_bins(variant, Z);
            C[i * ldc + j] = epilogue(alpha, X, beta, C[i * ldc + j]);
        }
    free(PA);
    free(PB);
    return 0;
}

int orc_gemm(int variant, int64_t M, int64_t N, int64_t K, float alpha,
             const float *A, int64_t lda, const float *B, int64_t ldb,
             float beta, float *C, int64_t ldc)
{
    return orc_gemm_ex(variant, 0, M, N, K, alpha, A, lda, B, ldb, beta, C,
                       ldc);
}

/* The nine FP32 partial inner products Z^(i,j) of one entry, for       */
/* white-box tests of Sec. II-D/II-E.  Z is 3x3 row-major.              */
int orc_dot_partials(int64_t K, const float *x, int64_t incx, const float *y,
                     int64_t incy, float *Z)
{
    if (K < 0) return -1;
    float *px = (float *)malloc(sizeof(float) * 3 * (size_t)(K ? K : 1));
    float *py = (float *)malloc(sizeof(float) * 3 * (size_t)(K ? K : 1));
    if (!px || !py) { free(px); free(py); return -100; }
    for (int64_t l = 0; l < K; ++l) {
        uint16_t h[3], g[3];
        split_one(x[l * incx], &h[0], &h[1], &h[2]);
        split_one(y[l * incy], &g[0], &g[1], &g[2]);
        for (int p = 0; p < 3; ++p) {
            px[(size_t)p * K + l] = orc_bf16_to_f32(h[p]);
            py[(size_t)p * K + l] = orc_bf16_to_f32(g[p]);
        }
    }
    float Zl[3][3];
    partials(9, K, px, (size_t)K, py, (size_t)K, Zl);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Z[i * 3 + j] = Zl[i][j];
    free(px);
    free(py);
    return 0;
}

/* Selected entries C[rows[t], cols[t]] of the split GEMM A x B         */
/* (alpha = 1, beta = 0), for parity sampling of large products.        */
int orc_gemm_entries(int variant, int64_t K, const float *A, int64_t lda,
                     const float *B, int64_t ldb, int64_t count,
                     const int64_t *rows, const int64_t *cols, float *out)
{
    if (!variant_ok(variant)) return -1;
    if (K < 0) return -2;
#pragma omp parallel
    {
        float *x = (float *)malloc(sizeof(float) * 3 * (size_t)(K ? K : 1));
        float *y = (float *)malloc(sizeof(float) * 3 * (size_t)(K ? K : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < count; ++t) {
            const float *ar = A + rows[t] * lda;
            for (int64_t l = 0; l < K; ++l) {
                uint16_t h[3], g[3];
                split_one(ar[l], &h[0], &h[1], &h[2]);
                split_one(B[l * ldb + cols[t]], &g[0], &g[1], &g[2]);
                for (int p = 0; p < 3; ++p) {
                    x[(size_t)p * K + l] = orc_bf16_to_f32(h[p]);
                    y[(size_t)p * K + l] = orc_bf16_to_f32(g[p]);
                }
            }
            float Z[3][3];
            partials(variant, K, x, (size_t)K, y, (size_t)K, Z);
            out[t] = combine_bins(variant, Z);
        }
        free(x);
        free(y);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sec. II-C: the reference FP32 computation, one FMA per term.         */
/* ------------------------------------------------------------------ */
int orc_sgemm(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
              int64_t lda, const float *B, int64_t ldb, float beta, float *C,
              int64_t ldc)
{
    if (M < 0) return -1;
    if (N < 0) return -2;
    if (K < 0) return -3;
    if (M == 0 || N == 0) return 0;
    float *BT = (float *)malloc(sizeof(float) * (size_t)N * (size_t)(K ? K : 1));
    if (!BT) return -100;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        for (int64_t k = 0; k < K; ++k) BT[(size_t)j * K + k] = B[k * ldb + j];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            const float *x = A + i * lda;
            const float *y = BT + (size_t)j * K;
            float Z = 0.0f;
            for (int64_t l = 0; l < K; ++l) Z = fmaf(x[l], y[l], Z);
            C[i * ldc + j] = epilogue(alpha, Z, beta, C[i * ldc + j]);
        }
    free(BT);
    return 0;
}

int orc_sgemm_entries(int64_t K, const float *A, int64_t lda, const float *B,
                      int64_t ldb, int64_t count, const int64_t *rows,
                      const int64_t *cols, float *out)
{
    if (K < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < count; ++t) {
        const float *x = A + rows[t] * lda;
        float Z = 0.0f;
        for (int64_t l = 0; l < K; ++l)
            Z = fmaf(x[l], B[l * ldb + cols[t]], Z);
        out[t] = Z;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Blocked LU with partial pivoting (SGETRF semantics, Sec. I and       */
/* Sec. IV-A), the trailing update done by the split GEMM.              */
/* update_variant: 0 = plain FP32 FMA update (SGETRF), else 1..9.       */
/* ipiv[i] = 0-based row interchanged with row i.  Returns info:        */
/* 0, or c+1 for the first column c with an exactly zero pivot (the     */
/* factorisation is completed regardless), or a negative argument.      */
/* ------------------------------------------------------------------ */
static void swap_rows(float *A, int64_t lda, int64_t r1, int64_t r2,
                      int64_t c0, int64_t c1)
{
    if (r1 == r2) return;
    for (int64_t c = c0; c < c1; ++c) {
        float t = A[r1 * lda + c];
        A[r1 * lda + c] = A[r2 * lda + c];
        A[r2 * lda + c] = t;
    }
}

int orc_lu(int update_variant, int64_t n, float *A, int64_t lda,
           int32_t *ipiv, int64_t nb)
{
    if (update_variant != 0 && !variant_ok(update_variant)) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (nb < 1) return -6;
    int info = 0;
    for (int64_t j = 0; j < n; j += nb) {
        int64_t jb = (n - j < nb) ? n - j : nb;
        /* Panel: columns j..j+jb-1, rows j..n-1, column by column. */
        for (int64_t c = j; c < j + jb; ++c) {
            /* Pivot: first row of largest magnitude (ISAMAX rule). */
            int64_t p = c;
            float best = fabsf(A[c * lda + c]);
            for (int64_t r = c + 1; r < n; ++r) {
                float v = fabsf(A[r * lda + c]);
                if (v > best) { best = v; p = r; }
            }
            ipiv[c] = (int32_t)p;
            swap_rows(A, lda, c, p, 0, n); /* full rows, as LASWP does */
            float piv = A[c * lda + c];
            if (piv == 0.0f) {
                if (info == 0) info = (int)(c + 1);
            } else {
                for (int64_t r = c + 1; r < n; ++r)
                    A[r * lda + c] = A[r * lda + c] / piv;
            }
            /* Rank-1 update of the rest of the panel. */
            for (int64_t r = c + 1; r < n; ++r) {
                float l = A[r * lda + c];
                for (int64_t q = c + 1; q < j + jb; ++q)
                    A[r * lda + q] = fmaf(-l, A[c * lda + q], A[r * lda + q]);
            }
        }
        int64_t rest = n - j - jb;
        if (rest <= 0) continue;
        /* U12 = L11^{-1} A12: unit lower forward substitution, FP32.  */
        for (int64_t r = j + 1; r < j + jb; ++r)
            for (int64_t q = j + jb; q < n; ++q) {
                float s = A[r * lda + q];
                for (int64_t p = j; p < r; ++p)
                    s = fmaf(-A[r * lda + p], A[p * lda + q], s);
                A[r * lda + q] = s;
            }
        /* A22 = A22 - L21 x U12. */
        float *A21 = A + (j + jb) * lda + j;
        float *A12 = A + j * lda + (j + jb);
        float *A22 = A + (j + jb) * lda + (j + jb);
        int rc = update_variant == 0
                     ? orc_sgemm(rest, rest, jb, -1.0f, A21, lda, A12, lda,
                                 1.0f, A22, lda)
                     : orc_gemm(update_variant, rest, rest, jb, -1.0f, A21,
                                lda, A12, lda, 1.0f, A22, lda);
        if (rc) return rc;
    }
    return info;
}

/* ------------------------------------------------------------------ */
/* Single-format LU (the BF16 and FP16 rows of the Sec. IV-B tables):   */
/* the matrix rounded to the format, then right-looking elimination     */
/* with partial pivoting in which every result is rounded to the format */
/* once: multipliers l = R(a / pivot) and updates a = R(a - l u), the   */
/* latter as a fused multiply-add (l u + a is exact in FP64 for these   */
/* formats, so one rounding of the FP64 value is one rounding of the    */
/* exact value).  fmt 1: BF16 (8 significant bits, FP32 exponent       */
/* range), fmt 2: FP16 (11 bits, exponents -14..15); nearest-even,     */
/* gradual underflow, overflow to Inf.                                  */
/* ------------------------------------------------------------------ */
static double round_fmt(double x, int fmt)
{
    const int p = fmt == 1 ? 8 : 11;
    const int emin = fmt == 1 ? -126 : -14, emax = fmt == 1 ? 127 : 15;
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);          /* |x| in [2^(e-1), 2^e) */
    e -= 1;
    if (e < emin) e = emin;      /* subnormal: fixed quantum 2^(emin-p+1) */
    const double q = ldexp(1.0, e - p + 1);
    const double r = rint(x / q) * q;   /* x / q exact (power of two), rint: nearest even */
    if (fabs(r) >= ldexp(1.0, emax + 1)) return copysign(INFINITY, x);
    return r;
}

double orc_round_fmt(double x, int fmt) { return round_fmt(x, fmt); }

int orc_lu_fmt(int fmt, int64_t n, float *A, int64_t lda, int32_t *ipiv)
{
    if (fmt != 1 && fmt != 2) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    int info = 0;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t q = 0; q < n; ++q)
            A[r * lda + q] = (float)round_fmt(A[r * lda + q], fmt);
    for (int64_t c = 0; c < n; ++c) {
        int64_t p = c;
        float best = fabsf(A[c * lda + c]);
        for (int64_t r = c + 1; r < n; ++r) {
            float v = fabsf(A[r * lda + c]);
            if (v > best) { best = v; p = r; }
        }
        ipiv[c] = (int32_t)p;
        swap_rows(A, lda, c, p, 0, n);
        double piv = A[c * lda + c];
        if (piv == 0.0) {
            if (info == 0) info = (int)(c + 1);
            continue;
        }
        for (int64_t r = c + 1; r < n; ++r) {
            double l = round_fmt((double)A[r * lda + c] / piv, fmt);
            A[r * lda + c] = (float)l;
            for (int64_t q = c + 1; q < n; ++q)
                A[r * lda + q] = (float)round_fmt(fma(-l, (double)A[c * lda + q], (double)A[r * lda + q]), fmt);
        }
    }
    return info;
}

/* Solve (LU) x = b in FP32 in place: row interchanges, unit lower      */
/* forward substitution, upper back substitution (division).            */
int orc_lu_solve(int64_t n, const float *LU, int64_t lda,
                 const int32_t *ipiv, float *b)
{
    if (n < 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = ipiv[i];
        if (p != i) { float t = b[i]; b[i] = b[p]; b[p] = t; }
    }
    for (int64_t i = 0; i < n; ++i) {
        float s = b[i];
        for (int64_t p = 0; p < i; ++p) s = fmaf(-LU[i * lda + p], b[p], s);
        b[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        float s = b[i];
        for (int64_t p = i + 1; p < n; ++p) s = fmaf(-LU[i * lda + p], b[p], s);
        b[i] = s / LU[i * lda + i];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sec. III: iterative refinement in residual form.  The cubic work     */
/* (the LU) is low precision; the residual and the update are FP64.     */
/*   x0 = LUsolve32(b)                                                   */
/*   repeat: r = b - A x (FP64, A promoted exactly)                      */
/*           eta = |r|_inf / (|A|_inf |x|_inf + |b|_inf); stop if <= tol */
/*           s = |r|_inf;  d = s * LUsolve32(r / s);  x = x + d (FP64)   */
/* status: 0 converged (eta <= tol), 1 max_iter corrections made without */
/* converging, 2 stagnated (eta failed to decrease on two consecutive    */
/* iterations), 3 non-finite residual.  iters = corrections applied.     */
/* ------------------------------------------------------------------ */
static double inf_norm_vec(int64_t n, const double *v)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (a > m || a != a) m = a;
    }
    return m;
}

double orc_inf_norm_mat(int64_t n, const float *A, int64_t lda)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += fabs((double)A[i * lda + j]);
        if (s > m) m = s;
    }
    return m;
}

void orc_residual(int64_t n, const float *A, int64_t lda, const double *b,
                  const double *x, double *r)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int64_t j = 0; j < n; ++j) s = fma(-(double)A[i * lda + j], x[j], s);
        r[i] = s;
    }
}

int orc_ir(int64_t n, const float *A, int64_t lda, const float *LU,
           int64_t ldlu, const int32_t *ipiv, const double *b, double *x,
           double tol, int max_iter, int *iters_out, double *eta_out,
           int *status_out, double *eta_hist)
{
    if (n < 0) return -1;
    if (max_iter < 0) return -11;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    float *w = (float *)malloc(sizeof(float) * (size_t)(n ? n : 1));
    if (!r || !w) { free(r); free(w); return -100; }
    double normA = orc_inf_norm_mat(n, A, lda);
    double normb = inf_norm_vec(n, b);
    for (int64_t i = 0; i < n; ++i) w[i] = (float)b[i];
    orc_lu_solve(n, LU, ldlu, ipiv, w);
    for (int64_t i = 0; i < n; ++i) x[i] = (double)w[i];
    int status, it = 0, rises = 0;
    double eta, prev_eta = INFINITY;
    for (;;) {
        orc_residual(n, A, lda, b, x, r);
        double rn = inf_norm_vec(n, r);
        double den = normA * inf_norm_vec(n, x) + normb;
        eta = den > 0.0 ? rn / den : rn;
        if (eta_hist) eta_hist[it] = eta;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        if (!isfinite(eta)) { status = 3; break; }
        if (eta <= tol) { status = 0; break; }
        if (it >= max_iter) { status = 1; break; }
        if (rises >= 2) { status = 2; break; }
        double s = rn;
        for (int64_t i = 0; i < n; ++i) w[i] = (float)(r[i] / s);
        orc_lu_solve(n, LU, ldlu, ipiv, w);
        for (int64_t i = 0; i < n; ++i) x[i] += s * (double)w[i];
        ++it;
    }
    *iters_out = it;
    *eta_out = eta;
    *status_out = status;
    free(r);
    free(w);
    return 0;
}


/* ------------------------------------------------------------------ */
/* Sec. III / Sec. IV-B: iterative refinement whose correction equation */
/* A d = r is solved by GMRES preconditioned with the low-precision LU   */
/* (left preconditioning, M = LU), all of GMRES in FP64: the matrix-     */
/* vector product uses A promoted exactly, the preconditioner applies    */
/* the FP32 factors in FP64 arithmetic (row interchanges, unit lower and */
/* upper substitution), Arnoldi with modified Gram-Schmidt, Givens       */
/* rotations on the Hessenberg matrix.  One GMRES cycle of at most       */
/* `restart` steps per refinement step, stopped when the preconditioned  */
/* residual falls below inner_tol times its initial norm.                */
/* Outer loop and status codes as orc_ir; inner_out = total GMRES steps. */
/* ------------------------------------------------------------------ */
static void lu_apply_f64(int64_t n, const float *LU, int64_t lda, const int32_t *ipiv,
                         double *v)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = ipiv[i];
        if (p != i) { double t = v[i]; v[i] = v[p]; v[p] = t; }
    }
    for (int64_t i = 0; i < n; ++i) {
        double s = v[i];
        for (int64_t p = 0; p < i; ++p) s = fma(-(double)LU[i * lda + p], v[p], s);
        v[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = v[i];
        for (int64_t p = i + 1; p < n; ++p) s = fma(-(double)LU[i * lda + p], v[p], s);
        v[i] = s / (double)LU[i * lda + i];
    }
}

static double dot64(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = fma(a[i], b[i], s);
    return s;
}

int orc_gmres_ir(int64_t n, const float *A, int64_t lda, const float *LU,
                 int64_t ldlu, const int32_t *ipiv, const double *b, double *x,
                 double tol, int max_iter, int restart, double inner_tol,
                 int *iters_out, int *inner_out, double *eta_out, int *status_out,
                 double *eta_hist)
{
    if (n < 0) return -1;
    if (max_iter < 0) return -11;
    if (restart < 1) return -12;
    int m = restart;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *V = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1) * (size_t)(m + 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    float *f = (float *)malloc(sizeof(float) * (size_t)(n ? n : 1));
    if (!r || !V || !w || !H || !cs || !sn || !g || !y || !f) {
        free(r); free(V); free(w); free(H); free(cs); free(sn); free(g); free(y); free(f);
        return -100;
    }
    double normA = orc_inf_norm_mat(n, A, lda);
    double normb = inf_norm_vec(n, b);
    for (int64_t i = 0; i < n; ++i) f[i] = (float)b[i];
    orc_lu_solve(n, LU, ldlu, ipiv, f);
    for (int64_t i = 0; i < n; ++i) x[i] = (double)f[i];
    int status, it = 0, rises = 0, inner_total = 0;
    double eta, prev_eta = INFINITY;
    for (;;) {
        orc_residual(n, A, lda, b, x, r);
        double rn = inf_norm_vec(n, r);
        double den = normA * inf_norm_vec(n, x) + normb;
        eta = den > 0.0 ? rn / den : rn;
        if (eta_hist) eta_hist[it] = eta;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        if (!isfinite(eta)) { status = 3; break; }
        if (eta <= tol) { status = 0; break; }
        if (it >= max_iter) { status = 1; break; }
        if (rises >= 2) { status = 2; break; }
        /* GMRES on M^{-1} A d = M^{-1} r, d0 = 0 */
        for (int64_t i = 0; i < n; ++i) V[i] = r[i];
        lu_apply_f64(n, LU, ldlu, ipiv, V);
        double beta = sqrt(dot64(n, V, V));
        int k = 0;
        if (beta > 0.0) {
            for (int64_t i = 0; i < n; ++i) V[i] /= beta;
            for (int j = 0; j <= m; ++j) g[j] = 0.0;
            g[0] = beta;
            for (k = 0; k < m; ++k) {
                double *vk = V + (size_t)k * n;
                /* w = M^{-1} A v_k */
                for (int64_t i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int64_t c = 0; c < n; ++c) s = fma((double)A[i * lda + c], vk[c], s);
                    w[i] = s;
                }
                lu_apply_f64(n, LU, ldlu, ipiv, w);
                /* modified Gram-Schmidt */
                for (int j = 0; j <= k; ++j) {
                    double h = dot64(n, w, V + (size_t)j * n);
                    H[j * m + k] = h;
                    for (int64_t i = 0; i < n; ++i) w[i] = fma(-h, V[(size_t)j * n + i], w[i]);
                }
                double hn = sqrt(dot64(n, w, w));
                H[(k + 1) * m + k] = hn;
                /* earlier rotations on the new column, then a new rotation */
                for (int j = 0; j < k; ++j) {
                    double a = H[j * m + k], c2 = H[(j + 1) * m + k];
                    H[j * m + k] = cs[j] * a + sn[j] * c2;
                    H[(j + 1) * m + k] = -sn[j] * a + cs[j] * c2;
                }
                double a = H[k * m + k], c2 = H[(k + 1) * m + k];
                double rho = hypot(a, c2);
                cs[k] = rho > 0.0 ? a / rho : 1.0;
                sn[k] = rho > 0.0 ? c2 / rho : 0.0;
                H[k * m + k] = rho;
                H[(k + 1) * m + k] = 0.0;
                g[k + 1] = -sn[k] * g[k];
                g[k] = cs[k] * g[k];
                ++inner_total;
                if (hn > 0.0 && k + 1 < m + 1)
                    for (int64_t i = 0; i < n; ++i) V[(size_t)(k + 1) * n + i] = w[i] / hn;
                if (fabs(g[k + 1]) <= inner_tol * beta || hn == 0.0) { ++k; break; }
            }
            /* y = H(1:k,1:k) \ g(1:k); d = V y */
            for (int j = k - 1; j >= 0; --j) {
                double s = g[j];
                for (int q = j + 1; q < k; ++q) s -= H[j * m + q] * y[q];
                y[j] = s / H[j * m + j];
            }
            for (int j = 0; j < k; ++j)
                for (int64_t i = 0; i < n; ++i) x[i] = fma(y[j], V[(size_t)j * n + i], x[i]);
        }
        ++it;
    }
    *iters_out = it;
    *inner_out = inner_total;
    *eta_out = eta;
    *status_out = status;
    free(r); free(V); free(w); free(H); free(cs); free(sn); free(g); free(y); free(f);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
