/*
 * bfx -- FP32-accurate linear algebra from BF16 pieces on AMD MI355X (gfx950).
 *
 * C ABI of libbfx.so.  Method: G. Henry, P. T. P. Tang, A. Heinecke,
 * "Leveraging the bfloat16 Artificial Intelligence Datatype For
 * Higher-Precision Computations" (2019).
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major FP32 with a leading dimension (elements between
 *     consecutive rows), as PyTorch lays them out.
 *   - Every pointer named A, B, C, a, b*, x, ipiv, info, ws is a DEVICE pointer
 *     unless the argument documentation says "host".  The caller owns all of
 *     them; the library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     calls are asynchronous on that stream; no call synchronises the device
 *     except where documented.
 *   - Return value: BFX_OK (0); -i when the i-th argument (1-based) is
 *     invalid, in the style of LAPACK's xerbla; BFX_E_HIP when the HIP runtime
 *     reported an error (the message is in bfx_last_error_string()).
 *   - Numerical status (a zero pivot, refinement that did not converge) is not
 *     an error return: it is written to device memory (info, bfx_ir_result).
 *   - No exception crosses this interface.  Entry points without a plan are
 *     reentrant; a plan must be launched from one stream at a time.
 *
 * Number conversion used throughout (Sec. I, Sec. II-A): FP32 -> BF16 rounds to
 * nearest, ties to even; a finite value that would round past the largest
 * BF16 saturates to +-0x7F7F; NaN becomes the quiet NaN 0x7FC0 of its sign;
 * subnormals are kept (no flush to zero).
 */
#ifndef BFX_H
#define BFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFX_OK 0
#define BFX_E_HIP (-1000)       /* HIP runtime error; see bfx_last_error_string */
#define BFX_E_WORKSPACE (-1001) /* workspace pointer NULL or too small */
#define BFX_E_INTERNAL (-1002)  /* a kernel's own bounded wait expired */

/* Library version, as 10000*major + 100*minor + patch. */
int bfx_version(void);

/* Text of the last error recorded by this thread (never NULL). */
const char *bfx_last_error_string(void);

/* ------------------------------------------------------------------------ */
/* Split (Sec. II-A): b0 = (B16)a, b1 = (B16)(a - b0), b2 = (B16)(a - b0 - b1) */
/* ------------------------------------------------------------------------ */
/* a:  n FP32 values (device).  nterms: 2 or 3.
 * b0, b1, b2: n BF16 bit patterns each (device, uint16); b2 is ignored and may
 * be NULL when nterms == 2.  b0 + b1 + b2 == a exactly for a = +-0 and
 * 2^-110 <= |a| <= FLT_MAX (Sec. II-F); for Inf/NaN, b1 = b2 = +0.
 * Errors: -2 if n < 0, -3 if nterms not in {2,3}, -1/-4/-5/-6 for a NULL
 * required pointer (only checked when n > 0). */
int bfx_split_f32(const float *a, int64_t n, int nterms, uint16_t *b0,
                  uint16_t *b1, uint16_t *b2, void *stream);

/* ------------------------------------------------------------------------ */
/* Split-BF16 GEMM (Sec. II-D, II-G, IV-A):                                  */
/*   C = alpha * (A x B) + beta * C,  A: M x K, B: K x N, C: M x N.          */
/* Both operands are split into BF16 terms inside the kernel; the partial    */
/* products run on BF16 MFMA with FP32 accumulation, bins added smallest     */
/* first.  variant = number of BF16 products per scalar product:             */
/*   3 -> Z0 + Z1            (two terms each)                                */
/*   6 -> Z0 + (Z1 + Z2)     (three terms, the paper's six-product sum)      */
/*   7 -> x6 plus A1 B2 (half of bin 3)                                      */
/*   8 -> Z0 + (Z1 + (Z2 + Z3))  (bins 0-3, eight products)                 */
/*   9 -> Z0 + (Z1 + (Z2 + (Z3 + Z4)))  (all nine products)                  */
/*   1 -> Z0 (one term each)                                                 */
/* Per-operand split counts (Sec. II-G, a different number of terms per      */
/* operand): variant 10 * pa + pb in {12, 13, 21, 23, 31, 32} takes pa terms */
/* of A and pb of B and the products a_i b_j with i < pa, j < pb, i + j <= 2 */
/* (bins 0-2; e.g. 23 = a0 b0; a0 b1, a1 b0; a0 b2, a1 b1: five products).   */
/* They run on the general engine (in-kernel split) or, with the workspace  */
/* of bfx_gemm_ws_size, on pre-split operands; accuracy as variant 1 when    */
/* min(pa, pb) = 1 and as variant 3 when it is 2, plus what the dropped      */
/* terms of the operand with more terms contribute.                          */
/* The products of bins 1.. accumulate in one FP32 sum, smallest bin first;  */
/* Z0 in another; X = Z0 + that sum.                                         */
/* beta == 0: C is not read (it may hold NaN).  lda >= max(1,K),             */
/* ldb >= max(1,N), ldc >= max(1,N).  ws/ws_bytes: device workspace of at    */
/* least bfx_gemm_ws_size(...) bytes (NULL allowed when that is 0); the      */
/* library uses it for split-K partial sums of long inner dimensions, and    */
/* on large problems (>= 256 output tiles of 128 x 128, K >= 512) for the    */
/* operands' BF16 planes: with a 16-byte aligned workspace of at least       */
/* bfx_gemm_ws_size bytes, A and B are split once (bfx_split_blocks) and     */
/* the products run on the planes (bfx_gemm_blocks); with a smaller one the  */
/* split happens inside the GEMM kernel.  Both give the same bits.           */
/* Accuracy: |C - alpha A B| <= 2K 2^-24 |alpha| |A||B| componentwise for    */
/* variants 6-9 (K >= 8), plus 3*2^-16 |alpha||A||B| for variant 3 and       */
/* 3*2^-8 |alpha||A||B| for variant 1.                                       */
/* Errors: -1 variant, -2/-3/-4 negative sizes, -6/-8/-11 NULL operands,     */
/* -7/-9/-12 leading dimensions, -14 workspace too small (BFX_E_WORKSPACE is */
/* not used for this case so the argument is named).                         */
int bfx_gemm(int variant, int64_t M, int64_t N, int64_t K, float alpha,
             const float *A, int64_t lda, const float *B, int64_t ldb,
             float beta, float *C, int64_t ldc, void *ws, size_t ws_bytes,
             void *stream);

/* bfx_gemm with options.  flags: 0 or BFX_GEMM_FP64_SUM, the "d" option of  */
/* Sec. IV-A: the final sum X = Z0 + (bins 1..) and the alpha/beta           */
/* combination are formed in FP64 and rounded to FP32 once.  The two FP32   */
/* accumulators are added exactly in FP64, so with alpha = 1 and beta = 0   */
/* the result has the bits of bfx_gemm; otherwise it avoids the rounding of */
/* X and of beta C.  Errors as bfx_gemm, and -2 for unknown flags (the       */
/* negative-size codes of M, N, K stay -2, -3, -4 after the flags check).    */
#define BFX_GEMM_FP64_SUM 1
int bfx_gemm_ex(int variant, int flags, int64_t M, int64_t N, int64_t K,
                float alpha, const float *A, int64_t lda, const float *B,
                int64_t ldb, float beta, float *C, int64_t ldc, void *ws,
                size_t ws_bytes, void *stream);

/* Workspace bytes bfx_gemm uses for this shape: the split-K partial sums,  */
/* or the pre-split planes of both operands; 0 when it needs neither.        */
size_t bfx_gemm_ws_size(int variant, int64_t M, int64_t N, int64_t K);

/* For callers that cannot allocate device memory (code under HIP graph      */
/* capture, tight serving loops, harnesses that forbid hipMalloc): bfx_gemm   */
/* without a workspace argument.  Same arguments (minus ws, ws_bytes), same   */
/* kernels, same bits and the same error codes as bfx_gemm.  The workspace is */
/* a fixed device array inside the library, bfx_gemm_noalloc_scratch_bytes() */
/* (64 MiB) long, that every GPU the library runs on holds from the first    */
/* call on it until the process ends.  It holds the split-K partial sums of  */
/* long inner dimensions and, when they fit, the pre-split planes of large   */
/* products (when they do not, the split happens inside the GEMM kernel, as  */
/* in bfx_gemm with a small workspace).  A shape whose split-K partial sums   */
/* exceed the scratch is rejected with BFX_E_WORKSPACE before any launch     */
/* (the message names both sizes).  The call allocates nothing, on the host  */
/* or the device.  All calls on one GPU share that GPU's scratch and leave   */
/* their contents in it: calls that overlap in time on one GPU (different    */
/* streams, or different host threads) race and give wrong results; calls   */
/* ordered on one stream are safe.                                           */
int bfx_gemm_noalloc(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                     const float *A, int64_t lda, const float *B, int64_t ldb,
                     float beta, float *C, int64_t ldc, void *stream);

/* Size of bfx_gemm_noalloc's fixed device scratch in bytes. */
size_t bfx_gemm_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------ */
/* Pre-split operands (Sec. II-A once per operand, then Sec. II-D, II-G).   */
/* Splitting costs O(N^2) against the O(N^3) products (Sec. V), so an        */
/* operand used in several products can be split once and reused.           */
/* ------------------------------------------------------------------------ */
/* Block layout: nterms planes, plane t at element t * ceil(R/128) * KS *    */
/* 4096 (KS = ceil(K/32)).  Plane t holds the t-th BF16 term of every value  */
/* in 128 x 32 blocks of 4096 BF16: block (r, s) at element (r * KS + s) *   */
/* 4096 covers rows 128 r .. 128 r + 127 (A rows; B columns) and k = 32 s .. */
/* 32 s + 31, zeros outside R x K.  Inside a block, row n (0..127) is stored */
/* at 64-byte row n ^ ((n >> 2) & 1) and its 16-byte chunk c (k = 8c..8c+7) */
/* at chunk position c ^ ((n >> 1) & 3) of that row.                        */
/* Bytes of one operand's planes (0 for invalid arguments or R, K <= 0).   */
size_t bfx_split_blocks_size(int nterms, int64_t R, int64_t K);

/* Split one FP32 operand into that layout, exactly (bfx_split_f32's terms).  */
/* trans = 0: X is R x K row-major (the A operand, R = M), ld >= max(1,K);    */
/* trans = 1: X is K x R row-major (the B operand, R = N), ld >= max(1,R).    */
/* nterms: 1, 2 or 3 (variants 1, 3 and 6-9 read 1, 2 and 3 terms; the     */
/* per-operand variants 10 pa + pb read max(pa, pb) terms of both operands). */
/* out: device, 16-byte aligned, out_bytes >= bfx_split_blocks_size.          */
/* Errors: -1 nterms, -2 trans, -3 R < 0, -4 K < 0 or K, R too large for the  */
/* 32-bit block offsets (ceil(K/32) * 8192 >= 2^31), -5 X NULL, -6 ld,        */
/* -7 out NULL or misaligned, -8 out_bytes too small.  R == 0 or K == 0: no   */
/* work.                                                                      */
int bfx_split_blocks(int nterms, int trans, int64_t R, int64_t K, const float *X,
                     int64_t ld, uint16_t *out, size_t out_bytes, void *stream);

/* C = alpha * (A x B) + beta * C from pre-split operands: Ab from            */
/* bfx_split_blocks(P, 0, M, K, A, ...), Bb from bfx_split_blocks(P, 1, N, K,  */
/* B, ...), P = 1, 2, 3 for variant 1, 3, 6-9, P = max(pa, pb) for variant   */
/* 10 pa + pb (the kernel reads P planes of both).  Same variants, accumulation */
/* order, accuracy and beta rule as bfx_gemm (bitwise equal results).  Ab, Bb  */
/* device, 16-byte aligned, read only; C device, ldc >= max(1,N).  One        */
/* 128 x 128 output tile per workgroup, no workspace.                         */
/* Errors: -1 variant, -2/-3/-4 negative sizes (-4 also for K beyond the       */
/* block offsets), -6/-7 Ab/Bb NULL or misaligned, -9 C NULL, -10 ldc.        */
int bfx_gemm_blocks(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                    const uint16_t *Ab, const uint16_t *Bb, float beta, float *C,
                    int64_t ldc, void *stream);

/* Plain FP32 GEMM on the vector ALU, one rounding per FMA (Sec. II-C): the   */
/* comparator the split variants are measured against.  Without split-K      */
/* (ws size 0) every output is one FMA chain in increasing k; with split-K   */
/* (few output tiles, long K) the chains of each K range are added in a      */
/* fixed order.  Same argument meanings as bfx_gemm without `variant`        */
/* (indices shift down by one); -13 when the workspace is too small.         */
int bfx_sgemm_fp32(int64_t M, int64_t N, int64_t K, float alpha,
                   const float *A, int64_t lda, const float *B, int64_t ldb,
                   float beta, float *C, int64_t ldc, void *ws, size_t ws_bytes,
                   void *stream);

/* Workspace bytes bfx_sgemm_fp32 needs for this shape (0 when no split-K). */
size_t bfx_sgemm_ws_size(int64_t M, int64_t N, int64_t K);

/* ------------------------------------------------------------------------ */
/* Batched uneven GEMMs in one persistent launch (many independent          */
/* instances of the Sec. IV-A GEMM).                                         */
/* ------------------------------------------------------------------------ */
typedef struct bfx_gemm_desc {
    int64_t M, N, K;
    const float *A; int64_t lda;   /* device */
    const float *B; int64_t ldb;   /* device */
    float *C; int64_t ldc;         /* device */
    float alpha, beta;
} bfx_gemm_desc;

typedef struct bfx_plan bfx_plan;

/* Build a plan for `count` problems (descs: HOST array, copied).  The plan
 * picks a tile shape per problem from the tuning table at `tune_table`
 * (a JSON file written by the autotuner: "tile" 0-3 = general engine
 * 64x64/128x128/128x64/64x128, 4-5 = wave-specialised 64x64/128x128;
 * NULL or "" = built-in defaults), orders the tiles longest-first, uploads
 * the work lists, and captures "reset the work counters + persistent
 * kernels" into a HIP graph on first launch: one persistent kernel for the
 * problems the wave-specialised engine takes (K % 4 == 0, A 16-byte aligned
 * with lda % 4 == 0), one for the rest.  A wave-specialised tile asked for a
 * problem it cannot take falls back to the default general tile.  The plan
 * owns its device buffers until bfx_plan_destroy.
 * Errors: -1 variant, -2 count < 0, -3 descs NULL, -4 out NULL, -(100+i)
 * when descriptor i is invalid (sizes, NULL pointers, leading dims). */
int bfx_gemm_batched_plan_create(int variant, int64_t count,
                                 const bfx_gemm_desc *descs,
                                 const char *tune_table, bfx_plan **out);

/* Launch the plan's graph on `stream` (the only host->device crossing). */
int bfx_plan_launch(bfx_plan *plan, void *stream);

/* Same work as bfx_plan_launch, as one kernel launch per problem (the
 * baseline the persistent launch is measured against). */
int bfx_plan_launch_per_problem(bfx_plan *plan, void *stream);

/* Number of tiles and of problems in the plan (host ints). */
int bfx_plan_info(const bfx_plan *plan, int64_t *tiles, int64_t *problems);

int bfx_plan_destroy(bfx_plan *plan);

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting (SGETRF semantics, Sec. I and IV-A): in place,   */
/* P A = L U with L unit lower (below the diagonal) and U upper.  The panel, */
/* the row interchanges and the triangular solve are FP32; every trailing    */
/* update A22 -= L21 U12 is the split GEMM with `variant` products (1, 3, 6, */
/* 9), or, with variant 0, the plain FP32 vector GEMM (bfx_sgemm_fp32): the   */
/* SGEMM-based SGETRF that Sec. IV-A's LU experiment compares against.       */
/* ipiv: n int32 (device), ipiv[i] = 0-based row interchanged with row i.    */
/* info: one int32 (device): 0, or c+1 for the first column c whose pivot is */
/* exactly zero (the factorisation is completed regardless).                 */
/* ws: device workspace of bfx_lu_ws_size(n) bytes.                          */
/* Synchronisation: the host waits for each panel's pivot block before the   */
/* next panel is started only through stream order; the call returns after  */
/* queueing all work.                                                        */
/* Errors: -1 variant, -2 n < 0, -3 A NULL, -4 lda < max(1,n), -5 ipiv NULL, */
/* -6 info NULL, -8 workspace too small.                                     */
int bfx_lu_factor(int variant, int64_t n, float *A, int64_t lda,
                  int32_t *ipiv, int32_t *info, void *ws, size_t ws_bytes,
                  void *stream);

size_t bfx_lu_ws_size(int64_t n);

/* ------------------------------------------------------------------------ */
/* Iterative refinement in residual form (Sec. III):                          */
/*   x0 = LUsolve32(b);  repeat  r = b - A x (FP64, A promoted exactly),      */
/*   eta = |r|_inf / (|A|_inf |x|_inf + |b|_inf), stop when eta <= tol;       */
/*   s = |r|_inf, d = s * LUsolve32(r / s) (FP32 solves), x += d (FP64).      */
/* ------------------------------------------------------------------------ */
typedef struct bfx_ir_opts {
    double tol;        /* normwise backward error target (default 1e-14) */
    int32_t max_iter;  /* maximum number of corrections (default 30) */
    int32_t reserved;
} bfx_ir_opts;

typedef struct bfx_ir_result {
    int32_t iters;     /* corrections applied */
    int32_t status;    /* 0 converged, 1 max_iter reached (also: not yet
                          decided), 2 stagnated (eta did not decrease twice
                          in a row), 3 non-finite residual, 4 a kernel's
                          bounded wait expired (internal error) */
    double eta;        /* backward error of the returned x */
} bfx_ir_result;

/* A: the FP32 matrix that was factored (n x n, lda), LU/ipiv: the output of
 * bfx_lu_factor (ldlu), b: n FP64 (device), x: n FP64 (device, output),
 * opts: HOST pointer (NULL = defaults), res: DEVICE pointer to one
 * bfx_ir_result, written by the convergence test on the device.
 * Asynchronous: the call queues the whole solve on `stream` and returns
 * without waiting; the test that stops the refinement runs on the device,
 * and the steps queued after it return at once.  Read x and *res after the
 * stream has reached this point.  ws: device workspace of bfx_ir_ws_size(n)
 * bytes, in use until then.
 * Errors: -1 n, -2 A, -3 lda, -4 LU, -5 ldlu, -6 ipiv, -7 b, -8 x,
 * -9 opts (tol < 0 or max_iter < 0), -10 res, -12 workspace. */
int bfx_ir_solve(int64_t n, const float *A, int64_t lda, const float *LU,
                 int64_t ldlu, const int32_t *ipiv, const double *b, double *x,
                 const bfx_ir_opts *opts, bfx_ir_result *res, void *ws,
                 size_t ws_bytes, void *stream);

size_t bfx_ir_ws_size(int64_t n);

/* ------------------------------------------------------------------------ */
/* Refinement with GMRES as the correction solver (Sec. III, Sec. IV-B):      */
/* each step solves A d = r with GMRES on M^{-1} A d = M^{-1} r, M = the      */
/* low-precision LU, in FP64 (the preconditioner applies the FP32 factors in  */
/* FP64 arithmetic); one GMRES cycle of at most `restart` steps per           */
/* refinement step, stopped when the preconditioned residual falls below      */
/* inner_tol times its initial norm.  The residual, update, stopping rule and */
/* status codes are those of bfx_ir_solve.  This is the variant that reaches  */
/* an FP64-level backward error when kappa(A) * 2^-24 is well above 1.        */
/* ------------------------------------------------------------------------ */
typedef struct bfx_gmres_opts {
    double tol;         /* backward error target (default 1e-14) */
    int32_t max_iter;   /* refinement steps (default 10) */
    int32_t restart;    /* GMRES steps per refinement step (default 50) */
    double inner_tol;   /* relative GMRES tolerance (default 1e-8) */
} bfx_gmres_opts;

typedef struct bfx_gmres_result {
    int32_t iters;      /* refinement steps */
    int32_t inner;      /* total GMRES steps */
    int32_t status;     /* as bfx_ir_result */
    int32_t reserved;
    double eta;
} bfx_gmres_result;

/* Arguments as bfx_ir_solve; res is a DEVICE pointer and the call is
 * asynchronous in the same way: GMRES orthogonalises the basis (classical
 * Gram-Schmidt twice), applies the Givens rotations of its Hessenberg
 * least-squares problem and solves it on the device.  The host queues
 * max_iter refinement steps of `restart` GMRES steps each; every step after
 * a cycle or the refinement has stopped costs one empty launch per kernel.
 * ws: bfx_gmres_ir_ws_size(n, restart) bytes (the basis, (restart+1) n
 * doubles, and the rotated Hessenberg matrix, restart^2 doubles, dominate).
 * Errors as bfx_ir_solve; -9 also for restart < 1 or a negative inner_tol. */
int bfx_gmres_ir_solve(int64_t n, const float *A, int64_t lda, const float *LU,
                       int64_t ldlu, const int32_t *ipiv, const double *b,
                       double *x, const bfx_gmres_opts *opts,
                       bfx_gmres_result *res, void *ws, size_t ws_bytes,
                       void *stream);

size_t bfx_gmres_ir_ws_size(int64_t n, int restart);

/* FP32 solve with an LU from bfx_lu_factor: rhs (n FP32, device) is
 * overwritten by (LU)^-1 P rhs.  ws: bfx_ir_ws_size(n) bytes.  Errors as
 * bfx_ir_solve for the shared arguments. */
int bfx_lu_solve_f32(int64_t n, const float *LU, int64_t ldlu,
                     const int32_t *ipiv, float *rhs, void *ws,
                     size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Many independent solves A x = b in one persistent, graph-captured launch:  */
/* split-BF16 blocked LU (Sec. I, IV-A) + FP64-residual refinement (Sec. III) */
/* for each problem, one workgroup per problem, longest problems first.  A    */
/* problem that LU-IR leaves unconverged (max_iter reached or stagnation)     */
/* is solved again from x0 = LUsolve(b) with GMRES-IR (Sec. III, Sec. IV-B)   */
/* when gmres_max_iter > 0, in the same workgroup.                            */
/* ------------------------------------------------------------------------ */
typedef struct bfx_solve_desc {
    int64_t n;                     /* 1 <= n <= 1024 */
    const float *A; int64_t lda;   /* device, row-major FP32 n x n, not modified */
    const double *b;               /* device, n FP64 */
    double *x;                     /* device, n FP64, output */
} bfx_solve_desc;

typedef struct bfx_batched_solve_opts {
    double tol;              /* backward error target (default 1e-14) */
    int32_t max_iter;        /* LU-IR corrections (default 30) */
    int32_t gmres_max_iter;  /* GMRES-IR steps after LU-IR fails (default 10;
                                0 = LU-IR only) */
    int32_t restart;         /* GMRES steps per cycle (default 0 = n, a full
                                Krylov space) */
    double inner_tol;        /* relative GMRES tolerance (default 1e-8) */
    int32_t lu_format;       /* 0: split-BF16 blocked LU with `variant` (default);
                                1, 2: single-format BF16 / FP16 LU (the Sec. IV-B
                                tables): the matrix and every multiplier and
                                update rounded once to the format */
    int32_t mode;            /* 0: LU-IR, GMRES-IR when it fails (default);
                                1: GMRES-IR from the start (needs
                                gmres_max_iter > 0) */
} bfx_batched_solve_opts;

typedef struct bfx_solve_plan bfx_solve_plan;

/* descs: HOST array (copied).  opts: HOST pointer (NULL = defaults).  The
 * plan owns the factor storage (sum of n^2 FP32), the pivots, the
 * per-problem results and, when GMRES is enabled, one scratch slice per
 * workgroup for the GMRES basis and Hessenberg matrix ((m+1) nmax + m^2
 * doubles, m = restart or nmax) until bfx_solve_plan_destroy.  The stopping
 * rule and status codes are those of bfx_ir_solve.
 * Errors: -1 variant, -2 count < 0, -3 descs NULL, -4 opts invalid, -5 out
 * NULL, -(100+i) when descriptor i is invalid. */
int bfx_lu_ir_batched_plan_create(int variant, int64_t count,
                                  const bfx_solve_desc *descs,
                                  const bfx_batched_solve_opts *opts,
                                  bfx_solve_plan **out);

/* All solves as one graph replay on `stream` (asynchronous). */
int bfx_solve_plan_launch(bfx_solve_plan *plan, void *stream);

/* Same solves with bfx_lu_factor + bfx_ir_solve per problem, queued one
 * after another on `stream` (the baseline the persistent launch is measured
 * against; LU-IR only). */
int bfx_solve_plan_launch_per_problem(bfx_solve_plan *plan, void *stream);

/* Synchronises the device and copies the per-problem results (iters =
 * refinement steps of LU-IR and GMRES-IR together, inner = GMRES steps,
 * status, eta) and LU info (HOST arrays of `count` entries, in descriptor
 * order; either may be NULL). */
int bfx_solve_plan_results(const bfx_solve_plan *plan, bfx_gmres_result *results,
                           int32_t *info);

/* Synchronises the device and copies problem `index`'s factors (n x n FP32,
 * row-major, L below the diagonal, U on and above) and pivots to HOST arrays
 * (either may be NULL).  Errors: -1 plan NULL, -2 index out of range. */
int bfx_solve_plan_factors(const bfx_solve_plan *plan, int64_t index, float *lu,
                           int32_t *ipiv);

int bfx_solve_plan_destroy(bfx_solve_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* BFX_H */
