/* blws.h - C ABI of the MI355X BLWS singular-value-thresholding library.
 *
 * The library computes the singular value thresholding step of nuclear norm
 * minimisation, A = T_eps(W) = U Theta_eps(S) V^T (Lin & Wei, Eq. (3)-(4)),
 * with a partial SVD by block Lanczos with a warm start (BLWS: Sec. 4,
 * Algorithms 2-3 with k = 2 as in Sec. 4.1, block width following the
 * predicted rank as in Sec. 4.2), and the inexact-ALM solvers that host it:
 * robust PCA (Eq. (1) relaxed to nuclear + l1 norms) and matrix completion
 * (Eq. (2) relaxed to the nuclear norm), as in the experiments of Sec. 5.
 *
 * Conventions for every call:
 *  - Matrices are dense and row-major: element (i, j) at p[i * ld + j], with
 *    ld >= number of columns. All matrix and vector pointers are DEVICE pointers
 *    unless a parameter says "host". The caller owns every buffer it passes; the
 *    library owns only the context's workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work is
 *    queued on it; the solvers block the calling thread until their result is
 *    complete, blws_svt returns as soon as its work is queued.
 *  - Element type of the W/D/U/V/A/E buffers: double for BLWS_FP64, float for
 *    BLWS_FP32, BLWS_BF16 and BLWS_BF16X3. Singular values S are always double.
 *    In BLWS_FP32 the products with W run on FP32 matrix cores; BLWS_BF16
 *    (robust PCA only) is the precision ladder: the products with W run in BF16
 *    (FP32 accumulation) while the residual is large, then (ladder3_tol > 0) in
 *    split-precision BF16 x 3, then in FP32, and a last reduced-precision
 *    iterate is refined by one FP32 step. BLWS_BF16X3 (blws_svt only) runs the
 *    products of one step in BF16 x 3: W = W_hi + W_lo and the block likewise
 *    split into two BF16 halves, W_hi X_hi + W_hi X_lo + W_lo X_hi on BF16
 *    matrix cores with FP32 accumulation (about 16 significant bits). Gram
 *    matrices, Cholesky factors, the projected SVD and the reconstruction of A
 *    are FP64 in every mode.
 *  - Return value: a blws_status. Arguments are validated before any work is
 *    queued, so an error leaves every output untouched. No call aborts, exits
 *    or throws. blws_last_error() gives a detail message for the last failure.
 *  - Threads: a context may be used by one host thread at a time.
 */
#ifndef BLWS_H
#define BLWS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct blws_ctx_s* blws_ctx;

typedef enum { BLWS_FP64 = 0, BLWS_FP32 = 1, BLWS_BF16 = 2, BLWS_BF16X3 = 3 } blws_precision;

typedef enum {
    BLWS_OK = 0,
    BLWS_NOT_CONVERGED = 1, /* iteration cap reached; outputs hold the last iterate */
    BLWS_EINVAL = -1,       /* bad argument (nothing was queued)                   */
    BLWS_ENOMEM = -2,       /* device workspace allocation failed                  */
    BLWS_EDEVICE = -3,      /* a HIP call failed                                   */
    BLWS_ENUMERIC = -4,     /* NaN or Inf met in the data or a residual            */
    BLWS_EUNSUPPORTED = -5  /* precision or size not supported by this build       */
} blws_status;

/* Options of one BLWS call. */
typedef struct {
    int pow_steps;            /* cold start only: power half-step pairs on V (2)     */
    unsigned long long seed;  /* cold start: seed of the counter-based generator     */
} blws_svt_opts;

/* Options of the inexact-ALM solvers. Defaults from blws_default_alm_opts. */
typedef struct {
    double tol;               /* stop when ||D - A - E||_F / ||D||_F < tol (1e-7)      */
    int max_iter;             /* 1000                                                   */
    double rho;               /* mu <- min(rho mu, mu_bar) (1.5)                        */
    double mu0_scale;         /* mu_0 = mu0_scale / ||D||_2 (1.25)                      */
    double mu_max_factor;     /* mu_bar = mu_max_factor * mu_0 (1e7)                    */
    int sv0;                  /* initial predicted rank (10)                            */
    double sv_step_frac;      /* rank-prediction increment as a fraction of min(m,n)    */
    int b_round;              /* Lanczos block width = predicted rank rounded up (16)   */
    int pow_steps;            /* power half-step pairs of the first (cold) block (2)    */
    unsigned long long seed;  /* counter-based generator seed                           */
    int norm_steps;           /* max BLWS steps for the ||D||_2 estimate (8)            */
    double norm_rtol;         /* relative change that stops the ||D||_2 steps (1e-13)   */
    int b_max;                /* upper bound on the block width, <= 512 (512; MC 256);  */
                              /* the width is the predicted rank rounded up to b_round, */
                              /* at most min(m, n) / 2 and b_max                        */
    double ladder_tol;        /* BLWS_BF16 solves: W products in BF16 while the relative */
                              /* residual is at or above this, FP32 below (1e-3)         */
    int svt_start;            /* robust PCA in FP64 only: a start block other than      */
    int k_blocks;             /* BLWS_START_SPLIT, or k_blocks != 2, runs each SVT by   */
                              /* blws_svt_lanczos (the Sec. 4.1 ablations); defaults  */
                              /* BLWS_START_SPLIT and 2 (the default step)               */
    double ladder3_tol;       /* BLWS_BF16 robust PCA: > 0 adds a split-precision phase  */
                              /* after the BF16 one, W products in BF16 x 3 (W = W_hi +  */
                              /* W_lo, block likewise, three BF16 products) while the    */
                              /* residual is at or above this, FP32 below (0: off)       */
} blws_alm_opts;

typedef struct {
    int status;               /* BLWS_OK or BLWS_NOT_CONVERGED                          */
    int iters;                /* ALM iterations (= SVT calls)                           */
    int rank;                 /* rank of the returned A                                 */
    int b_final;              /* Lanczos block width of the last iteration              */
    int fallbacks;            /* columns replaced after an orthonormalisation breakdown */
    long long nnz_E;          /* nonzeros of the returned E (RPCA)                      */
    double rel_residual;      /* final ||D - A - E||_F / ||D||_F                        */
    double norm2_D;           /* ||D||_2 used for mu_0                                  */
    double seconds;           /* wall time of the solve, measured on the host           */
    int iters_bf16;           /* iterations whose W products ran in BF16 (BLWS_BF16)    */
    int refined;              /* 1 if a final FP32 step refined a BF16 last iterate     */
    int iters_bf16x3;         /* iterations whose W products ran in BF16 x 3            */
} blws_solve_info;

/* Create a context on HIP device `device` (its workspace grows on demand). */
int blws_create(blws_ctx* out, int device);
int blws_destroy(blws_ctx ctx);
const char* blws_status_string(int status);
/* Detail of the last failure on this context (never NULL). */
const char* blws_last_error(blws_ctx ctx);
void blws_default_alm_opts(blws_alm_opts* opts);
void blws_default_svt_opts(blws_svt_opts* opts);

/* A = T_eps(W) by one BLWS step (Eq. (4) with the partial SVD of Sec. 4).
 *   W: m x n (ldw). b: block width, 1 <= b <= min(m, n) / 2.
 *   warm = 1: U (m x b, ldu) and V (n x b, ldv) hold orthonormal columns (the
 *             previous principal subspaces) on entry.
 *   warm = 0: U, V are ignored on entry; a cold block is drawn (opts->seed).
 *   On exit U, V hold the top-b Ritz vectors (orthonormal), S (device double[b])
 *   the Ritz values in decreasing order, rank_dev (device int, may be NULL) the
 *   count of S_i > eps, and A (m x n, lda; may be NULL) = U_r diag(S_r - eps) V_r^T.
 *   eps >= 0. prec: BLWS_FP64 or BLWS_FP32. Asynchronous on `stream`. */
int blws_svt(blws_ctx ctx, void* stream, int prec, int m, int n, const void* W, int ldw,
             double eps, int b, void* U, int ldu, void* V, int ldv, int warm, double* S,
             int* rank_dev, void* A, int lda, const blws_svt_opts* opts);

/* blws_svt for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and errors as blws_svt (FP64 or FP32), with every
 * scratch buffer carved from a static device array of the library (64 MiB per
 * device, held from the first context on that device until the process ends)
 * and every launch on `stream` (no second stream, events or helper thread).
 * The call makes no hipMalloc / hipFree and no allocating library call; it
 * zeroes what must start at zero itself. A size whose scratch exceeds 64 MiB
 * returns BLWS_EINVAL (m = n = 2000 at b = 112 needs about 50 MiB in FP64).
 * All calls on one device share that array: calls whose work overlaps on the
 * device (other streams, other host threads, other contexts) race and must
 * be serialised by the caller. */
int blws_svt_noalloc(blws_ctx ctx, void* stream, int prec, int m, int n, const void* W, int ldw,
                     double eps, int b, void* U, int ldu, void* V, int ldv, int warm, double* S,
                     int* rank_dev, void* A, int lda, const blws_svt_opts* opts);

/* Start blocks of blws_svt_lanczos (Sec. 4.1). */
enum {
    BLWS_START_SPLIT = 0, /* blockdiag(U, V): 2b columns                          */
    BLWS_START_AUG = 1,   /* (U; V) / sqrt(2): b columns (BLWS as Sec. 4.1 writes it) */
    BLWS_START_LEFT = 2,  /* (U; 0): the standard half-information starts       */
    BLWS_START_RIGHT = 3  /* (0; V)                                              */
};

/* The start-block ablations of Sec. 4.1: one SVT step by Algorithms 2 and 3
 * taken literally on the augmented matrix [[0, W], [W^T, 0]] (Theorem 1),
 * never formed, from the start block `start` built from the orthonormal U
 * (m x b, ldu) and V (n x b, ldv), with k >= 1 blocks and block
 * reorthogonalisation (each new block orthonormalised against all earlier
 * ones; 2k - 1 products with W). The Rayleigh-Ritz matrix T_k (k c x k c,
 * c = 2b for BLWS_START_SPLIT, else b; k c <= 1024 and <= m + n) is
 * decomposed by the SVD of T_k + c I with c >= its spectral radius. FP64,
 * device pointers, queued on `stream`.
 *   On exit U = sqrt(2) Y_top, V = sqrt(2) Y_bottom for the top b Ritz
 *   vectors Y (orthonormal for the split and half starts; only nearly so for
 *   BLWS_START_AUG), S (device double[b]) the top b Ritz values in decreasing
 *   order (possibly negative for the aug start), rank_dev (device int, may
 *   be NULL) #{S_i > eps}, A (may be NULL, m x n, lda) U_r diag(S_r - eps) V_r^T.
 * Errors: BLWS_EINVAL for bad sizes or pointers, BLWS_EUNSUPPORTED for
 * k c above 1024. The default step (blws_svt) is BLWS_START_SPLIT with
 * k = 2 and its zero blocks skipped: the same Ritz values up to rounding. */
int blws_svt_lanczos(blws_ctx ctx, void* stream, int m, int n, const double* W, int ldw,
                     double eps, int b, int start, int k, double* U, int ldu, double* V,
                     int ldv, double* S, int* rank_dev, double* A, int lda);

/* Robust PCA: min ||A||_* + lambda ||E||_1 s.t. D = A + E, by inexact ALM with
 * one BLWS step per iteration (Sec. 5). lambda <= 0 selects 1/sqrt(max(m, n)).
 * D (m x n, ldd) is read only; A (lda) and E (lde) receive the solution; E is
 * also used as iteration state. opts may be NULL (defaults); info is a HOST
 * struct (may be NULL). Blocks until the result is complete.
 * Returns BLWS_OK, BLWS_NOT_CONVERGED, or an error. */
int blws_rpca_solve(blws_ctx ctx, void* stream, int prec, int m, int n, const void* D,
                    int ldd, double lambda, const blws_alm_opts* opts, void* A, int lda,
                    void* E, int lde, blws_solve_info* info);

/* Defaults of the matrix-completion solver: those of blws_default_alm_opts
 * with tol = 1e-6, rho = 1.05 and mu0_scale = 1.0 (mu_0 = 1/||P_Omega(M)||_2);
 * rho = 1.05 is the largest value with which n = 5000, rank 50, 10% sampled
 * ends at the planted rank (larger ones keep spurious components just above
 * the last threshold). */
void blws_default_mc_opts(blws_alm_opts* opts);

/* Matrix completion: min ||A||_* s.t. P_Omega(A) = P_Omega(M), by inexact ALM
 * (Sec. 2, Eq. (2) and its ALM host, Sec. 5) with one BLWS step per iteration.
 * The matrix W = A + P_Omega(D + Y/mu - A) whose SVT each iteration takes is
 * low rank plus sparse and is applied to blocks without being formed.
 *   Omega and the samples: CSR on the device, row_ptr (int32[m + 1]),
 *   col_idx (int32[nnz]), values (nnz, type of prec; both may be NULL when
 *   nnz = 0, which returns rank 0). Columns within a row may
 *   come in any order; row_ptr must be nondecreasing from 0 to nnz and every
 *   column index in [0, n), else BLWS_EINVAL (checked on the device before
 *   any other use). Read only.
 *   Output: A = U diag(S) V^T with rank r = info->rank; the first
 *   min(r, r_cap) columns of U (m x r_cap, ldu >= r_cap), V (n x r_cap,
 *   ldv >= r_cap) and entries of S (device double[r_cap]) are written.
 *   Stop at ||P_Omega(M) - P_Omega(A)||_F / ||P_Omega(M)||_F < tol.
 *   opts may be NULL (blws_default_mc_opts); info is a HOST struct (may be
 *   NULL). prec: BLWS_FP64 or BLWS_FP32. Blocks until the result is complete.
 * Returns BLWS_OK, BLWS_NOT_CONVERGED, or an error. */
int blws_mc_solve(blws_ctx ctx, void* stream, int prec, int m, int n, int nnz,
                  const int* row_ptr, const int* col_idx, const void* values,
                  const blws_alm_opts* opts, int r_cap, void* U, int ldu, double* S, void* V,
                  int ldv, blws_solve_info* info);

/* Options of the SVT matrix-completion solver (defaults from
 * blws_default_svt_mc_opts). */
typedef struct {
    double tau;               /* threshold; <= 0 selects 5 sqrt(m n)                    */
    double delta;             /* step size; <= 0 selects 1.2 m n / nnz                  */
    double tol;               /* stop at ||P_Omega(M - X)||_F / ||P_Omega(M)||_F <= tol */
                              /* (1e-4)                                                 */
    int max_iter;             /* 500                                                    */
    int rank_step;            /* values added to a request that fell short (5)          */
    int b_round;              /* block width = requested count rounded up to this (16)  */
    int b_max;                /* upper bound on the block width, <= 512 (512)           */
    int pow_steps;            /* power half-step pairs of the first (cold) block (2)    */
    unsigned long long seed;  /* counter-based generator seed                           */
    int norm_steps;           /* max BLWS steps for the ||P_Omega(M)||_2 estimate (8)   */
    double norm_rtol;         /* relative change that stops those steps (1e-13)         */
} blws_svt_mc_opts;

void blws_default_svt_mc_opts(blws_svt_mc_opts* opts);

/* Matrix completion by the singular value thresholding algorithm, the MC
 * host of the experiments of Sec. 5 (its Table 2), with each thresholding
 * X_k = T_tau(Y_{k-1}) computed by BLWS on the purely sparse W = Y_{k-1}:
 *   Y_0 = k0 delta P_Omega(M), k0 = ceil(tau / (delta ||P_Omega(M)||_2));
 *   Y_k = Y_{k-1} + delta P_Omega(M - X_k) until
 *   ||P_Omega(M - X_k)||_F / ||P_Omega(M)||_F <= tol.
 * Each thresholding asks for r_{k-1} + 1 values and, while all of them
 * exceed tau, for rank_step more (BLWS steps warm-started from the block
 * just computed). Arguments, pattern checks and outputs as blws_mc_solve
 * (the factors of the last X_k); opts may be NULL. Blocks until done.
 * Returns BLWS_OK, BLWS_NOT_CONVERGED, or an error. */
int blws_mc_svt_solve(blws_ctx ctx, void* stream, int prec, int m, int n, int nnz,
                      const int* row_ptr, const int* col_idx, const void* values,
                      const blws_svt_mc_opts* opts, int r_cap, void* U, int ldu, double* S,
                      void* V, int ldv, blws_solve_info* info);

/* ---------------------------------------------------------------------- */
/* Diagnostics (used by the parity tests and the bench).                   */
/* ---------------------------------------------------------------------- */

/* X (rows x cols, ldx, device double) = the counter-based uniform generator:
 * X[i][j] = u(seed, stream_id * 2^40 + i * 4096 + j), u = the (counter+1)-th
 * SplitMix64 output mapped to [-1, 1) as ((z >> 11) * 2^-53) * 2 - 1. */
int blws_fill_uniform(blws_ctx ctx, void* stream, int rows, int cols, double* X, int ldx,
                      unsigned long long seed, unsigned long long stream_id);

/* C (M x N, ldc) = alpha * op(A) * B + beta * C, op(A) = A (trans_a = 0, A is
 * M x K) or A^T (trans_a = 1, A is K x M); B is K x N. All double. This is the
 * library's skinny-GEMM kernel family (MFMA, split-K, deterministic). */
int blws_gemm_f64(blws_ctx ctx, void* stream, int trans_a, int M, int N, int K, double alpha,
                  const double* A, int lda, const double* B, int ldb, double beta, double* C,
                  int ldc);

/* Diagnostic: C (M x N, float) = op(A) B on the FP32 (bf16 = 0: A float) or
 * BF16 (bf16 = 1: A holds BF16 bits as uint16, B is rounded to BF16 on the
 * way in) matrix cores with FP32 accumulation: the kernel of the W products
 * in the FP32 and BF16 modes. op(A) = A (M x K, lda) or A^T (A is K x M).
 * B is K x N (ldb). Asynchronous on `stream`. */
int blws_gemm_lp(blws_ctx ctx, void* stream, int bf16, int trans_a, int M, int N, int K,
                 const void* A, int lda, const float* B, int ldb, float* C, int ldc);

/* Diagnostic: C (M x N, float) = op(A) B in split-precision BF16 x 3, the
 * kernel of the BLWS_BF16X3 W products: A_hi, A_lo (BF16 bits as uint16, the
 * same layout and lda; A = A_hi + A_lo), B float split on the way in into
 * b_hi = bf16(b), b_lo = bf16(b - b_hi); C = A_hi B_hi + A_hi B_lo + A_lo B_hi
 * with FP32 accumulation. op(A) = A (M x K) or A^T (A is K x M). Asynchronous
 * on `stream`. */
int blws_gemm_bf16x3(blws_ctx ctx, void* stream, int trans_a, int M, int N, int K,
                     const void* A_hi, const void* A_lo, int lda, const float* B, int ldb,
                     float* C, int ldc);

/* SVD of a small dense N x N FP64 matrix B (ldb) on the device: U_B (N x N),
 * V_B (N x N) row-major with ld = N, S (N) decreasing, sign chosen so that the
 * largest-magnitude entry of each left vector is positive. */
int blws_small_svd_f64(blws_ctx ctx, void* stream, int N, const double* B, int ldb,
                       double* UB, double* S, double* VB);

/* The cold start block of blws_svt (warm = 0) on its own: V = orth(random
 * n x b drawn from generator stream `stream_v`) refined by `pow_steps` power
 * half-step pairs V <- orth(W^T orth(W V)); U = orth(random m x b, stream
 * stream_v + 1), independent of V. U (m x b, ldu), V (n x b, ldv) receive
 * orthonormal columns. FP64 or FP32 per prec. */
int blws_cold_block(blws_ctx ctx, void* stream, int prec, int m, int n, const void* W, int ldw,
                    int b, int pow_steps, unsigned long long seed, unsigned long long stream_v,
                    void* U, int ldu, void* V, int ldv);

/* Per-kernel timing with HIP events on the launching stream. enable = 1 starts
 * recording (and clears the totals); 0 stops. */
int blws_timing_enable(blws_ctx ctx, int enable);
/* Totals for the kernel family `name` ("gemm_w", "gemm_ts", "alm_epilogue",
 * "small_svd", "chol", ...): launches and summed milliseconds, and the summed
 * algorithmic flop and byte counts of those launches. Synchronises the device. */
int blws_timing_get(blws_ctx ctx, const char* name, long long* launches, double* ms,
                    double* flops, double* bytes);
/* Autotuning: force the split-K plans of the generic W-product GEMM kernels
 * to aim at `target` workgroups (0 restores the tuned table the library was
 * built with). Process-wide, for paper_1012_0365_amd/autotune.py; a plan
 * change changes the order in which partial sums are added, so results then
 * differ from the tuned ones in the last bits. Returns BLWS_EINVAL for
 * target < 0 or > 65536. */
int blws_set_plan_target(int target);
/* Comma-separated names of the kernel families recorded since timing was
 * enabled, into buf (host, len bytes, NUL-terminated). */
int blws_timing_list(blws_ctx ctx, char* buf, size_t len);
/* Restrict timing to the comma-separated kernel families in `families` (host
 * string; NULL or "" records every family). Recording a family costs two
 * event records per launch; restricting it keeps that cost off the other
 * launches. Takes effect for launches after the call; synchronises the
 * device. */
int blws_timing_only(blws_ctx ctx, const char* families);

/* ------------------------------------------------------------------------
 * Request server (serving many solves on one GPU).
 *
 * RPCA and matrix-completion requests of any sizes are submitted at any time
 * and run with continuous batching: a scheduler thread keeps up to max_slots
 * solves in flight, each on its own stream with its own workspace (D, E, Y or
 * the samples and multipliers, and the warm Lanczos block stay resident in
 * HBM until the solve ends), and advances whichever solve's last step has
 * finished, so the work of different requests overlaps on the device.
 * Requests are admitted in submission order as soon as a slot is free and
 * their workspace fits the memory budget next to the solves in flight (a
 * request larger than the budget runs alone). Each request computes exactly
 * what blws_rpca_solve / blws_mc_solve compute for the same arguments,
 * whatever else is in flight.
 *
 * Buffers: the input buffers must hold their data when submit is called (the
 * server's streams do not wait on the caller's streams) and, like the output
 * buffers, stay valid and untouched until the request is reported done. Every
 * request is retrieved once, by blws_server_poll or blws_server_wait.
 * info->seconds is the latency from submit to completion.
 *
 * Grouped launches (group_products = 1): the solves whose last step has
 * finished are advanced together, their host logic on one thread per slot;
 * the dense W-products of their BLWS steps (W V, W^T U, then W G) are handed
 * to one collector, which queues all of them as one grouped launch per
 * precision (each problem with the block grid and K split it has alone, so a
 * result is the same bits grouped or not) once every solve of the round has
 * either handed over its products or finished its step. A solve that becomes
 * ready waits up to group_window_us for the others in flight to be ready too.
 * ------------------------------------------------------------------------ */
typedef struct blws_server_s* blws_server;

typedef struct {
    int max_slots;       /* solves in flight at once, 1..16 (4)                        */
    size_t mem_budget;   /* device bytes the in-flight solves' workspaces may hold;    */
                         /* 0 selects 80% of the free device memory at creation (0)     */
    int group_products;  /* 1: grouped W-product launches across solves (1)            */
    int group_window_us; /* wait for other solves to become ready, 0..10000 us (200)   */
} blws_server_opts;

typedef struct {
    long long submitted, completed, failed;
    int active;        /* solves in flight now                                         */
    int queued;        /* requests waiting for admission                               */
    int max_active;    /* most solves in flight at once so far                         */
    size_t mem_in_use, mem_peak, mem_budget;
    long long grouped_launches; /* grouped W-product launches queued                   */
    long long grouped_products; /* W-products that went through them                   */
    int max_group;              /* most W-products in one grouped launch               */
} blws_server_stats;

void blws_default_server_opts(blws_server_opts* opts);
/* Start a server on HIP device `device` (opts may be NULL). */
int blws_server_create(blws_server* out, int device, const blws_server_opts* opts);
/* Finish every submitted request, then release the server. */
int blws_server_destroy(blws_server srv);
/* Queue a robust-PCA solve (arguments as blws_rpca_solve; prec FP64, FP32 or
 * BF16). Arguments are checked here: on an error nothing is queued. On
 * success *ticket (host) identifies the request. */
int blws_server_submit_rpca(blws_server srv, int prec, int m, int n, const void* D, int ldd,
                            double lambda, const blws_alm_opts* opts, void* A, int lda, void* E,
                            int lde, long long* ticket);
/* Queue a matrix-completion solve (arguments as blws_mc_solve). */
int blws_server_submit_mc(blws_server srv, int prec, int m, int n, int nnz, const int* row_ptr,
                          const int* col_idx, const void* values, const blws_alm_opts* opts,
                          int r_cap, void* U, int ldu, double* S, void* V, int ldv,
                          long long* ticket);
/* *done = 1 and the request's status returned (info filled, may be NULL) once
 * it has finished; *done = 0 and BLWS_OK while it is queued or running.
 * BLWS_EINVAL for an unknown or already retrieved ticket. */
int blws_server_poll(blws_server srv, long long ticket, int* done, blws_solve_info* info);
/* Block until the request has finished; returns its status. */
int blws_server_wait(blws_server srv, long long ticket, blws_solve_info* info);
int blws_server_get_stats(blws_server srv, blws_server_stats* stats);
/* Detail of the last failure seen through this server (never NULL). */
const char* blws_server_last_error(blws_server srv);

#ifdef __cplusplus
}
#endif
#endif
