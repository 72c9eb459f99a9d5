/* Test-only CPU oracle for block Lanczos with warm start (BLWS) singular value
 * thresholding inside inexact-ALM nuclear-norm solvers.
 *
 * TEST INFRASTRUCTURE: only tests, the smoke check and the bench's CPU baseline
 * call this library. It shares no code with the GPU library.
 *
 * All matrices are dense, row-major, FP64, element (i, j) at p[i * cols + j]
 * (no leading-dimension argument: rows are packed). Every entry point returns 0
 * on success and a negative value on a bad argument or allocation failure.
 */
#ifndef BLWS_ORACLE_H
#define BLWS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The (counter + 1)-th 64-bit output of SplitMix64 seeded with `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t counter);

/* The (counter + 1)-th output of SplitMix64 seeded with `seed`, mapped to
 * [-1, 1) as ((z >> 11) * 2^-53) * 2 - 1. Exact in binary64. */
double orc_uniform(uint64_t seed, uint64_t counter);

/* Fill X (rows x cols) with orc_uniform(seed, stream * 2^40 + i * 4096 + j). */
void orc_fill_uniform(int rows, int cols, uint64_t seed, uint64_t stream, double* X);

/* Thin SVD W = U diag(S) V^T by one-sided (Hestenes) Jacobi. p = min(m, n).
 * U: m x p, S: p (descending), V: n x p. Returns the number of sweeps. */
int orc_jacobi_svd(int m, int n, const double* W, double* U, double* S, double* V);

/* Eq. (4): A = T_eps(W) computed from the full Jacobi SVD. S_all (p values,
 * may be NULL) receives all singular values; *rank = #{sigma_i > eps}. */
int orc_svt_exact(int m, int n, const double* W, double eps, double* A, double* S_all,
                  int* rank);

/* Start blocks of the literal block Lanczos on [[0, W], [W^T, 0]] (Sec. 4.1). */
#define ORC_START_SPLIT 0 /* blockdiag(U, V): 2b columns                        */
#define ORC_START_AUG 1   /* (U; V) / sqrt(2): b columns                        */
#define ORC_START_LEFT 2  /* (U; 0)                                              */
#define ORC_START_RIGHT 3 /* (0; V)                                              */

/* Algorithms 2 and 3 literally on the explicitly formed augmented matrix, from
 * the start block `start` built from U (m x b) and V (n x b), with k blocks
 * (k * columns of the start block <= m + n) and block reorthogonalisation.
 * On exit U = sqrt(2) Y_top, V = sqrt(2) Y_bottom for the top b Ritz vectors Y,
 * S (b) the top b Ritz values (decreasing), *rank = #{S_i > eps}, A (m x n,
 * may be NULL) = U_r diag(S_r - eps) V_r^T. Returns 1 if the Jacobi EVD of T_k
 * did not settle in 100 sweeps, < 0 on bad arguments. */
int orc_lanczos_svt(int m, int n, const double* W, double eps, int b, int start, int k,
                    double* U, double* V, double* S, double* A, int* rank);

/* One BLWS step (block Lanczos, k = 2, warm start from U, V; split Rayleigh-Ritz).
 * U (m x b) and V (n x b) hold orthonormal columns on entry and the top-b Ritz
 * vectors on exit. S (b) receives the Ritz values (descending); *rank =
 * #{S_i > eps}; A (m x n, may be NULL) receives U_r diag(S_r - eps) V_r^T. */
int orc_blws_step(int m, int n, const double* W, double eps, int b, double* U, double* V,
                  double* S, double* A, int* rank);

/* Cold start block: V = orth(random n x b) refined by `pow_steps` power
 * half-step pairs V <- orth(W^T orth(W V)); U = orth(random m x b), drawn
 * independently. Streams: V uses stream_v, U uses stream_v + 1. */
int orc_cold_block(int m, int n, const double* W, int b, int pow_steps, uint64_t seed,
                   uint64_t stream_v, double* U, double* V);

/* Spectral norm by repeated BLWS steps from a cold block of width bs. */
double orc_spectral_norm_blws(int m, int n, const double* W, int bs, int pow_steps,
                              uint64_t seed, double rtol, int max_steps, int* steps_out);

typedef struct {
    double tol;            /* stop when ||D - A - E||_F / ||D||_F < tol            */
    int max_iter;
    double rho;            /* mu <- min(rho * mu, mu_bar)                          */
    double mu0_scale;      /* mu0 = mu0_scale / ||D||_2                            */
    double mu_max_factor;  /* mu_bar = mu_max_factor * mu0                         */
    int sv0;               /* initial predicted rank                                */
    double sv_step_frac;   /* rank-prediction increment, as a fraction of min(m,n) */
    int b_round;           /* Lanczos block width = sv rounded up to this          */
    int pow_steps;         /* power half-step pairs in the cold start               */
    uint64_t seed;
    int norm_steps;        /* safety bound on the BLWS steps of the ||D||_2 estimate */
    double norm_rtol;      /* those steps stop once the top value changes less      */
    int svt_start;         /* BLWS-mode SVT: ORC_START_SPLIT with k_blocks = 2 is    */
    int k_blocks;          /* the default step; anything else runs orc_lanczos_svt  */
} orc_alm_opts;

typedef struct {
    int iters;
    int rank;
    int b_final;
    long long nnz_E;
    double rel_residual;
    double norm2_D;
    int status;            /* 0 converged, 1 max_iter reached */
} orc_info;

void orc_default_opts(orc_alm_opts* o);

/* Rank prediction: svp + 1 if svp < sv, else min(svp + round(step_frac p), p). */
int orc_predict_rank(int svp, int sv, double step_frac, int p);

/* Block width for a predicted rank: sv rounded up to b_round, at most p / 2. */
int orc_block_width(int sv, int b_round, int p);

/* The warm block X (rows x b_old) resized to Y (rows x b_new): truncation keeps
 * the leading columns; growth keeps X and appends the columns of
 * orc_fill_uniform(rows, b_new - b_old, seed, stream) orthonormalised against X
 * (Householder QR of [X, R], second block). */
int orc_resize_block(int rows, int b_old, int b_new, const double* X, uint64_t seed,
                     uint64_t stream, double* Y);

/* mode: 0 = exact SVT (full Jacobi SVD each iteration, the plain form),
 *       1 = BLWS SVT.
 * Y (m x n, may be NULL) receives the final multiplier. sv_trace (may be NULL,
 * length max_iter) receives the per-iteration svp. */
int orc_rpca(int m, int n, const double* D, double lambda, const orc_alm_opts* opts,
             int mode, double* A, double* E, double* Y, int* svp_trace, orc_info* info);

/* The BLWS-mode RPCA loop of orc_rpca stopped at the start of iteration `it`
 * (1-based): W (m x n) receives that iteration's W = D - E + Y/mu, U (m x b)
 * and V (n x b) its warm block, *b its width (<= b_cap) and *eps = 1/mu.
 * Returns -3 if the loop converges first or the width exceeds b_cap. */
int orc_rpca_snapshot(int m, int n, const double* D, double lambda, const orc_alm_opts* opts,
                      int it, double* W, double* U, double* V, int b_cap, int* b, double* eps);

/* Matrix completion by inexact ALM: min ||A||_* s.t. P_Omega(A) = P_Omega(M).
 * Omega as CSR (row_ptr m+1, col_idx nnz). mode as for orc_rpca; the exact mode
 * forms W densely. Output: factors U (m x r_cap, row stride r_cap), V (n x r_cap),
 * S (r_cap) of the final A = U diag(S) V^T (the first min(*rank, r_cap) columns). */
int orc_mc(int m, int n, int nnz, const int* row_ptr, const int* col_idx,
           const double* values, const orc_alm_opts* opts, int mode, int r_cap,
           double* U, double* S, double* V, int* rank, orc_info* info);

/* Options of the SVT algorithm for matrix completion. */
typedef struct {
    double tau;        /* threshold; <= 0 selects 5 sqrt(m n)                    */
    double delta;      /* step; <= 0 selects 1.2 m n / nnz                       */
    double tol;        /* stop at ||P_Omega(X - M)||_F / ||P_Omega(M)||_F <= tol */
    int max_iter;
    int rank_step;     /* values added to a partial-SVD request that fell short  */
    int b_round;       /* BLWS block width = requested count rounded up to this  */
    int pow_steps;
    uint64_t seed;
    int norm_steps;    /* safety bound on the BLWS steps of ||P_Omega(M)||_2     */
    double norm_rtol;
} orc_svt_mc_opts;

void orc_default_svt_mc_opts(orc_svt_mc_opts* o);

/* The SVT algorithm for matrix completion with exact (mode 0, dense Jacobi)
 * or BLWS (mode 1) singular value thresholding; outputs as orc_mc. */
int orc_mc_svt(int m, int n, int nnz, const int* row_ptr, const int* col_idx,
               const double* values, const orc_svt_mc_opts* opts, int mode, int r_cap,
               double* U, double* S, double* V, int* rank, orc_info* info);

#ifdef __cplusplus
}
#endif
#endif
