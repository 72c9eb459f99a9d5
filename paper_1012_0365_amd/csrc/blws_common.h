// Internal declarations shared by the HIP translation units of libblws.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/blws.h"

namespace blws {

// Counter-based uniform draw: the (counter + 1)-th output of SplitMix64
// (Steele, Lea & Flood 2014) seeded with `seed`, mapped to [-1, 1).
__device__ __forceinline__ double uniform_pm1(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

// ---------------------------------------------------------------------------
// Error plumbing: every HIP call in host code goes through HIP_TRY, which turns
// a failure into a BlwsError carrying BLWS_EDEVICE and the HIP message.
// ---------------------------------------------------------------------------
struct BlwsError {
    int status;
    std::string msg;
};

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::blws::BlwsError{BLWS_EDEVICE, std::string(#expr) + ": " +           \
                                                      hipGetErrorString(e_)};           \
    } while (0)

#define BLWS_REQUIRE(cond, status, text)                                               \
    do {                                                                               \
        if (!(cond)) throw ::blws::BlwsError{(status), (text)};                       \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel timing (HIP events on the launching stream) for the bench.
// ---------------------------------------------------------------------------
struct Timer;
// Start/stop one timed launch of a kernel family; no-ops unless timing is on.
struct TimedLaunch {
    Timer* t;
    int slot;
    hipStream_t stream;
    const char* fam;
    TimedLaunch(Timer* timer, const char* family, hipStream_t s, double flops, double bytes);
    ~TimedLaunch();
};

// ---------------------------------------------------------------------------
// Kernel launchers (device code in k_*.hip). All take the stream last.
// ---------------------------------------------------------------------------

// Skinny GEMM: C (M x N, ldc) = alpha * op(A) * B + beta * Cin, with
// op(A) = A (M x K, lda) or A^T (A is K x M). B is K x N (ldb). Cin may alias C.
// Types: TA for A, TB for B, TC for C/Cin; compute type TM (double or float).
// `partial` is a device scratch of at least gemm_partial_elems(...) doubles.
template <typename TA, typename TB, typename TC>
void gemm(Timer* tm, const char* family, bool trans_a, int M, int N, int K, double alpha,
          const TA* A, int lda, const TB* B, int ldb, double beta, const TC* Cin, int ldcin,
          TC* C, int ldc, double* partial, size_t partial_elems, hipStream_t s);
size_t gemm_partial_elems(int M, int N, int K);

// Workgroup target of the split-K plan of a generic GEMM (prec 0 FP64,
// 1 FP32, 2 BF16) from the autotuned table (tuning.hip); `fallback` outside
// the shapes it covers. set_plan_override(t > 0) forces t for tuning runs.
int plan_target(int prec, int M, int N, int K, int fallback);
void set_plan_override(int target);

// One W-product C = op(A) B (op(A) = A^T if trans) for a grouped launch:
// prec 0 = FP64 (A, B, C double, partial doubles), 1 = FP32 (float), 2 = BF16
// (A holds BF16 bits, B and C float, partial floats). partial is the
// problem's own split-K scratch. A grouped launch computes every problem with
// the block grid and K split it gets alone, so the results are the same bits.
constexpr int GEMM_GROUP_MAX = 16;
struct WProduct {
    int prec;
    bool trans;
    int M, N, K;
    const void* A;
    int lda;
    const void* B;
    int ldb;
    void* C;
    int ldc;
    void* partial;
    size_t partial_elems;
};
// FP64: true if the problem takes the generic split-K kernel (the only one
// with a grouped form); FP32 / BF16: always (with enough partial scratch).
bool wproduct_groupable(const WProduct& w);
bool wproduct_lp_groupable(const WProduct& w);
// n <= GEMM_GROUP_MAX groupable problems of one precision, on stream s.
// C = X R (X M x N, R N x N FP64, N <= 512) with the columns j where
// flags[j] != 0 replaced by the counter-based draws uniform_pm1(seed,
// (sid << 40) + 4096 i + j): the apply step of a Cholesky-QR pass whose
// dependent columns are redrawn.
template <typename T>
void gemm_apply_flagged(Timer* tm, int M, int N, const T* X, int ldx, const double* R, int ldr,
                        T* C, int ldc, const int* flags, uint64_t seed, uint64_t sid,
                        hipStream_t s);
void gemm_f64_grouped(const WProduct* ps, int n, hipStream_t s);
void gemm_lp_grouped(const WProduct* ps, int n, hipStream_t s);

// W-products in FP32 on FP32 MFMA (bf16 = false: A float) or BF16 MFMA
// (bf16 = true: A holds BF16 bits, B is rounded to BF16), FP32 accumulation:
// C (M x N, float) = op(A) B. `partial` holds gemm_lp_partial_elems floats.
size_t gemm_lp_partial_elems(int M, int N, int K);
// A_lo non-null (BF16 mode only): split-precision BF16 x 3, A holding the high
// and A_lo the low BF16 halves of the FP32 matrix (A_hi + A_lo), B split the
// same way on the fly: C = A_hi B_hi + A_hi B_lo + A_lo B_hi.
void gemm_lp(Timer* tm, const char* family, bool bf16, bool trans_a, int M, int N, int K,
             const void* A, int lda, const float* B, int ldb, float* C, int ldc, float* partial,
             size_t partial_elems, hipStream_t s, const unsigned short* A_lo = nullptr);
// Y[e] = BF16(X[e]) for e < count (round to nearest even).
void to_bf16(long long count, const float* X, unsigned short* Y, hipStream_t s);
// Hi = BF16(X), Lo = BF16(X - Hi) over rows x cols (all with leading dimension ld).
void split_bf16x2(int rows, int cols, const float* X, int ld, unsigned short* Hi,
                  unsigned short* Lo, hipStream_t s);

// Scaled LDL^T / Cholesky with breakdown detection on an n x n Gram matrix:
// writes Rinv (n x n, ld n) such that X * Rinv has orthonormal columns when
// G = X^T X; columns whose scaled pivot is <= eta are flagged (flags[j] = 1)
// and get a zero column in Rinv. nflag (device int) += number of flags.
// When n <= 128 and n max|G_ij - I_ij| (a bound on ||G - I||_2) is within
// ni_tol, Rinv = (3 I - G) / 2 instead (X Rinv orthonormal to 3 ni_tol^2 / 4)
// and no column is flagged.
void chol_inv(Timer* tm, int n, const double* G, int ldg, double* Rinv, int* flags,
              int* nflag, double eta, double ni_tol, double* scratch, hipStream_t s);
size_t chol_scratch_elems(int n);

// The columns j of Q (rows x c, ldq, c <= 128) with flags0[j] or flags1[j]
// set (the dependent columns of a chunk's two Cholesky-QR passes, zero in Q)
// re-formed from src (the chunk as the first pass saw it, lds) by classical
// Gram-Schmidt with reorthogonalisation against Xa (rows x ba), Xb (rows x bb)
// and the finished columns of Q, normalised; a column in that span to
// rounding is replaced by the draws uniform_pm1(seed, (sid << 40) + 4096 i +
// j) orthogonalised the same way. xv: rows doubles of scratch. nflag += the
// columns flagged by the second pass only. No work when nothing is flagged.
template <typename T>
void orth_fallback(Timer* tm, int rows, int c, const int* flags0, const int* flags1, const T* src,
                   int lds, T* Q, int ldq, const T* Xa, int lda, int ba, const T* Xb, int ldb,
                   int bb, double* xv, int* nflag, uint64_t seed, uint64_t sid, hipStream_t s);

// Two Cholesky-QR passes on X0 and X1 (rows x c each, leading dimension ld,
// rows <= 512, c <= 128) in place, one workgroup per matrix: dependent
// columns of the first pass redrawn (stream ids sid0, sid1), counted in nflag.
// G0, G1 (c x c each) receive the Gram matrices formed first; when a side's
// is within 1e-8 of I in the bound c max|G_ij - I_ij| on ||G - I||_2,
// X (3I - G)/2 replaces the passes, over many workgroups.
bool cholqr2_small_supported(int rows, int c);
void cholqr2_small(Timer* tm, int rows, int c, double* X0, double* X1, int ld, int* nflag,
                   double eta, uint64_t seed, uint64_t sid0, uint64_t sid1, double* G0, double* G1,
                   hipStream_t s);

// X[i][j] = u(seed, stream_id * 2^40 + i * 4096 + j) for i < rows, j < cols.
template <typename T>
void fill_uniform(int rows, int cols, T* X, int ldx, uint64_t seed, uint64_t stream_id,
                  hipStream_t s);

// SVD of a 1 x 1 matrix B: UB = 1, S = |B|, VB = sign(B).
void small_svd_1x1(const double* B, double* UB, double* S, double* VB, hipStream_t s);

// Golub-Kahan bidiagonalisation + bisection / inverse iteration on the
// Golub-Kahan tridiagonal (N <= 512): the top nv singular values S[0..nv) and
// the first nv columns of UB, VB (N x N, ld N). The vectors of close values are
// not yet orthogonalised (the caller polishes them). Above N = 224 the
// bidiagonalisation is a cooperative launch; *err (device int, zeroed by the
// caller) is set if one of its barrier waits timed out.
bool small_svd_gk_supported(int N);
size_t small_svd_gk_scratch_elems(int N);
// With a second stream s2 and two events, the blocked reflectors' T factors
// are built on s2 (after the bidiagonalisation on s) while s finds the values
// and vectors; s waits for them before the back-transformation.
void small_svd_gk(Timer* tm, int N, int nv, const double* B, int ldb, double* UB, double* S,
                  double* VB, double* scratch, int* err, hipStream_t s, hipStream_t s2 = nullptr,
                  hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr);

// Copy a rows x cols block (types may differ).
template <typename TS, typename TD>
void copy2d(int rows, int cols, const TS* src, int lds, TD* dst, int ldd, hipStream_t s);

// Zero `bytes` bytes at p (both multiples of 4) with a kernel: used in place
// of hipMemsetAsync, whose nodes in a captured graph have given wrong results
// on replays.
void zero_bytes(void* p, size_t bytes, hipStream_t s);

// rank_out[0] = #{S_i > eps, i < b}.
void count_above(int b, const double* S, double eps, int* rank_out, hipStream_t s);

// Literal block Lanczos on [[0, W], [W^T, 0]] (k_lanczos.hip): M = S + S^T and
// Bt = B^T (c x c); T (K x K, K = k c) = T_k + shift I with T_k block
// tridiagonal from Ms (k blocks M_l) and Bs (k - 1 blocks B_l, below the
// diagonal), shift (device scalar, written) the largest absolute row sum of
// T_k; lam[i] = sig[i] - shift (i < b).
void lanczos_sym(int c, const double* S, double* M, hipStream_t s);
void lanczos_transpose(int c, const double* B, double* Bt, hipStream_t s);
void lanczos_assemble(int k, int c, const double* Ms, const double* Bs, double* shift, double* T,
                      hipStream_t s);
void lanczos_eigvals(int b, const double* sig, const double* shift, double* lam, hipStream_t s);

// Sum of squares and max |.| of an m x n matrix: two-pass, deterministic.
// out[0] = sum of squares, out[1] = max abs. scratch >= norms_scratch_elems().
template <typename T>
void norms(int m, int n, const T* X, int ldx, double* out, double* scratch, hipStream_t s);
size_t norms_scratch_elems();

// RPCA start: Y = D / J, E = 0, W = D - E + Y / mu (Y, W with ld = n).
template <typename T>
void rpca_init(int m, int n, const T* D, int ldd, double J, double mu, T* Y, T* E, int lde,
               T* W, hipStream_t s);

// Fused SVT reconstruction + inexact-ALM update for RPCA (one pass over D, Y):
// a = sum_{k < r} U[i][k] (S[k] - eps) V[j][k] with r = #{S_k > eps} (k < b);
// t = d - a + y / mu;  e = shrink(t, lam / mu);  z = d - a - e;
// y' = y + mu z;  w' = d - e + y' / mu_next.
// Writes E, Y, W (and its BF16 copy Wh when non-null, with the low half
// Wl = BF16(W - Wh) of the split-precision copy when Wl is non-null too), and
// per-workgroup partial sums of z^2 into `partials`
// (size alm_partials(m, n)); A_out (may be null) receives a.
template <typename T>
void alm_epilogue(Timer* tm, int m, int n, int b, const T* U, int ldu, const T* V, int ldv,
                  const double* S, double eps, double lam, double mu, double mu_next,
                  const T* D, int ldd, T* Y, T* E, int lde, T* W, unsigned short* Wh, T* A_out,
                  int lda, double* partials, hipStream_t s, unsigned short* Wl = nullptr);
size_t alm_partials(int m, int n);
// A = U_r diag(S_r - eps) V_r^T only.
template <typename T>
void svt_reconstruct(Timer* tm, int m, int n, int b, const T* U, int ldu, const T* V, int ldv,
                     const double* S, double eps, T* A, int lda, hipStream_t s);

// out[0] = sum of partials[0..count) in a fixed order.
void sum_partials(int count, const double* partials, double* out, hipStream_t s);
void iter_readback(int count, const double* partials, const int* rank, const int* err, double* zz,
                   int* rank_out, int* err_out, hipStream_t s);

// Count nonzeros of an m x n matrix into out (long long), deterministic.
template <typename T>
void count_nonzeros(int m, int n, const T* X, int ldx, long long* out, long long* scratch,
                    hipStream_t s);

// ---------------------------------------------------------------------------
// Matrix-completion operator (k_sparse.hip).
// ---------------------------------------------------------------------------

// flag[0] = 0, then |= 1 if row_ptr is not nondecreasing from 0 to nnz, |= 2 if
// a column index lies outside [0, n).
void csr_check(int m, int n, int nnz, const int* row_ptr, const int* col_idx, int* flag,
               hipStream_t s);
// Transposed pattern: col_ptr (n + 1), csc_row / csc_perm (nnz): for position
// q of column j, the row and the CSR index of the entry, rows ascending.
// maxcnt[0] = longest column. scratch >= csc_scratch_ints(n, nnz) ints.
size_t csc_scratch_ints(int n, int nnz);
void csc_build(int m, int n, int nnz, const int* row_ptr, const int* col_idx, int* col_ptr,
               int* csc_row, int* csc_perm, int* maxcnt, int* scratch, hipStream_t s);
// out (rows x c, ldo) = sparse (rows, pattern ptr/idx, values val or val[perm]) * X.
template <typename T>
void spmm(Timer* tm, const char* family, int rows, int c, const int* ptr, const int* idx,
          const int* perm, const T* val, const T* X, int ldx, T* out, int ldo, long long nnz,
          hipStream_t s);
// Row k of C (r x c) times S[k] - eps.
void lr_scale(int r, int c, const double* S, double eps, double* C, int ldc, hipStream_t s);
// Fused update over Omega: A_Omega from the factors (the first min(rank_dev,
// rmax) columns, coefficients S - eps), y += mu (d - A_Omega), the next sparse
// part sv = d + y / mu_next - A_Omega (skipped when sv is null), per-row-block
// partial sums of (d - A_Omega)^2; partials has mc_partials(m) entries. When
// rank_dev >= need nothing is written but zero partials (the caller repeats
// the thresholding with a larger request first).
size_t mc_partials(int m);
template <typename T>
void mc_update(Timer* tm, int m, long long nnz, const int* row_ptr, const int* col_idx,
               const T* d, T* y, T* sv, const T* U, int ldu, const T* V, int ldv, const double* S,
               double eps, const int* rank_dev, int rmax, double mu, double mu_next, int need,
               double* partials, hipStream_t s);
// y[e] = alpha d[e] for e < nnz.
template <typename T>
void scale_copy(long long nnz, double alpha, const T* d, T* y, hipStream_t s);
template <typename T>
void mc_init(long long nnz, const T* d, T* y, T* sv, hipStream_t s);
void theta_out(int r, const double* S, double eps, double* Sout, hipStream_t s);

}  // namespace blws
