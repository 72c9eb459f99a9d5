// Small dense FP64 kernels of the BLWS step: the Cholesky factor of the Gram
// matrix used to orthonormalise the new Lanczos block (the QR step
// (X_{l+1}, B_l) = qr(R_l) of Algorithm 2, done as Cholesky-QR), and the SVD of
// the 2b x 2b projected matrix whose singular values are the Ritz values
// (Algorithm 3 with Theorem 1). Both run in one workgroup.
#include "blws_common.h"

namespace blws {
namespace {

constexpr int CHOL_LDS_MAX = 128;  // Gram matrices up to 128 x 128 live in LDS

typedef double d4 __attribute__((ext_vector_type(4)));

// Scaled LDL^T elimination of the Gram matrix G = X^T X, tracking L^{-1} in the
// strictly lower triangle of the same array (the trailing matrix lives in the
// upper triangle). With d the pivots and s_i = G_ii^{-1/2}:
//   R^{-1}[r][c] = s_r * (L^{-1})[c][r] / sqrt(d_c),  r <= c,
// so X R^{-1} has orthonormal columns. A pivot <= eta (the squared sine of the
// angle between a scaled column and the span of the earlier ones) marks the
// column as dependent: it is skipped and its R^{-1} column is zero.
template <bool LDS>
__global__ __launch_bounds__(1024) void chol_inv_kernel(int n, const double* __restrict__ G,
                                                        int ldg, double* __restrict__ Rinv,
                                                        int* flags, int* nflag, double eta,
                                                        double* gscratch)
{
    __shared__ double lds[LDS ? CHOL_LDS_MAX * CHOL_LDS_MAX : 1];
    __shared__ double scal[512];
    __shared__ int flg[512];
    double* S = LDS ? lds : gscratch;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int i = tid; i < n; i += nth) {
        const double g = G[(size_t)i * ldg + i];
        scal[i] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
        flg[i] = 0;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, k = e - i * n;
        S[e] = (k >= i) ? G[(size_t)i * ldg + k] * scal[i] * scal[k] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double piv = S[j * n + j];
        if (!(piv > eta)) {
            if (tid == 0) flg[j] = 1;
        } else {
            const double inv = 1.0 / piv;
            const int rows = n - j - 1;
            const int items = rows * n;
            for (int e = tid; e < items; e += nth) {
                const int i = j + 1 + e / n, col = e % n;
                const double l = S[j * n + i] * inv;
                if (col >= i) {
                    S[i * n + col] -= l * S[j * n + col];
                } else if (col < j) {
                    S[i * n + col] -= l * S[j * n + col];
                } else if (col == j) {
                    S[i * n + j] = -l;
                }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += nth) {
        const int r = e / n, c = e - r * n;
        double v = 0.0;
        if (r <= c && !flg[c]) {
            const double lic = (r == c) ? 1.0 : S[c * n + r];
            v = scal[r] * lic / sqrt(S[c * n + c]);
        }
        Rinv[e] = v;
    }
    int cnt = 0;
    for (int i = tid; i < n; i += nth) {
        flags[i] = flg[i];
        cnt += flg[i];
    }
    if (cnt) atomicAdd(nflag, cnt);
}

// 1 / p from the hardware estimate and two Newton steps, e <- 1 - p r,
// r <- r + r e (each squares the relative error); the same instruction
// sequence in every thread, so all of them hold the same bits.
__device__ __forceinline__ double recip_nr(double p)
{
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// Steps j of row group JB (32 JB <= j < 32 JB + 32) of the register
// elimination below. The trailing matrix is kept in both triangles, so every
// element takes the same update S[i][c] -= l_i row_j[c] (l_i = 0 for rows
// i <= j): the upper copies are the Schur complement that later pivots are
// taken from, the lower copies of columns c < j hold L^{-1} (column c is
// overwritten with -l_i when it is eliminated), and the lower copies of
// columns c > j are never read. Row groups above JB are finished and skipped
// at compile time.
template <int JB>
__device__ __forceinline__ void chol_inv_steps(int n, double (&S)[4][4], double* rowbuf, double* piv,
                                               int* flg, double eta)
{
    if constexpr (JB < 4) {
        const int tid = threadIdx.x, tr = tid >> 5, tc = tid & 31;
        const int jend = min(32 * JB + 32, n);
        for (int j = 32 * JB; j < jend; ++j) {
            double* row = rowbuf + 128 * (j & 1);
            // the owners of row j (row group JB) publish it
            if (tr == (j & 31)) {
#pragma unroll
                for (int b = 0; b < 4; ++b) row[tc + 32 * b] = S[JB][b];
            }
            __syncthreads();
            const double p = row[j];
            const bool dep = !(p > eta);
            if (tid == 0) {
                piv[j] = p;
                flg[j] = dep ? 1 : 0;
            }
            if (!dep) {
                const double inv = recip_nr(p);
                double rc[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) rc[b] = row[tc + 32 * b];
                const bool jcol = tc == (j & 31);  // column j is tc + 32 JB
#pragma unroll
                for (int a = JB; a < 4; ++a) {
                    const int i = tr + 32 * a;
                    const double l = (i > j) ? row[i] * inv : 0.0;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const double v = fma(-l, rc[b], S[a][b]);
                        if (b == JB)
                            S[a][b] = (jcol && i > j) ? -l : v;
                        else
                            S[a][b] = v;
                    }
                }
            }
        }
        chol_inv_steps<JB + 1>(n, S, rowbuf, piv, flg, eta);
    }
}

// The same elimination with the matrix in registers (n <= 128): thread
// (tr, tc) of a 32 x 32 grid holds S[tr + 32a][tc + 32b], a, b < 4. Each step
// broadcasts the pivot row through LDS, alternating between the two halves of
// `rowbuf` (2 x 128 doubles): the barrier after step j + 1's broadcast also
// orders every read of step j before step j + 2 overwrites that half, so one
// barrier per step. G (full, symmetric) and Rinv (leading dimension ld) may be
// global or LDS; Rinv may alias G (G is read once into registers before Rinv
// is written). All 1024 threads call it.
__device__ __forceinline__ void chol_inv_regs(int n, const double* G, int ldg, double* Rinv, int ldr, double eta,
                              double* scal, double* rowbuf, double* piv, int* flg)
{
    const int tid = threadIdx.x, tr = tid >> 5, tc = tid & 31;
    for (int i = tid; i < n; i += 1024) {
        const double g = G[(size_t)i * ldg + i];
        scal[i] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
        flg[i] = 0;
    }
    __syncthreads();
    double S[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = tr + 32 * a, c = tc + 32 * b;
            S[a][b] = (i < n && c < n) ? G[(size_t)i * ldg + c] * scal[i] * scal[c] : 0.0;
        }
    __syncthreads();  // G fully read before Rinv (which may alias it) is written
    chol_inv_steps<0>(n, S, rowbuf, piv, flg, eta);
    __syncthreads();
    // R^{-1}[r][c] = s_r (L^{-1})[c][r] / sqrt(d_c), r <= c; thread (i, col)
    // holds (L^{-1})[i][col] for col < i and writes element (col, i).
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = tr + 32 * a;
        if (i >= n) continue;
        const double rs = flg[i] ? 0.0 : 1.0 / sqrt(piv[i]);  // one root per row
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int c = tc + 32 * b;
            if (c >= n) continue;
            const double lic = (c == i) ? 1.0 : S[a][b];
            Rinv[(size_t)c * ldr + i] = (c <= i) ? scal[c] * lic * rs : 0.0;
        }
    }
    __syncthreads();
}

// Thread (ty, tx) of an 8 x 128 grid (1024 threads) loads rows ty + 8 k,
// k < 16, of column tx of the n x n matrix G (n <= 128, leading dimension
// ldg) into g[k], every load issued before any is used, and returns the
// largest |G - I| over the workgroup (dev_w: 16 doubles of LDS).
__device__ __forceinline__ double load_dev_from_identity(int n, const double* G, int ldg,
                                                         double (&g)[16], double* dev_w)
{
    const int tid = threadIdx.x, ty = tid >> 7, tx = tid & 127;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = ty + 8 * k;
        g[k] = (i < n && tx < n) ? G[(size_t)i * ldg + tx] : 0.0;
    }
    double dv = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = ty + 8 * k;
        if (i < n && tx < n) dv = fmax(dv, fabs(g[k] - (i == tx ? 1.0 : 0.0)));
    }
    for (int off = 32; off > 0; off >>= 1) dv = fmax(dv, __shfl_xor(dv, off, 64));
    if ((tid & 63) == 0) dev_w[tid >> 6] = dv;
    __syncthreads();
    double m = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) m = fmax(m, dev_w[w]);
    return m;
}

__global__ __launch_bounds__(1024) void chol_inv_reg_kernel(int n, const double* __restrict__ G,
                                                            int ldg, double* __restrict__ Rinv,
                                                            int* flags, int* nflag, double eta,
                                                            double ni_tol)
{
    __shared__ double scal[128];
    __shared__ double row[2 * 128];
    __shared__ double piv[128];
    __shared__ int flg[128];
    __shared__ double dev_w[16];
    const int tid = threadIdx.x;
    // Columns already orthonormal (the second Cholesky-QR pass of a block):
    // with E = G - I and ||E||_2 <= n max|E_ij| <= ni_tol, R^{-1} is replaced
    // by (3 I - G) / 2, with which X R^{-1} has the Gram matrix
    // I - 3 E^2 / 4 + O(E^3), and no column is dependent.
    double g[16];
    if ((double)n * load_dev_from_identity(n, G, ldg, g, dev_w) <= ni_tol) {
        const int ty = tid >> 7, tx = tid & 127;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int i = ty + 8 * k;
            if (i < n && tx < n) Rinv[(size_t)i * n + tx] = (i == tx ? 1.5 : 0.0) - 0.5 * g[k];
        }
        for (int i = tid; i < n; i += 1024) flags[i] = 0;
        return;
    }
    chol_inv_regs(n, G, ldg, Rinv, n, eta, scal, row, piv, flg);
    int cnt = 0;
    for (int i = tid; i < n; i += 1024) {
        flags[i] = flg[i];
        cnt += flg[i];
    }
    if (cnt) atomicAdd(nflag, cnt);
}

// Two Cholesky-QR passes on the columns of X (rows x c, ld; rows <= 512,
// c <= 128) in ONE workgroup per matrix (blockIdx.x picks X0 or X1): the Gram
// matrix by FP64 MFMA into LDS, the Cholesky inverse in registers (in place
// in LDS), X <- X R^{-1} in place row by row. Columns found dependent in the
// first pass are redrawn from the counter-based generator (stream ids sid0,
// sid1) before the second; *nflag counts them. When the first Gram matrix is
// already the identity to 1e-8, one pass of X <- X (3 I - G) / 2 replaces
// both.
constexpr int CQ_LD = 129;

// Gram matrices G_s = X_s^T X_s (rows x c, c <= 128) of the two sides, one
// wavefront per 16 x 16 tile (grid T*T x 2), two interleaved MFMA chains over
// the rows; G_s is c x c, row-major.
__global__ __launch_bounds__(64) void polish_gram_kernel(int rows, int c, const double* X0,
                                                         const double* X1, int ld, double* G0,
                                                         double* G1)
{
    const double* X = blockIdx.y == 0 ? X0 : X1;
    double* G = blockIdx.y == 0 ? G0 : G1;
    const int T = (c + 15) / 16;
    const int ti = blockIdx.x / T, tj = blockIdx.x - ti * T;
    const int lane = threadIdx.x;
    const int ca = 16 * ti + (lane & 15), cb = 16 * tj + (lane & 15);
    d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
    // batches of 16 rows (four k-steps), the next batch's loads in flight
    // while the current one feeds the matrix cores; loads are unconditional,
    // from clamped in-range addresses, and masked only when used, so that
    // neither a branch nor a select waits on them early
    double a0[4], b0[4], a1[4], b1[4];
    const int cac = min(ca, c - 1), cbc = min(cb, c - 1);
    auto fetch = [&](int k0, double (&av)[4], double (&bv)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u + (lane >> 4);
            const double* xr = X + (size_t)min(k, rows - 1) * ld;
            av[u] = xr[cac];
            bv[u] = xr[cbc];
        }
        // keeps the compiler from merging the two register sets' loads
        asm volatile("" ::: "memory");
    };
    auto compute = [&](int k0, const double (&av)[4], const double (&bv)[4]) {
#pragma unroll
        for (int u = 0; u < 4; u += 2) {
            const int k = k0 + 4 * u + (lane >> 4);
            const bool i0 = k < rows, i1 = k + 4 < rows;
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64((i0 && ca < c) ? av[u] : 0.0,
                                                        (i0 && cb < c) ? bv[u] : 0.0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64((i1 && ca < c) ? av[u + 1] : 0.0,
                                                        (i1 && cb < c) ? bv[u + 1] : 0.0, acc1, 0,
                                                        0, 0);
        }
    };
    // (the prefetches past the last row read clamped rows and go unused:
    // unconditional, they leave no branch for the wait counts to merge over)
    fetch(0, a0, b0);
    for (int k0 = 0; k0 < rows; k0 += 32) {  // uniform trip count
        fetch(k0 + 16, a1, b1);
        compute(k0, a0, b0);
        if (k0 + 16 >= rows) break;
        fetch(k0 + 32, a0, b0);
        compute(k0 + 16, a1, b1);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 16 * ti + (lane >> 4) + 4 * i;
        if (r < c && cb < c) G[(size_t)r * c + cb] = acc0[i] + acc1[i];
    }
}

__global__ __launch_bounds__(1024) void cholqr2_small_kernel(int rows, int c, double* X0, double* X1,
                                                             int ld, int* nflag, double eta,
                                                             uint64_t seed, uint64_t sid0,
                                                             uint64_t sid1, const double* G0pre,
                                                             const double* G1pre)
{
    __shared__ double G[128 * CQ_LD];
    __shared__ double scal[128], row[2 * 128], piv[128];
    __shared__ int flg[128];
    __shared__ double dev_w[16];
    __shared__ int one_pass;
    __shared__ double Xs[16][128];
    double* X = blockIdx.x == 0 ? X0 : X1;
    const uint64_t sid = blockIdx.x == 0 ? sid0 : sid1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int T = (c + 15) / 16;
    {
        // The side's Gram matrix, formed beforehand by polish_gram_kernel. When
        // ||G - I||_2 <= c max|G_ij - I_ij| <= 1e-8 (the usual case), X (3 I - G) / 2
        // is orthonormal to 3 ||G - I||^2 / 4 <= 1e-16: workgroup (side, rb) replaces rows 16 rb ..
        // 16 rb + 15 of X by X (3 I - G) / 2, a column tile per wavefront, and
        // nothing else is done. Otherwise workgroup (side, 0) runs the two
        // Cholesky-QR passes below and the others leave.
        const double* Gp = blockIdx.x == 0 ? G0pre : G1pre;
        double g[16];
        if ((double)c * load_dev_from_identity(c, Gp, c, g, dev_w) <= 1e-8) {
            const int r0 = 16 * blockIdx.y;
            {
                const int ty = tid >> 7, tx = tid & 127;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int i = ty + 8 * k;
                    if (i < c && tx < c) G[i * CQ_LD + tx] = (i == tx ? 1.5 : 0.0) - 0.5 * g[k];
                }
            }
            for (int j = lane; j < c; j += 64)  // row r0 + wave of the block
                Xs[wave][j] = r0 + wave < rows ? X[(size_t)(r0 + wave) * ld + j] : 0.0;
            __syncthreads();
            if (wave < T) {  // uniform per wavefront
                const int cb = 16 * wave + (lane & 15);
                d4 acc = d4{0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < c; k0 += 4) {
                    const int k = k0 + (lane >> 4);
                    const double a = k < c ? Xs[lane & 15][k] : 0.0;
                    const double b = (k < c && cb < c) ? G[k * CQ_LD + cb] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = r0 + (lane >> 4) + 4 * i;
                    if (r < rows && cb < c) X[(size_t)r * ld + cb] = acc[i];
                }
            }
            return;
        }
        if (blockIdx.y != 0) return;
        __syncthreads();  // dev_w is reused
    }
    for (int pass = 0; pass < 2; ++pass) {
        // Gram G = X^T X: 16 x 16 tiles, wavefront w takes tiles w + 16 u,
        // two at a time (independent MFMA chains)
        for (int u0 = 0; u0 < 4; u0 += 2) {
            const int t0 = wave + 16 * u0, t1 = t0 + 16;
            const bool v0 = t0 / 8 < T && t0 % 8 < T, v1 = t1 / 8 < T && t1 % 8 < T;
            if (!v0 && !v1) continue;  // uniform per wavefront
            const int ca0 = 16 * (t0 / 8) + (lane & 15), cb0 = 16 * (t0 % 8) + (lane & 15);
            const int ca1 = 16 * (t1 / 8) + (lane & 15), cb1 = 16 * (t1 % 8) + (lane & 15);
            d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
            for (int k0 = 0; k0 < rows; k0 += 4) {  // uniform trip count
                const int k = k0 + (lane >> 4);
                const bool kin = k < rows;
                const double* xr = X + (size_t)(kin ? k : 0) * ld;
                const double a0 = (kin && v0 && ca0 < c) ? xr[ca0] : 0.0;
                const double b0 = (kin && v0 && cb0 < c) ? xr[cb0] : 0.0;
                const double a1 = (kin && v1 && ca1 < c) ? xr[ca1] : 0.0;
                const double b1 = (kin && v1 && cb1 < c) ? xr[cb1] : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r0 = 16 * (t0 / 8) + (lane >> 4) + 4 * i;
                const int r1 = 16 * (t1 / 8) + (lane >> 4) + 4 * i;
                if (v0 && r0 < c && cb0 < c) G[r0 * CQ_LD + cb0] = acc0[i];
                if (v1 && r1 < c && cb1 < c) G[r1 * CQ_LD + cb1] = acc1[i];
            }
        }
        __syncthreads();
        if (pass == 0) {
            // Columns already orthonormal to 1e-8 (the usual case for inverse
            // iteration vectors): one pass leaves them orthonormal to rounding
            // (its error is of order u cond(G), cond(G) <= 1 + 2e-8), so the
            // second is skipped.
            double dv = 0.0;
            for (int e = tid; e < c * c; e += 1024) {
                const int i = e / c, j = e - i * c;
                dv = fmax(dv, fabs(G[i * CQ_LD + j] - (i == j ? 1.0 : 0.0)));
            }
            for (int off = 32; off > 0; off >>= 1) dv = fmax(dv, __shfl_xor(dv, off, 64));
            if (lane == 0) dev_w[wave] = dv;
            __syncthreads();
            if (tid == 0) {
                double m = 0.0;
                for (int w = 0; w < 16; ++w) m = fmax(m, dev_w[w]);
                one_pass = m <= 1e-8 ? 1 : 0;
            }
            __syncthreads();
        }
        if (pass == 0 && one_pass) {
            // G = I + E with |E| <= 1e-8: X (3 I - G) / 2 is orthonormal to
            // O(|E|^2) (its Gram matrix is I - 3 E^2 / 4 + O(E^3)), the
            // symmetric orthonormalisation to first order, with no Cholesky
            // factorisation; no column is dependent
            for (int e = tid; e < c * c; e += 1024) {
                const int i = e / c, j = e - i * c;
                G[i * CQ_LD + j] = (i == j ? 1.5 : 0.0) - 0.5 * G[i * CQ_LD + j];
            }
            for (int j = tid; j < c; j += 1024) flg[j] = 0;
            __syncthreads();
        } else {
            chol_inv_regs(c, G, CQ_LD, G, CQ_LD, eta, scal, row, piv, flg);
        }
        // X <- X R^{-1} by MFMA: wavefront w owns row blocks w, w + 16, ... (16
        // rows each, all column tiles), so each row block is read completely
        // before it is overwritten
        for (int rb = wave; rb * 16 < rows; rb += 16) {
            d4 acc[8];
#pragma unroll
            for (int tj = 0; tj < 8; ++tj) acc[tj] = d4{0.0, 0.0, 0.0, 0.0};
            const int ra = 16 * rb + (lane & 15);
            const double* xa = X + (size_t)(ra < rows ? ra : 0) * ld;
#pragma unroll 2
            for (int k0 = 0; k0 < c; k0 += 4) {
                const int k = k0 + (lane >> 4);
                const double a = (ra < rows && k < c) ? xa[k] : 0.0;
#pragma unroll
                for (int tj = 0; tj < 8; ++tj) {
                    if (tj >= T) break;  // uniform
                    const int cb = 16 * tj + (lane & 15);
                    const double b = (k < c && cb < c) ? G[k * CQ_LD + cb] : 0.0;
                    acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[tj], 0, 0, 0);
                }
            }
#pragma unroll
            for (int tj = 0; tj < 8; ++tj) {
                if (tj >= T) break;
                const int cb = 16 * tj + (lane & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * rb + (lane >> 4) + 4 * i;
                    if (r < rows && cb < c) X[(size_t)r * ld + cb] = acc[tj][i];
                }
            }
        }
        __syncthreads();
        if (pass == 0) {
            for (int e = tid; e < rows * c; e += 1024) {
                const int i = e / c, j = e - i * c;
                if (flg[j])
                    X[(size_t)i * ld + j] =
                        uniform_pm1(seed, (sid << 40) + (uint64_t)i * 4096ULL + (uint64_t)j);
            }
        }
        if (tid == 0) {
            int cnt = 0;
            for (int j = 0; j < c; ++j) cnt += flg[j];
            if (cnt) atomicAdd(nflag, cnt);
        }
        __syncthreads();
        if (one_pass) break;  // uniform (set before the barriers of chol_inv_regs)
    }
}

// SVD of a 1 x 1 matrix: the left vector +1 (the sign convention), the
// value |b|, the right vector sign(b) (+1 for b = 0).
__global__ void svd1_kernel(const double* B, double* UB, double* S, double* VB)
{
    const double v = B[0];
    UB[0] = 1.0;
    S[0] = fabs(v);
    VB[0] = v < 0.0 ? -1.0 : 1.0;
}

template <typename T>
__global__ void fill_uniform_kernel(int rows, int cols, T* X, int ldx, uint64_t seed,
                                    uint64_t stream_id)
{
    const size_t total = (size_t)rows * cols;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / cols), j = (int)(e - (size_t)i * cols);
        X[(size_t)i * ldx + j] =
            (T)uniform_pm1(seed, (stream_id << 40) + (uint64_t)i * 4096ULL + (uint64_t)j);
    }
}

template <typename TS, typename TD>
__global__ void copy2d_kernel(int rows, int cols, const TS* src, int lds, TD* dst, int ldd)
{
    const size_t total = (size_t)rows * cols;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / cols), j = (int)(e - (size_t)i * cols);
        dst[(size_t)i * ldd + j] = (TD)src[(size_t)i * lds + j];
    }
}

__global__ void zero_words_kernel(unsigned* p, size_t words)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < words;
         e += (size_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

__global__ void count_above_kernel(int b, const double* S, double eps, int* out)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int c = 0;
    for (int i = threadIdx.x; i < b; i += blockDim.x) c += S[i] > eps;
    if (c) atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) out[0] = cnt;
}

// ---------------------------------------------------------------------------
// Columns of a Cholesky-QR block that the Gram matrix cannot resolve.
//
// A column whose scaled pivot is <= eta (the squared sine of the angle between
// the column and the span of the ones before it) is known to the Gram matrix
// only to about c u / sin^2, so the Cholesky-QR passes give it a zero column.
// This pass re-forms each such column j from the vectors themselves: x_j as
// the first pass saw it is orthogonalised by classical Gram-Schmidt against
// the blocks the chunk is projected out of and against every finished column
// of the result, the pass repeated while it removes more than half of the
// norm squared (at most three: "twice is enough" with Kahan's test), and
// normalised. Its direction is then accurate to about u / sin, so the span of
// the result holds x_j to rounding, as a Householder QR of the block would.
// When the residual is below keep_tol |x_j| (x_j in the span to rounding:
// exact breakdown), the counter-based draws uniform_pm1(seed, (sid << 40) +
// 4096 i + j) take the column's place and are orthogonalised the same way.
// One workgroup; it returns at once when no column is flagged.
// ---------------------------------------------------------------------------
constexpr int FB_MAXW = 2048;  // widest basis [Xa, Xb, Q] the pass handles

// sum over the workgroup of one value per wavefront (the same in all its
// lanes); every thread adds the 16 partial sums in the same order
__device__ __forceinline__ double fb_wave_total(double v, double* red)
{
    const int tid = threadIdx.x;
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += red[w];
    return t;
}

__device__ __forceinline__ double fb_wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__global__ __launch_bounds__(1024) void orth_fallback_kernel(
    int rows, int c, const int* __restrict__ flags0, const int* __restrict__ flags1,
    const T* __restrict__ src, int lds, T* Q, int ldq, const T* __restrict__ Xa, int lda, int ba,
    const T* __restrict__ Xb, int ldb, int bb, double* xv, int* nflag, double keep_tol,
    uint64_t seed, uint64_t sid)
{
    __shared__ double coef[FB_MAXW];
    __shared__ double xs[1024];
    __shared__ double red[16];
    __shared__ int fl[128];  // 1: a column still to re-form; 0: a finished column
    __shared__ int nfl, nnew;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        nfl = 0;
        nnew = 0;
    }
    __syncthreads();
    if (tid < c) {
        const int f0 = flags0[tid] != 0, f1 = flags1[tid] != 0;
        fl[tid] = f0 | f1;
        if (f0 | f1) atomicAdd(&nfl, 1);
        if (f1 && !f0) atomicAdd(&nnew, 1);  // the first pass counted its own
    }
    __syncthreads();
    if (nfl == 0) return;
    if (tid == 0 && nnew) atomicAdd(nflag, nnew);
    const int W = ba + bb + c;
    // basis column k: Xa (k < ba), Xb (k < ba + bb), then the chunk's columns
    auto column = [&](int k, const T*& p, int& ld) -> bool {
        if (k < ba) {
            p = Xa + k;
            ld = lda;
            return true;
        }
        if (k < ba + bb) {
            p = Xb + (k - ba);
            ld = ldb;
            return true;
        }
        if (k < W) {
            p = Q + (k - ba - bb);
            ld = ldq;
            return !fl[k - ba - bb];
        }
        p = nullptr;
        ld = 0;
        return false;
    };
    for (int j = 0; j < c; ++j) {
        if (!fl[j]) continue;  // uniform: LDS
        double nn = 0.0;
        for (int attempt = 0; attempt < 2; ++attempt) {
            double n0 = 0.0;
            for (int r = tid; r < rows; r += 1024) {
                const double v =
                    attempt == 0
                        ? (double)src[(size_t)r * lds + j]
                        : uniform_pm1(seed, (sid << 40) + (uint64_t)r * 4096ULL + (uint64_t)j);
                xv[r] = v;
                n0 += v * v;
            }
            n0 = fb_wave_total(fb_wave_sum(n0), red);
            double prev = n0;
            nn = n0;
            for (int pass = 0; pass < 3; ++pass) {
                // coef[k] = (basis column k)^T x, zero for the columns left out
                const T *p0, *p1;
                int l0, l1;
                const bool on0 = column(tid, p0, l0), on1 = column(tid + 1024, p1, l1);
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                for (int r0 = 0; r0 < rows; r0 += 1024) {
                    const int len = min(1024, rows - r0);
                    __syncthreads();  // the previous chunk's readers are done
                    if (tid < len) xs[tid] = xv[r0 + tid];
                    __syncthreads();
                    if (on0) {
                        int t = 0;
                        for (; t + 1 < len; t += 2) {
                            a0 += (double)p0[(size_t)(r0 + t) * l0] * xs[t];
                            a1 += (double)p0[(size_t)(r0 + t + 1) * l0] * xs[t + 1];
                        }
                        if (t < len) a0 += (double)p0[(size_t)(r0 + t) * l0] * xs[t];
                    }
                    if (on1) {
                        int t = 0;
                        for (; t + 1 < len; t += 2) {
                            a2 += (double)p1[(size_t)(r0 + t) * l1] * xs[t];
                            a3 += (double)p1[(size_t)(r0 + t + 1) * l1] * xs[t + 1];
                        }
                        if (t < len) a2 += (double)p1[(size_t)(r0 + t) * l1] * xs[t];
                    }
                }
                if (tid < W) coef[tid] = on0 ? a0 + a1 : 0.0;
                if (tid + 1024 < W) coef[tid + 1024] = on1 ? a2 + a3 : 0.0;
                __syncthreads();
                // x <- x - B coef, one row per wavefront at a time
                double wn = 0.0;
                for (int r = wave; r < rows; r += 16) {
                    double a = 0.0;
                    for (int k = lane; k < ba; k += 64) a += coef[k] * (double)Xa[(size_t)r * lda + k];
                    for (int k = lane; k < bb; k += 64)
                        a += coef[ba + k] * (double)Xb[(size_t)r * ldb + k];
                    for (int k = lane; k < c; k += 64)
                        a += coef[ba + bb + k] * (double)Q[(size_t)r * ldq + k];
                    a = fb_wave_sum(a);
                    const double x = xv[r] - a;
                    if (lane == 0) xv[r] = x;
                    wn += x * x;
                }
                nn = fb_wave_total(wn, red);
                const bool enough = nn > 0.5 * prev;
                prev = nn;
                if (enough) break;
            }
            if (nn > keep_tol * keep_tol * n0) break;  // attempt 1: a draw, kept as it is
        }
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int r = tid; r < rows; r += 1024) Q[(size_t)r * ldq + j] = (T)(xv[r] * inv);
        __syncthreads();
        if (tid == 0) fl[j] = 0;
        __syncthreads();
    }
}

int grid_for(size_t total)
{
    size_t b = (total + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

size_t chol_scratch_elems(int n) { return n > CHOL_LDS_MAX ? (size_t)n * n : 0; }

void chol_inv(Timer* tm, int n, const double* G, int ldg, double* Rinv, int* flags, int* nflag,
              double eta, double ni_tol, double* scratch, hipStream_t s)
{
    BLWS_REQUIRE(n >= 1 && n <= 512, BLWS_EUNSUPPORTED, "chol_inv: block width above 512");
    TimedLaunch tl(tm, "chol", s, (double)n * n * n / 3.0, 16.0 * n * n);
    if (n <= 128)
        hipLaunchKernelGGL(chol_inv_reg_kernel, dim3(1), dim3(1024), 0, s, n, G, ldg, Rinv, flags,
                           nflag, eta, ni_tol);
    else if (n <= CHOL_LDS_MAX)
        hipLaunchKernelGGL((chol_inv_kernel<true>), dim3(1), dim3(1024), 0, s, n, G, ldg, Rinv,
                           flags, nflag, eta, (double*)nullptr);
    else
        hipLaunchKernelGGL((chol_inv_kernel<false>), dim3(1), dim3(1024), 0, s, n, G, ldg, Rinv,
                           flags, nflag, eta, scratch);
}

bool cholqr2_small_supported(int rows, int c) { return rows >= 1 && rows <= 512 && c >= 1 && c <= 128; }

void cholqr2_small(Timer* tm, int rows, int c, double* X0, double* X1, int ld, int* nflag,
                   double eta, uint64_t seed, uint64_t sid0, uint64_t sid1, double* G0, double* G1,
                   hipStream_t s)
{
    BLWS_REQUIRE(cholqr2_small_supported(rows, c), BLWS_EUNSUPPORTED, "cholqr2_small: size");
    TimedLaunch tl(tm, "svd_polish", s, 2.0 * 2.0 * (2.0 * rows * (double)c * c + c * (double)c * c / 3.0),
                   0.0);
    const int T = (c + 15) / 16;
    hipLaunchKernelGGL(polish_gram_kernel, dim3(T * T, 2), dim3(64), 0, s, rows, c, X0, X1, ld, G0,
                       G1);
    hipLaunchKernelGGL(cholqr2_small_kernel, dim3(2, (rows + 15) / 16), dim3(1024), 0, s, rows, c,
                       X0, X1, ld, nflag, eta, seed, sid0, sid1, G0, G1);
}

void small_svd_1x1(const double* B, double* UB, double* S, double* VB, hipStream_t s)
{
    hipLaunchKernelGGL(svd1_kernel, dim3(1), dim3(1), 0, s, B, UB, S, VB);
}

template <typename T>
void fill_uniform(int rows, int cols, T* X, int ldx, uint64_t seed, uint64_t stream_id,
                  hipStream_t s)
{
    hipLaunchKernelGGL((fill_uniform_kernel<T>), dim3(grid_for((size_t)rows * cols)), dim3(256), 0,
                       s, rows, cols, X, ldx, seed, stream_id);
}

template <typename TS, typename TD>
void copy2d(int rows, int cols, const TS* src, int lds, TD* dst, int ldd, hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL((copy2d_kernel<TS, TD>), dim3(grid_for((size_t)rows * cols)), dim3(256), 0,
                       s, rows, cols, src, lds, dst, ldd);
}

void zero_bytes(void* p, size_t bytes, hipStream_t s)
{
    BLWS_REQUIRE(bytes % 4 == 0 && ((uintptr_t)p & 3) == 0, BLWS_EINVAL,
                 "zero_bytes: size or address not a multiple of 4");
    if (bytes == 0) return;
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for(bytes / 4)), dim3(256), 0, s,
                       (unsigned*)p, bytes / 4);
}

void count_above(int b, const double* S, double eps, int* rank_out, hipStream_t s)
{
    hipLaunchKernelGGL(count_above_kernel, dim3(1), dim3(256), 0, s, b, S, eps, rank_out);
}

template <typename T>
void orth_fallback(Timer* tm, int rows, int c, const int* flags0, const int* flags1, const T* src,
                   int lds, T* Q, int ldq, const T* Xa, int lda, int ba, const T* Xb, int ldb,
                   int bb, double* xv, int* nflag, uint64_t seed, uint64_t sid, hipStream_t s)
{
    if (rows <= 0 || c <= 0) return;
    BLWS_REQUIRE(c <= 128 && ba + bb + c <= FB_MAXW && (ba == 0 || Xa) && (bb == 0 || Xb),
                 BLWS_EUNSUPPORTED, "orth_fallback: block wider than the pass handles");
    TimedLaunch tl(tm, "orth_fallback", s, 0.0, 0.0);
    // below this relative residual the column lies in the span to the
    // storage precision's rounding, and a draw takes its place
    const double keep_tol = sizeof(T) == 4 ? 1e-6 : 1e-14;
    hipLaunchKernelGGL((orth_fallback_kernel<T>), dim3(1), dim3(1024), 0, s, rows, c, flags0,
                       flags1, src, lds, Q, ldq, Xa, lda, ba, Xb, ldb, bb, xv, nflag, keep_tol,
                       seed, sid);
}

template void orth_fallback<double>(Timer*, int, int, const int*, const int*, const double*, int,
                                    double*, int, const double*, int, int, const double*, int, int,
                                    double*, int*, uint64_t, uint64_t, hipStream_t);
template void orth_fallback<float>(Timer*, int, int, const int*, const int*, const float*, int,
                                   float*, int, const float*, int, int, const float*, int, int,
                                   double*, int*, uint64_t, uint64_t, hipStream_t);
template void fill_uniform<double>(int, int, double*, int, uint64_t, uint64_t, hipStream_t);
template void fill_uniform<float>(int, int, float*, int, uint64_t, uint64_t, hipStream_t);
template void copy2d<double, double>(int, int, const double*, int, double*, int, hipStream_t);
template void copy2d<float, float>(int, int, const float*, int, float*, int, hipStream_t);
template void copy2d<float, double>(int, int, const float*, int, double*, int, hipStream_t);
template void copy2d<double, float>(int, int, const double*, int, float*, int, hipStream_t);

}  // namespace blws
