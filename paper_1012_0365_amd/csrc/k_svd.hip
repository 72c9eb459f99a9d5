// SVD of the small projected matrix B (N x N, FP64) of the BLWS step, whose
// singular values are the Ritz values (Algorithm 3 with Theorem 1).
//
// 1. Golub-Kahan bidiagonalisation B = Q_L Bd Q_R^T. Up to N = 224 in ONE
//    workgroup, B held in registers: a 32 x 16 thread grid, thread (tr, tc)
//    owning rows tr + 32a and columns tc + 16c. Up to N = 512 across
//    ceil(N / 32) co-resident workgroups holding 32-column slabs, with one
//    device-wide barrier per column. Each step is a left and a right
//    Householder reflection; their vectors are written to global memory for
//    the back-transformation.
// 2. Singular values of Bd by multisection on the Golub-Kahan tridiagonal
//    T = tridiag(0; d0, e0, d1, e1, ..., d_{N-1}) of size 2N, whose eigenvalues
//    are +-sigma (Theorem 1 applied to the bidiagonal): one wavefront per value,
//    64 Sturm counts per step.
// 3. Singular vectors by inverse iteration on T - sigma I: the eigenvector is
//    (v0, u0, v1, u1, ...), so u and v come out paired.
// 4. Back-transformation through the stored reflectors (one workgroup per
//    column block).
#include "blws_common.h"

namespace blws {
namespace {

constexpr int GK_MAXN = 224;   // one-workgroup bidiagonalisation
constexpr int SVD_MAXN = 512;  // cooperative bidiagonalisation and the later stages

// Start vectors of the inverse iteration: SplitMix64 (Steele, Lea & Flood
// 2014) outputs mapped to [-1, 1), distinct per value so that vectors of a
// multiple singular value start independent.
__device__ __forceinline__ double start_pm1(uint64_t counter)
{
    uint64_t z = 0x5DEECE66DULL + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}
constexpr int GK_LD = GK_MAXN + 1;  // padded LDS row of the partial sums

// Thread (tr, tc) of the 32 x 16 grid owns rows tr + 32a (a < NPR) and
// columns tc + 16c (c < 2 NPR): 7 x 14 doubles at N = 224, which 512 threads
// (two wavefronts per SIMD, 256 registers each) hold without spilling.
template <int NPR>
__global__ __launch_bounds__(512) void gk_bidiag_kernel(int N, const double* __restrict__ B,
                                                        int ldb, double* __restrict__ dout,
                                                        double* __restrict__ eout,
                                                        double* __restrict__ VL,
                                                        double* __restrict__ tauL,
                                                        double* __restrict__ VR,
                                                        double* __restrict__ tauR)
{
    constexpr int NPC = 2 * NPR;
    __shared__ double part[32 * GK_LD];
    __shared__ double sx[GK_MAXN], svl[GK_MAXN], sw[GK_MAXN];
    __shared__ double sy[GK_MAXN], svr[GK_MAXN], sz[GK_MAXN];
    __shared__ double stauL, stauR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tr = tid & 31, tc = tid >> 5;

    double Br[NPR][NPC];
#pragma unroll
    for (int a = 0; a < NPR; ++a)
#pragma unroll
        for (int c = 0; c < NPC; ++c) {
            const int i = tr + 32 * a, j = tc + 16 * c;
            Br[a][c] = (i < N && j < N) ? B[(size_t)i * ldb + j] : 0.0;
        }

    for (int k = 0; k < N; ++k) {
        // ---- left reflector: column k, rows k..N-1
        if (tc == (k & 15)) {
            const int kc = k >> 4;
#pragma unroll
            for (int a = 0; a < NPR; ++a) {
                const int i = tr + 32 * a;
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < NPC; ++c)
                    if (c == kc) v = Br[a][c];
                if (i >= k && i < N) sx[i] = v;
            }
        }
        __syncthreads();
        if (wave == 0) {
            const double alpha = sx[k];
            double s2 = 0.0;
            for (int i = k + 1 + lane; i < N; i += 64) s2 += sx[i] * sx[i];
            for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (s2 > 0.0) {
                const double nrm = sqrt(alpha * alpha + s2);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            for (int i = k + 1 + lane; i < N; i += 64) {
                const double v = sx[i] * scale;
                svl[i] = v;
                VL[(size_t)k * N + i] = v;
            }
            if (lane == 0) {
                svl[k] = 1.0;
                VL[(size_t)k * N + k] = 1.0;
                tauL[k] = tau;
                dout[k] = beta;
                stauL = tau;
            }
        }
        __syncthreads();
        const double tl = stauL;
        if (tl != 0.0) {
            // w_j = tau * sum_{i >= k} v_i B[i][j], j > k; v_i read once per row block
            double vi[NPR];
#pragma unroll
            for (int a = 0; a < NPR; ++a) {
                const int i = tr + 32 * a;
                vi[a] = (32 * a + 31 >= k && i >= k && i < N) ? svl[i] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < NPC; ++c) {
                if (16 * c + 15 < k + 1) continue;  // uniform: no column > k in this block
                const int j = tc + 16 * c;
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a < NPR; ++a) {
                    if (32 * a + 31 < k) continue;  // uniform: no row >= k in this block
                    acc += vi[a] * Br[a][c];
                }
                if (j < N) part[tr * GK_LD + j] = acc;
            }
            __syncthreads();
            if (tid < N && tid > k) {
                double s = 0.0;
                for (int r = 0; r < 32; ++r) s += part[r * GK_LD + tid];
                sw[tid] = tl * s;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < NPC; ++c) {
                if (16 * c + 15 < k + 1) continue;
                const int j = tc + 16 * c;
                const double wj = (j > k && j < N) ? sw[j] : 0.0;
#pragma unroll
                for (int a = 0; a < NPR; ++a) {
                    if (32 * a + 31 < k) continue;
                    Br[a][c] -= vi[a] * wj;
                }
            }
        }
        if (k + 1 >= N) break;
        // ---- right reflector: row k, columns k+1..N-1
        if (tr == (k & 31)) {
            const int ka = k >> 5;
#pragma unroll
            for (int c = 0; c < NPC; ++c) {
                const int j = tc + 16 * c;
                double v = 0.0;
#pragma unroll
                for (int a = 0; a < NPR; ++a)
                    if (a == ka) v = Br[a][c];
                if (j > k && j < N) sy[j] = v;
            }
        }
        __syncthreads();
        if (wave == 0) {
            const double alpha = sy[k + 1];
            double s2 = 0.0;
            for (int j = k + 2 + lane; j < N; j += 64) s2 += sy[j] * sy[j];
            for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (s2 > 0.0) {
                const double nrm = sqrt(alpha * alpha + s2);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            for (int j = k + 2 + lane; j < N; j += 64) {
                const double v = sy[j] * scale;
                svr[j] = v;
                VR[(size_t)k * N + j] = v;
            }
            if (lane == 0) {
                svr[k + 1] = 1.0;
                VR[(size_t)k * N + k + 1] = 1.0;
                tauR[k] = tau;
                eout[k] = beta;
                stauR = tau;
            }
        }
        __syncthreads();
        const double tq = stauR;
        if (tq != 0.0) {
            // z_i = tau * sum_{j > k} B[i][j] v_j, i > k: column-outer loops so
            // that only one accumulator per row block stays live
            double acc[NPR];
#pragma unroll
            for (int a = 0; a < NPR; ++a) acc[a] = 0.0;
#pragma unroll
            for (int c = 0; c < NPC; ++c) {
                if (16 * c + 15 < k + 1) continue;
                const int j = tc + 16 * c;
                const double vj = (j > k && j < N) ? svr[j] : 0.0;
#pragma unroll
                for (int a = 0; a < NPR; ++a) {
                    if (32 * a + 31 < k + 1) continue;
                    acc[a] += Br[a][c] * vj;
                }
            }
#pragma unroll
            for (int a = 0; a < NPR; ++a) {
                if (32 * a + 31 < k + 1) continue;
                const int i = tr + 32 * a;
                if (i < N) part[tc * GK_LD + i] = acc[a];
            }
            __syncthreads();
            if (tid < N && tid > k) {
                double sum = 0.0;
                for (int t = 0; t < 16; ++t) sum += part[t * GK_LD + tid];
                sz[tid] = tq * sum;
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < NPR; ++a) {
                const int i = tr + 32 * a;
                acc[a] = (32 * a + 31 >= k + 1 && i > k && i < N) ? sz[i] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < NPC; ++c) {
                if (16 * c + 15 < k + 1) continue;
                const int j = tc + 16 * c;
                const double vj = (j > k && j < N) ? svr[j] : 0.0;
#pragma unroll
                for (int a = 0; a < NPR; ++a) {
                    if (32 * a + 31 < k + 1) continue;
                    Br[a][c] -= acc[a] * vj;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Cooperative Golub-Kahan bidiagonalisation for GK_MAXN < N <= SVD_MAXN.
//
// P = ceil(N / 32) workgroups, all resident at once (cooperative launch).
// Workgroup p holds columns 32p .. 32p + 31 of B in registers: thread (g, c)
// of a 16 x 32 grid owns column 32p + c and rows g + 16q (q < NQ). Per step k:
//  - every workgroup forms the left reflector of column k on its own, from
//    the column as published in the previous step, and applies it to its
//    columns (no barrier needed);
//  - for the right reflector of row k (x = row k beyond the superdiagonal)
//    each workgroup publishes the sum of squares of its part of x and its
//    part of sum_j B[i][j] x_j, and the owner of column k + 1 publishes that
//    column; after ONE device-wide barrier every workgroup forms the
//    reflector, z = B v and the next column from these in a fixed order
//    (so all workgroups hold bit-identical copies) and updates its columns.
// The barrier waits are bounded: on a timeout the error flag is set and every
// workgroup leaves the kernel.
// ---------------------------------------------------------------------------
constexpr unsigned CO_SPIN_LIMIT = 1u << 22;

struct CoopBuf {
    double* colpub;  // 2 x N: column k + 1 before the right update
    double* nrm;     // 2 x P: partial sums of squares of row k
    double* part;    // 2 x P x N: partial products B x
    unsigned* ctr;   // barrier arrivals (zero at launch)
    int* err;        // set on a barrier timeout
};

__device__ __forceinline__ double ld_agent(double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier among the co-resident workgroups: release of this
// workgroup's writes, arrival count, bounded wait, acquire.
__device__ bool coop_barrier(unsigned* ctr, unsigned target, int* err, int* ok_lds)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > CO_SPIN_LIMIT) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *ok_lds = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *ok_lds != 0;
}

template <int NQ>
__global__ __launch_bounds__(512) void gk_bidiag_coop_kernel(
    int N, const double* __restrict__ B, int ldb, double* __restrict__ dout,
    double* __restrict__ eout, double* __restrict__ VL, double* __restrict__ tauL,
    double* __restrict__ VR, double* __restrict__ tauR, CoopBuf cb)
{
    __shared__ double xcol[SVD_MAXN];  // column k, then the left vector
    __shared__ double zs[SVD_MAXN];    // z = B v of the right reflector
    __shared__ double red[16][33];
    __shared__ double wcol[32];
    __shared__ double rowk[32];
    __shared__ double sc[4];
    __shared__ int okl;
    const int P = gridDim.x, p = blockIdx.x;
    const int tid = threadIdx.x, c = tid & 31, g = tid >> 5, lane = tid & 63, wave = tid >> 6;
    const int j = 32 * p + c;
    const bool jv = j < N;

    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = g + 16 * q;
        a[q] = (i < N && jv) ? B[(size_t)i * ldb + j] : 0.0;
    }
    for (int i = tid; i < N; i += 512) xcol[i] = B[(size_t)i * ldb];
    __syncthreads();

    for (int k = 0; k < N; ++k) {
        // ---- left reflector of column k (rows k..N-1), formed by every workgroup
        if (wave == 0) {
            const double alpha = xcol[k];
            double s2 = 0.0;
            for (int i = k + 1 + lane; i < N; i += 64) s2 += xcol[i] * xcol[i];
            for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (s2 > 0.0) {
                const double nrm = sqrt(alpha * alpha + s2);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            for (int i = k + 1 + lane; i < N; i += 64) {
                const double v = xcol[i] * scale;
                xcol[i] = v;
                if (p == 0) VL[(size_t)k * N + i] = v;
            }
            if (lane == 0) {
                xcol[k] = 1.0;
                sc[0] = tau;
                if (p == 0) {
                    VL[(size_t)k * N + k] = 1.0;
                    tauL[k] = tau;
                    dout[k] = beta;
                }
            }
        }
        __syncthreads();
        const double tl = sc[0];
        if (tl != 0.0) {
            // w_j = tau sum_{i >= k} u_i B[i][j] for own columns j > k
            double pw = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (16 * q + 15 < k) continue;  // uniform
                const int i = g + 16 * q;
                if (i >= k && i < N) pw += xcol[i] * a[q];
            }
            red[g][c] = pw;
            __syncthreads();
            if (tid < 32) {
                double w = 0.0;
                for (int gg = 0; gg < 16; ++gg) w += red[gg][tid];
                wcol[tid] = tl * w;
            }
            __syncthreads();
            const double wj = (jv && j > k) ? wcol[c] : 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (16 * q + 15 < k) continue;
                const int i = g + 16 * q;
                if (i >= k && i < N) a[q] -= xcol[i] * wj;
            }
        }
        if (k + 1 >= N) break;

        // ---- right reflector of row k: this workgroup's partials
        const int slot = k & 1;
        if (g == (k & 15)) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q == (k >> 4)) v = a[q];
            rowk[c] = jv ? v : 0.0;
        }
        __syncthreads();
        {
            const double xj = (jv && j >= k + 2) ? rowk[c] : 0.0;
            double* prow = cb.part + ((size_t)slot * P + p) * N;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (16 * q + 15 < k + 1) continue;  // uniform
                const int i = g + 16 * q;
                double sq = a[q] * xj;
                for (int off = 16; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
                if (c == 0 && i >= k + 1 && i < N) st_agent(prow + i, sq);
            }
        }
        if (tid == 0) {
            double s2 = 0.0;
            for (int cc = 0; cc < 32; ++cc) {
                const int jj = 32 * p + cc;
                if (jj >= k + 2 && jj < N) s2 += rowk[cc] * rowk[cc];
            }
            st_agent(cb.nrm + slot * P + p, s2);
        }
        if (p == ((k + 1) >> 5) && c == ((k + 1) & 31)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = g + 16 * q;
                if (i >= k && i < N) st_agent(cb.colpub + (size_t)slot * N + i, a[q]);
            }
        }
        if (!coop_barrier(cb.ctr, (unsigned)(k + 1) * (unsigned)P, cb.err, &okl)) return;

        // ---- the reflector, z = B v and the next column, from the partials
        if (tid == 0) {
            const double alpha = ld_agent(cb.colpub + (size_t)slot * N + k);
            double s2 = 0.0;
            for (int q = 0; q < P; ++q) s2 += ld_agent(cb.nrm + slot * P + q);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (s2 > 0.0) {
                const double nrm = sqrt(alpha * alpha + s2);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
            sc[1] = tau;
            sc[2] = scale;
            if (p == 0) {
                tauR[k] = tau;
                eout[k] = beta;
            }
        }
        __syncthreads();
        const double tq = sc[1], scl = sc[2];
        for (int i = k + 1 + tid; i < N; i += 512) {
            double acc = 0.0;
            for (int q = 0; q < P; ++q) acc += ld_agent(cb.part + ((size_t)slot * P + q) * N + i);
            const double cp = ld_agent(cb.colpub + (size_t)slot * N + i);
            const double z = cp + scl * acc;
            zs[i] = z;
            xcol[i] = cp - tq * z;
        }
        if (g == 0 && jv && j >= k + 1) VR[(size_t)k * N + j] = (j == k + 1) ? 1.0 : rowk[c] * scl;
        __syncthreads();
        if (tq != 0.0) {
            const double vj = (jv && j >= k + 1) ? ((j == k + 1) ? 1.0 : rowk[c] * scl) : 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (16 * q + 15 < k + 1) continue;
                const int i = g + 16 * q;
                if (i >= k + 1 && i < N) a[q] -= tq * zs[i] * vj;
            }
        }
        __syncthreads();  // rowk, zs and sc are rewritten in the next step
    }
}

// Number of singular values of the bidiagonal (d, e) that are >= x (x > 0),
// from the Sturm count of the Golub-Kahan tridiagonal T (zero diagonal,
// off-diagonals f2 squared): #{eig(T) < x} = N + #{sigma < x}. The LDL^T
// recurrence q_j = -x - f_{j-1}^2 / q_{j-1} counts negative pivots.
__device__ int count_ge(int N, const double* f2, double x, double pivmin)
{
    int neg = 0;
    double q = -x;
    if (fabs(q) < pivmin) q = -pivmin;
    neg += q < 0.0;
    for (int j = 1; j < 2 * N; ++j) {
        q = -x - f2[j - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        neg += q < 0.0;
    }
    return 2 * N - neg;  // = N - #{sigma < x}
}

// One wavefront per singular value: sigma_t, the t-th largest, by multisection.
__global__ __launch_bounds__(64) void tgk_bisect_kernel(int N, const double* __restrict__ d,
                                                        const double* __restrict__ e,
                                                        double* __restrict__ sig)
{
    __shared__ double f2[2 * SVD_MAXN];
    __shared__ int cnt[64];
    const int t = blockIdx.x, lane = threadIdx.x;
    double bound = 0.0, fmax2 = 0.0;
    for (int j = lane; j < 2 * N - 1; j += 64) {
        const double f = (j & 1) ? e[j >> 1] : d[j >> 1];
        f2[j] = f * f;
    }
    __syncthreads();
    for (int j = 0; j < 2 * N - 1; ++j) fmax2 = fmax(fmax2, f2[j]);
    // Gershgorin bound of T: max_j |f_{j-1}| + |f_j|
    for (int j = 0; j < 2 * N; ++j) {
        const double l = j > 0 ? sqrt(f2[j - 1]) : 0.0;
        const double r = j < 2 * N - 1 ? sqrt(f2[j]) : 0.0;
        bound = fmax(bound, l + r);
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, fmax2);
    double lo = 0.0, hi = bound * (1.0 + 4.0 * 0x1.0p-52) + pivmin;
    // invariant: #{sigma >= lo} >= t + 1 (lo = 0 counts every value), #{sigma >= hi} <= t
    for (int step = 0; step < 14; ++step) {
        // relative precision 2u, or absolute u * ||T|| for values near zero
        if (hi - lo <= 2.0 * 0x1.0p-52 * fmax(fabs(lo), fabs(hi)) + pivmin ||
            hi - lo <= 0x1.0p-52 * bound)
            break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        cnt[lane] = count_ge(N, f2, x, pivmin);
        __syncthreads();
        // largest point still holding >= t + 1 values
        int best = -1;
        for (int l = 0; l < 64; ++l)
            if (cnt[l] >= t + 1) best = l;
        const double nlo = best >= 0 ? lo + (hi - lo) * (double)(best + 1) / 65.0 : lo;
        const double nhi = best < 63 ? lo + (hi - lo) * (double)(best + 2) / 65.0 : hi;
        lo = nlo;
        hi = nhi;
        __syncthreads();
    }
    // a value the bracket cannot separate from zero is reported as zero
    const bool zero = lo == 0.0 && hi <= 8.0 * 0x1.0p-52 * bound + 4.0 * pivmin;
    if (lane == 0) sig[t] = zero ? 0.0 : 0.5 * (lo + hi);
}

// Inverse iteration for the eigenvector of T at +sigma_t: LU factorisation
// with partial pivoting of the tridiagonal T - sigma I (row interchanges give
// U a second superdiagonal), then three solves from a fixed +-1 start vector,
// normalising each time. The eigenvector z = (v0, u0, v1, u1, ...) splits into
// the bidiagonal's right and left singular vectors. Work arrays live in LDS;
// one wavefront per value, the sequential recurrences on lane 0.
__global__ __launch_bounds__(64) void tgk_invit_kernel(int N, const double* __restrict__ d,
                                                       const double* __restrict__ e,
                                                       const double* __restrict__ sig,
                                                       double* __restrict__ ubd,
                                                       double* __restrict__ vbd, int ldv)
{
    __shared__ double f[2 * SVD_MAXN];
    __shared__ double z[2 * SVD_MAXN], dl[2 * SVD_MAXN], dd[2 * SVD_MAXN], du[2 * SVD_MAXN],
        du2[2 * SVD_MAXN];
    __shared__ unsigned char swp[2 * SVD_MAXN];
    const int t = blockIdx.x, lane = threadIdx.x;
    const int n = 2 * N;
    for (int j = lane; j < n - 1; j += 64) f[j] = (j & 1) ? e[j >> 1] : d[j >> 1];
    __syncthreads();
    if (lane == 0) {
        const double s = sig[t];
        double fm = fabs(s);
        for (int j = 0; j < n - 1; ++j) fm = fmax(fm, fabs(f[j]));
        const double tiny = fm * 0x1.0p-52 + 1e-300;
        for (int j = 0; j < n; ++j) {
            dd[j] = -s;
            if (j < n - 1) {
                dl[j] = f[j];
                du[j] = f[j];
            }
            if (j < n - 2) du2[j] = 0.0;
        }
        for (int j = 0; j < n - 1; ++j) {
            if (fabs(dd[j]) >= fabs(dl[j])) {
                swp[j] = 0;
                const double fact = dd[j] != 0.0 ? dl[j] / dd[j] : 0.0;
                dl[j] = fact;
                dd[j + 1] -= fact * du[j];
                if (j < n - 2) du2[j] = 0.0;
            } else {
                swp[j] = 1;
                const double fact = dd[j] / dl[j];
                dd[j] = dl[j];
                dl[j] = fact;
                const double tmp = du[j];
                du[j] = dd[j + 1];
                dd[j + 1] = tmp - fact * dd[j + 1];
                if (j < n - 2) {
                    du2[j] = du[j + 1];
                    du[j + 1] = -fact * du[j + 1];
                }
            }
        }
        for (int j = 0; j < n; ++j)
            if (fabs(dd[j]) < tiny) dd[j] = dd[j] < 0.0 ? -tiny : tiny;
        for (int j = 0; j < n; ++j)
            z[j] = start_pm1((uint64_t)t * 4096ULL + (uint64_t)j);
        for (int it = 0; it < 2; ++it) {
            for (int j = 0; j < n - 1; ++j) {
                if (!swp[j]) {
                    z[j + 1] -= dl[j] * z[j];
                } else {
                    const double tmp = z[j];
                    z[j] = z[j + 1];
                    z[j + 1] = tmp - dl[j] * z[j];
                }
            }
            z[n - 1] /= dd[n - 1];
            if (n >= 2) z[n - 2] = (z[n - 2] - du[n - 2] * z[n - 1]) / dd[n - 2];
            for (int j = n - 3; j >= 0; --j)
                z[j] = (z[j] - du[j] * z[j + 1] - du2[j] * z[j + 2]) / dd[j];
            double mx = 0.0;
            for (int j = 0; j < n; ++j) mx = fmax(mx, fabs(z[j]));
            const double inv = mx > 0.0 ? 1.0 / mx : 0.0;
            for (int j = 0; j < n; ++j) z[j] *= inv;
        }
    }
    __syncthreads();
    // split and normalise each half to unit length
    double nu = 0.0, nv = 0.0;
    for (int i = lane; i < N; i += 64) {
        nv += z[2 * i] * z[2 * i];
        nu += z[2 * i + 1] * z[2 * i + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        nu += __shfl_xor(nu, off, 64);
        nv += __shfl_xor(nv, off, 64);
    }
    nu = nu > 0.0 ? 1.0 / sqrt(nu) : 0.0;
    nv = nv > 0.0 ? 1.0 / sqrt(nv) : 0.0;
    for (int i = lane; i < N; i += 64) {
        vbd[(size_t)i * ldv + t] = z[2 * i] * nv;
        ubd[(size_t)i * ldv + t] = z[2 * i + 1] * nu;
    }
}

// X (N x nv, ld) <- H_0 H_1 ... H_{nref-1} X for reflectors stored column-wise
// in Vh (column k: entries k+off .. N-1, unit at k+off), tau[k]. One wavefront
// per column of X (four per workgroup), the column in registers (N <= 64 R);
// reflectors staged through LDS RCH at a time, applied last to first.
template <int MAXN, int RCH, int R>
__global__ __launch_bounds__(256) void reflect_apply_kernel(int N, int nref, int off,
                                                            const double* __restrict__ Vh,
                                                            const double* __restrict__ tau,
                                                            double* __restrict__ X, int ldx,
                                                            int nv)
{
    __shared__ double vs[RCH][MAXN];
    __shared__ double ts[RCH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = blockIdx.x * 4 + wave;
    double xr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
        xr[r] = (col < nv && i < N) ? X[(size_t)i * ldx + col] : 0.0;
    }
    for (int k1 = nref - 1; k1 >= 0; k1 -= RCH) {
        const int k0 = k1 - RCH + 1 < 0 ? 0 : k1 - RCH + 1;
        const int cnt = k1 - k0 + 1;
        __syncthreads();
        for (int e = tid; e < cnt * N; e += 256) {
            const int q = e / N, i = e - q * N;
            const int k = k0 + q;
            vs[q][i] = (i >= k + off) ? Vh[(size_t)k * N + i] : 0.0;
        }
        if (tid < cnt) ts[tid] = tau[k0 + tid];
        __syncthreads();
        for (int q = cnt - 1; q >= 0; --q) {
            const double tk = ts[q];
            if (tk == 0.0) continue;
            double dot = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = lane + 64 * r;
                if (i < N) dot += vs[q][i] * xr[r];
            }
            for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
            const double w = tk * dot;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = lane + 64 * r;
                if (i < N) xr[r] -= vs[q][i] * w;
            }
        }
    }
    if (col < nv) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lane + 64 * r;
            if (i < N) X[(size_t)i * ldx + col] = xr[r];
        }
    }
}

// Sign convention: the largest-magnitude entry of each left vector positive
// (the right vector flips with it).
__global__ void sign_fix_kernel(int N, int nv, double* UB, double* VB, int ld)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nv) return;
    int imax = 0;
    double vmax = 0.0;
    for (int i = 0; i < N; ++i) {
        const double a = fabs(UB[(size_t)i * ld + t]);
        if (a > vmax) {
            vmax = a;
            imax = i;
        }
    }
    if (UB[(size_t)imax * ld + t] < 0.0)
        for (int i = 0; i < N; ++i) {
            UB[(size_t)i * ld + t] = -UB[(size_t)i * ld + t];
            VB[(size_t)i * ld + t] = -VB[(size_t)i * ld + t];
        }
}

}  // namespace

bool small_svd_gk_supported(int N) { return N >= 2 && N <= SVD_MAXN; }

size_t small_svd_gk_scratch_elems(int N)
{
    // d, e, tauL, tauR, the reflector vectors VL, VR, and for the cooperative
    // bidiagonalisation the published column, partials and barrier counter
    const size_t P = (N + 31) / 32;
    return 4 * (size_t)N + 2 * (size_t)N * N + 2 * (size_t)N + 2 * P + 2 * P * N + 8;
}

// Outputs: S[0..nv), UB, VB (N x N, ld N) with their first nv columns set.
void small_svd_gk(Timer* tm, int N, int nv, const double* B, int ldb, double* UB, double* S,
                  double* VB, double* scratch, int* err, hipStream_t s)
{
    BLWS_REQUIRE(small_svd_gk_supported(N) && nv >= 1 && nv <= N, BLWS_EUNSUPPORTED,
                 "small_svd_gk: size out of range");
    double* d = scratch;
    double* e = d + N;
    double* tL = e + N;
    double* tR = tL + N;
    double* VL = tR + N;
    double* VR = VL + (size_t)N * N;
    static const char* const coop_fam[4] = {"gk_bidiag_coop_q20", "gk_bidiag_coop_q24",
                                            "gk_bidiag_coop_q28", "gk_bidiag_coop_q32"};
    static const char* const one_fam[7] = {"gk_bidiag_p1", "gk_bidiag_p2", "gk_bidiag_p3",
                                           "gk_bidiag_p4", "gk_bidiag_p5", "gk_bidiag_p6",
                                           "gk_bidiag_p7"};
    // bidiagonalisation flops: 4 N^3 - 4 N^3 / 3 (Householder, both sides)
    const double bd_flops = 8.0 / 3.0 * N * (double)N * N;
    if (N > GK_MAXN) {
        const int NQc = (N + 15) / 16;
        const int qi = NQc <= 20 ? 0 : NQc <= 24 ? 1 : NQc <= 28 ? 2 : 3;
        TimedLaunch tl(tm, coop_fam[qi], s, bd_flops, 16.0 * N * N);
        const int P = (N + 31) / 32;
        CoopBuf cb;
        cb.colpub = VR + (size_t)N * N;
        cb.nrm = cb.colpub + 2 * (size_t)N;
        cb.part = cb.nrm + 2 * (size_t)P;
        cb.ctr = (unsigned*)(cb.part + 2 * (size_t)P * N);
        cb.err = err;
        HIP_TRY(hipMemsetAsync(cb.ctr, 0, sizeof(unsigned), s));
        void* args[] = {(void*)&N,  (void*)&B,  (void*)&ldb, (void*)&d,  (void*)&e,
                        (void*)&VL, (void*)&tL, (void*)&VR,  (void*)&tR, (void*)&cb};
        const void* fn = nullptr;
        const int NQ = (N + 15) / 16;
        if (NQ <= 20) fn = (const void*)gk_bidiag_coop_kernel<20>;
        else if (NQ <= 24) fn = (const void*)gk_bidiag_coop_kernel<24>;
        else if (NQ <= 28) fn = (const void*)gk_bidiag_coop_kernel<28>;
        else fn = (const void*)gk_bidiag_coop_kernel<32>;
        HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(P), dim3(512), args, 0, s));
    } else {
        const int NP = (N + 31) / 32;
        TimedLaunch tl(tm, one_fam[NP - 1], s, bd_flops, 16.0 * N * N);
#define BLWS_GK_CASE(P)                                                                      \
    case P:                                                                                  \
        hipLaunchKernelGGL((gk_bidiag_kernel<P>), dim3(1), dim3(512), 0, s, N, B, ldb, d, e, VL, \
                           tL, VR, tR);                                                      \
        break;
        switch (NP) {
            BLWS_GK_CASE(1)
            BLWS_GK_CASE(2)
            BLWS_GK_CASE(3)
            BLWS_GK_CASE(4)
            BLWS_GK_CASE(5)
            BLWS_GK_CASE(6)
            default:
                BLWS_GK_CASE(7)
        }
#undef BLWS_GK_CASE
    }
    {
        TimedLaunch tl(tm, "tgk_solve", s, 0.0, 0.0);
        hipLaunchKernelGGL(tgk_bisect_kernel, dim3(nv), dim3(64), 0, s, N, d, e, S);
        hipLaunchKernelGGL(tgk_invit_kernel, dim3(nv), dim3(64), 0, s, N, d, e, S, UB, VB, N);
    }
    {
        TimedLaunch tl(tm, "gk_backtransform", s, 4.0 * N * (double)N * nv, 0.0);
        const int blocks = (nv + 3) / 4;
        if (N <= GK_MAXN) {
            hipLaunchKernelGGL((reflect_apply_kernel<GK_MAXN, 16, 4>), dim3(blocks), dim3(256), 0,
                               s, N, N, 0, VL, tL, UB, N, nv);
            hipLaunchKernelGGL((reflect_apply_kernel<GK_MAXN, 16, 4>), dim3(blocks), dim3(256), 0,
                               s, N, N - 1, 1, VR, tR, VB, N, nv);
        } else {
            hipLaunchKernelGGL((reflect_apply_kernel<SVD_MAXN, 8, 8>), dim3(blocks), dim3(256), 0,
                               s, N, N, 0, VL, tL, UB, N, nv);
            hipLaunchKernelGGL((reflect_apply_kernel<SVD_MAXN, 8, 8>), dim3(blocks), dim3(256), 0,
                               s, N, N - 1, 1, VR, tR, VB, N, nv);
        }
        hipLaunchKernelGGL(sign_fix_kernel, dim3((nv + 63) / 64), dim3(64), 0, s, N, nv, UB, VB,
                           N);
    }
}

}  // namespace blws
