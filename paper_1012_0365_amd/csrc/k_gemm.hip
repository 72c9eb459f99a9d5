// Skinny GEMMs on CDNA4 matrix cores.
//
// Every product of the BLWS step has one small dimension: the block products
// W V, W^T U, W G (Algorithm 2: the products of the augmented matrix with the
// Lanczos blocks) have N = b columns; the projections and Gram matrices
// X^T Y have a b x b output and a long K; the block updates X S have K <= 2b.
// One kernel family covers them all: C = alpha op(A) B + beta C with
// op(A) = A or A^T, B row-major K x N. A workgroup owns a 64-row strip of C
// and 16 * NT of its columns, four wavefronts each computing 16 rows with
// v_mfma_f64_16x16x4f64 tiles. Tiles of op(A) and B are staged through LDS,
// converted to the compute type on the way in. Long K is split across
// workgroups (split-K); the partial sums are reduced in a fixed order by a
// second kernel, so results do not depend on scheduling.
#include <algorithm>

#include "blws_common.h"

namespace blws {
namespace {

constexpr int BM = 64;  // rows of C per workgroup (4 wavefronts x 16)
constexpr int BK = 32;  // K per LDS stage (8 MFMA steps of 4)
constexpr int NTHREADS = 256;
constexpr int GROUP_MAX = GEMM_GROUP_MAX;  // problems per grouped launch

typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ double ld_d(const T* p) { return (double)(*p); }

// One 64 x 16 nt block (nt <= NT column tiles, nt uniform) of C, K range of
// split bz: the body shared by the single-problem kernel and the grouped one.
// As is BK x (BM + 1), Bs is BK x ldbs (ldbs >= 16 nt + 1) doubles of LDS.
// An element's products are accumulated in the same order whatever nt is.
template <typename TA, typename TB, typename TC, bool TRANS, int NT>
__device__ __forceinline__ void gemm_f64_block(double* As, double* Bs, int ldbs, int bx, int by,
                                               int bz, int nt, int M, int N, int K, int kchunk,
                                               double alpha, const TA* __restrict__ A, int lda,
                                               const TB* __restrict__ B, int ldb, double beta,
                                               const TC* Cin, int ldcin, TC* C, int ldc,
                                               double* __restrict__ partial)
{
    constexpr int LDA_S = BM + 1;
    const int BN = 16 * nt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = bx * BM, c0 = by * BN;
    const int kb = bz * kchunk;
    const int ke = min(K, kb + kchunk);

    d4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};

    // The next stage's tiles are loaded into registers while the current
    // one feeds the matrix cores: A 8 values per thread (NN: 4 threads read 32
    // consecutive k of one row; TN: 8 threads read 64 consecutive columns of
    // one row), B 2 NT values (element e = tid + 256 u of the BK x BN tile).
    // (held in the storage types and widened when stored to LDS, so that no
    // conversion waits on a load in flight)
    constexpr int NB = (BK * 16 * NT + NTHREADS - 1) / NTHREADS;
    TA ra[8];
    TB rb[NB];
    auto fetch = [&](int k0) {
        if (!TRANS) {
            const int row = tid >> 2, kq = (tid & 3) * 8;
            const int gr = r0 + row;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gk = k0 + kq + u;
                ra[u] = (gr < M && gk < ke) ? A[(size_t)gr * lda + gk] : TA(0);
            }
        } else {
            const int kr = tid >> 3, rq = (tid & 7) * 8;
            const int gk = k0 + kr;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gr = r0 + rq + u;
                ra[u] = (gr < M && gk < ke) ? A[(size_t)gk * lda + gr] : TA(0);
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + NTHREADS * u;
            const int kr = e / BN, cc = e - kr * BN;
            const int gk = k0 + kr, gc = c0 + cc;
            rb[u] = (e < BK * BN && gk < ke && gc < N) ? B[(size_t)gk * ldb + gc] : TB(0);
        }
    };
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        if (!TRANS) {
            const int row = tid >> 2, kq = (tid & 3) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) As[(kq + u) * LDA_S + row] = (double)ra[u];
        } else {
            const int kr = tid >> 3, rq = (tid & 7) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) As[kr * LDA_S + rq + u] = (double)ra[u];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + NTHREADS * u;
            const int kr = e / BN, cc = e - kr * BN;
            if (e < BK * BN) Bs[kr * ldbs + cc] = (double)rb[u];
        }
        __syncthreads();
        if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const double a = As[(kk * 4 + (lane >> 4)) * LDA_S + wave * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if (j >= nt) break;  // uniform
                const double bv = Bs[(kk * 4 + (lane >> 4)) * ldbs + j * 16 + (lane & 15)];
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // C layout of the FP64 16x16 tile (measured on gfx950): register i of lane l
    // holds row (l / 16) + 4 i, column l % 16.
    const int rbase = r0 + wave * 16 + (lane >> 4);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        if (j >= nt) break;
        const int col = c0 + j * 16 + (lane & 15);
        if (col >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rbase + 4 * i;
            if (row >= M) continue;
            const double v = acc[j][i];
            if (partial) {
                partial[((size_t)bz * M + row) * N + col] = v;
            } else {
                double out = alpha * v;
                if (beta != 0.0) out += beta * (double)Cin[(size_t)row * ldcin + col];
                C[(size_t)row * ldc + col] = (TC)out;
            }
        }
    }
}

template <typename TA, typename TB, typename TC, bool TRANS, int NT>
__global__ __launch_bounds__(NTHREADS) void gemm_f64_kernel(
    int M, int N, int K, int kchunk, double alpha, const TA* __restrict__ A, int lda,
    const TB* __restrict__ B, int ldb, double beta, const TC* Cin, int ldcin, TC* C, int ldc,
    double* __restrict__ partial)
{
    __shared__ double As[BK * (BM + 1)];
    __shared__ double Bs[BK * (16 * NT + 1)];
    gemm_f64_block<TA, TB, TC, TRANS, NT>(As, Bs, 16 * NT + 1, blockIdx.x, blockIdx.y, blockIdx.z,
                                          NT, M, N, K, kchunk, alpha, A, lda, B, ldb, beta, Cin,
                                          ldcin, C, ldc, partial);
}

// Grouped W-products (FP64): up to GROUP_MAX problems C_q = op_q(A_q) B_q in
// one launch, each with the block grid and K split it has alone (so the same
// results, bit for bit); block b belongs to problem q with
// start[q] <= b < start[q + 1].
struct GroupF64 {
    int n;
    int start[GROUP_MAX + 1];
    struct Prob {
        int M, N, K, kchunk, gx, gy, nt, trans, lda, ldb, ldc, splits;
        const double *A, *B;
        double *C, *partial;
    } p[GROUP_MAX];
};

__device__ __forceinline__ int group_find(const int* start, int n, int blk)
{
    int q = 0;
    while (q + 1 < n && blk >= start[q + 1]) ++q;
    return q;
}

__global__ __launch_bounds__(NTHREADS) void gemm_f64_grouped_kernel(GroupF64 g)
{
    __shared__ double As[BK * (BM + 1)];
    __shared__ double Bs[BK * (16 * 8 + 1)];
    const int q = group_find(g.start, g.n, blockIdx.x);
    const GroupF64::Prob& P = g.p[q];
    const int l = blockIdx.x - g.start[q], per = P.gx * P.gy;
    const int bz = l / per, rem = l - bz * per, by = rem / P.gx, bx = rem - by * P.gx;
    double* part = P.splits > 1 ? P.partial : nullptr;
    if (P.trans)
        gemm_f64_block<double, double, double, true, 8>(As, Bs, 16 * 8 + 1, bx, by, bz, P.nt, P.M,
                                                        P.N, P.K, P.kchunk, 1.0, P.A, P.lda, P.B,
                                                        P.ldb, 0.0, nullptr, 0, P.C, P.ldc, part);
    else
        gemm_f64_block<double, double, double, false, 8>(As, Bs, 16 * 8 + 1, bx, by, bz, P.nt, P.M,
                                                         P.N, P.K, P.kchunk, 1.0, P.A, P.lda, P.B,
                                                         P.ldb, 0.0, nullptr, 0, P.C, P.ldc, part);
}

// sum_s partial[s][e], s = 0 .. S-1 in order (eight loads in flight)
__device__ __forceinline__ double sum_splits(const double* partial, size_t total, size_t e, int S)
{
    double acc = 0.0;
    int s = 0;
    for (; s + 8 <= S; s += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(s + u) * total + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; s < S; ++s) acc += partial[(size_t)s * total + e];
    return acc;
}

// C = alpha * sum_s partial[s] + beta * Cin, summed in split order.
template <typename TC>
__global__ void splitk_reduce_kernel(int M, int N, int S, double alpha, const double* partial,
                                     double beta, const TC* Cin, int ldcin, TC* C, int ldc)
{
    const size_t total = (size_t)M * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const double acc = sum_splits(partial, total, e, S);
        const int row = (int)(e / N), col = (int)(e - (size_t)row * N);
        double out = alpha * acc;
        if (beta != 0.0) out += beta * (double)Cin[(size_t)row * ldcin + col];
        C[(size_t)row * ldc + col] = (TC)out;
    }
}

// The same sum for many splits (S >= RED_WIDE_MIN_S): a workgroup per 64
// consecutive elements, wavefront w adding splits w q .. w q + q - 1 in order
// (q = ceil(S / 4)) with sixteen loads in flight, and the four wavefront sums
// added in wavefront order, so the result does not depend on scheduling.
constexpr int RED_WIDE_MIN_S = 16;

template <typename TC>
__global__ __launch_bounds__(256) void splitk_reduce_wide_kernel(int M, int N, int S, double alpha,
                                                                 const double* __restrict__ partial,
                                                                 double beta, const TC* Cin,
                                                                 int ldcin, TC* C, int ldc)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t total = (size_t)M * N;
    const size_t e = (size_t)blockIdx.x * 64 + lane;
    const int q = (S + 3) / 4, s0 = wave * q, s1 = min(S, s0 + q);
    double acc = 0.0;
    if (e < total) {
        for (int s = s0; s < s1; s += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = s + u < s1 ? partial[(size_t)(s + u) * total + e] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v[u];
        }
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && e < total) {
        const double sum = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        const int row = (int)(e / N), col = (int)(e - (size_t)row * N);
        double out = alpha * sum;
        if (beta != 0.0) out += beta * (double)Cin[(size_t)row * ldcin + col];
        C[(size_t)row * ldc + col] = (TC)out;
    }
}

// C = alpha * sum_s partial[s] + beta * Cin by whichever reduction suits S.
template <typename TC>
void splitk_reduce(int M, int N, int S, double alpha, const double* partial, double beta,
                   const TC* Cin, int ldcin, TC* C, int ldc, hipStream_t s)
{
    const size_t total = (size_t)M * N;
    if (S >= RED_WIDE_MIN_S) {
        hipLaunchKernelGGL((splitk_reduce_wide_kernel<TC>), dim3((unsigned)((total + 63) / 64)),
                           dim3(256), 0, s, M, N, S, alpha, partial, beta, Cin, ldcin, C, ldc);
        return;
    }
    int blocks = (int)((total + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL((splitk_reduce_kernel<TC>), dim3(blocks), dim3(256), 0, s, M, N, S, alpha,
                       partial, beta, Cin, ldcin, C, ldc);
}

// The split-K sums of a grouped launch: problem q owns blocks start[q] ..
// start[q + 1] - 1 (the same sums, in the same order, as alone).
struct GroupRedF64 {
    int n;
    int start[GROUP_MAX + 1];
    struct Prob {
        int M, N, S, ldc;
        const double* partial;
        double* C;
    } p[GROUP_MAX];
};

__global__ void splitk_reduce_grouped_kernel(GroupRedF64 g)
{
    const int q = group_find(g.start, g.n, blockIdx.x);
    const GroupRedF64::Prob& P = g.p[q];
    const int nb = g.start[q + 1] - g.start[q], lb = blockIdx.x - g.start[q];
    const size_t total = (size_t)P.M * P.N;
    for (size_t e = lb * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)nb * blockDim.x) {
        const double acc = sum_splits(P.partial, total, e, P.S);
        const int row = (int)(e / P.N), col = (int)(e - (size_t)row * P.N);
        P.C[(size_t)row * P.ldc + col] = 1.0 * acc;
    }
}

struct Plan {
    int nt, gy, gx, splits, kchunk;
};

Plan make_plan(int M, int N, int K)
{
    Plan p;
    p.nt = N >= 128 ? 8 : (N + 15) / 16;
    if (p.nt < 1) p.nt = 1;
    p.gy = (N + 16 * p.nt - 1) / (16 * p.nt);
    p.gx = (M + BM - 1) / BM;
    const long tiles = (long)p.gx * p.gy;
    // Aim at the tuned workgroup count (~384, 1.5 per CU, outside the tuned
    // shapes), each split no shorter than 4 LDS stages, and keep the partial
    // sums below 4M doubles.
    const long target = plan_target(0, M, N, K, 384);
    long s = (target + tiles - 1) / tiles;
    const long smax_k = (K + 4 * BK - 1) / (4 * BK);
    if (s > smax_k) s = smax_k;
    const long smax_mem = (4L << 20) / ((long)M * N > 0 ? (long)M * N : 1);
    if (s > smax_mem) s = smax_mem;
    if (s < 1) s = 1;
    int kchunk = (int)((K + s - 1) / s);
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    if (kchunk < BK) kchunk = BK;
    p.kchunk = kchunk;
    p.splits = (K + kchunk - 1) / kchunk;
    if (p.splits < 1) p.splits = 1;
    return p;
}

template <typename TA, typename TB, typename TC, bool TRANS>
void launch_nt(const Plan& p, int M, int N, int K, double alpha, const TA* A, int lda,
               const TB* B, int ldb, double beta, const TC* Cin, int ldcin, TC* C, int ldc,
               double* partial, hipStream_t s)
{
    dim3 grid(p.gx, p.gy, p.splits), block(NTHREADS);
#define BLWS_GEMM_CASE(NTV)                                                                 \
    case NTV:                                                                               \
        hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, TC, TRANS, NTV>), grid, block, 0, s, M, N, \
                           K, p.kchunk, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc,    \
                           partial);                                                        \
        break;
    switch (p.nt) {
        BLWS_GEMM_CASE(1)
        BLWS_GEMM_CASE(2)
        BLWS_GEMM_CASE(3)
        BLWS_GEMM_CASE(4)
        BLWS_GEMM_CASE(5)
        BLWS_GEMM_CASE(6)
        BLWS_GEMM_CASE(7)
        default:
            BLWS_GEMM_CASE(8)
    }
#undef BLWS_GEMM_CASE
}


// ---------------------------------------------------------------------------
// Tall-skinny shapes. The generic kernel above gives a 64-row strip to each
// workgroup and runs its K range in LDS stages: for the orthonormalisation
// products (M ~ 2000, N ~ 112) that is ~32 workgroups on a 256-CU chip. Two
// dedicated forms instead:
//  - NN with K <= SK_MAXK: one workgroup per 16-row strip of C (and group
//    of column tiles, when C has few strips); the strip of A is staged once
//    in LDS (transposed, so fragment reads are unit-stride), B fragments are
//    read straight from L2, the four wavefronts take interleaved 16-column
//    tiles;
//  - TN with M, N <= TN_MAXMN and long K: a workgroup owns a 64 x 64 block of
//    C and one K chunk (LDS stages of 32 rows); the chunks' partial blocks are
//    summed in chunk order by the split-K reduction, so results do not depend
//    on scheduling.
// ---------------------------------------------------------------------------
constexpr int SK_MAXK = 512;
constexpr int TN_MAXMN = 512;
constexpr int TN_BK = 32;
#ifndef BLWS_TN_TARGET_WG
#define BLWS_TN_TARGET_WG 256
#endif
constexpr int TN_TARGET_WG = BLWS_TN_TARGET_WG;  // workgroups a long-K TN product aims at

template <typename TA, typename TB, typename TC, int NTW>
__global__ __launch_bounds__(256) void gemm_nn_sk_kernel(int M, int N, int K, double alpha,
                                                         const TA* __restrict__ A, int lda,
                                                         const TB* __restrict__ B, int ldb,
                                                         double beta, const TC* Cin, int ldcin,
                                                         TC* C, int ldc, const int* flags,
                                                         uint64_t seed, uint64_t sid)
{
    __shared__ double AsT[SK_MAXK][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * 16;
    const int K4 = (K + 3) & ~3;
    {
        // wavefront w stages rows w, w + 4, w + 8, w + 12 of the strip, every
        // load issued before the first LDS store
        constexpr int KCH = SK_MAXK / 64;
        TA st[4][KCH];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gr = r0 + wave + 4 * q;
#pragma unroll
            for (int u = 0; u < KCH; ++u) {
                const int k = lane + 64 * u;
                st[q][u] = (64 * u < K4 && gr < M && k < K) ? A[(size_t)gr * lda + k] : TA(0);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < KCH; ++u) {
                const int k = lane + 64 * u;
                if (k < K4) AsT[k][wave + 4 * q] = (double)st[q][u];
            }
    }
    __syncthreads();
    const int kq = lane >> 4, cl = lane & 15;
    d4 acc[NTW];
    int col[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        acc[t] = d4{0.0, 0.0, 0.0, 0.0};
        col[t] = 16 * (4 * NTW * (int)blockIdx.y + wave + 4 * t) + cl;
    }
    // B fragments by groups of PF k-steps, the next group's loads in flight
    // while the current one feeds the matrix cores
    constexpr int PF = NTW >= 8 ? 2 : (NTW >= 4 ? 4 : (NTW >= 2 ? 8 : 16));
    const int nst = K4 / 4, ng = (nst + PF - 1) / PF;
    TB b0[PF][NTW], b1[PF][NTW];  // storage type, widened at use
    auto load = [&](int g, TB (&bq)[PF][NTW]) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int k = 4 * (g * PF + u) + kq;
#pragma unroll
            for (int t = 0; t < NTW; ++t)
                bq[u][t] = (k < K && col[t] < N) ? B[(size_t)k * ldb + col[t]] : TB(0);
        }
    };
    auto compute = [&](int g, const TB (&bq)[PF][NTW]) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            if (g * PF + u >= nst) break;  // uniform
            const double a = AsT[4 * (g * PF + u) + kq][cl];
#pragma unroll
            for (int t = 0; t < NTW; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, (double)bq[u][t], acc[t], 0, 0, 0);
        }
    };
    load(0, b0);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) load(g + 1, b1);
        compute(g, b0);
        if (g + 1 >= ng) break;
        if (g + 2 < ng) load(g + 2, b0);
        compute(g + 1, b1);
    }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        if (col[t] >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = r0 + kq + 4 * i;
            if (row >= M) continue;
            double out = alpha * acc[t][i];
            if (beta != 0.0) out += beta * (double)Cin[(size_t)row * ldcin + col[t]];
            // a column flagged dependent is replaced by counter-based draws
            if (flags && flags[col[t]])
                out = uniform_pm1(seed, (sid << 40) + (uint64_t)row * 4096ULL + (uint64_t)col[t]);
            C[(size_t)row * ldc + col[t]] = (TC)out;
        }
    }
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void gemm_tn_lk_kernel(int M, int N, int K, int kchunk,
                                                         const TA* __restrict__ A, int lda,
                                                         const TB* __restrict__ B, int ldb,
                                                         double* __restrict__ partial)
{
    __shared__ double As[TN_BK][64 + 4];
    __shared__ double Bs[TN_BK][64 + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int kq = lane >> 4, cl = lane & 15;
    d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    // 4 rows of 64 per pass of the 256 threads, coalesced along M / N; the
    // next stage is loaded into registers while the current one is used
    constexpr int NU = TN_BK / 4;
    TA ra[NU];  // storage types, widened when stored to LDS
    TB rb[NU];
    const int gm = m0 + lane, gn = n0 + lane;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int gk = k0 + 4 * u + wave;
            ra[u] = (gk < ke && gm < M) ? A[(size_t)gk * lda + gm] : TA(0);
            rb[u] = (gk < ke && gn < N) ? B[(size_t)gk * ldb + gn] : TB(0);
        }
    };
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += TN_BK) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            As[4 * u + wave][lane] = (double)ra[u];
            Bs[4 * u + wave][lane] = (double)rb[u];
        }
        __syncthreads();
        if (k0 + TN_BK < ke) fetch(k0 + TN_BK);
#pragma unroll
        for (int kk = 0; kk < TN_BK / 4; ++kk) {
            const double a = As[4 * kk + kq][16 * wave + cl];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double bv = Bs[4 * kk + kq][16 * t + cl];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double* pz = partial + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = n0 + 16 * t + cl;
        if (c >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = m0 + 16 * wave + kq + 4 * i;
            if (r < M) pz[(size_t)r * N + c] = acc[t][i];
        }
    }
}

struct TnPlan {
    int gx, gy, splits, kchunk;
};

// about TN_TARGET_WG workgroups, chunks of at least one LDS stage, partials below
// min(4M, cap) doubles
TnPlan make_tn_plan(int M, int N, int K, size_t cap = (size_t)4 << 20)
{
    TnPlan p;
    p.gx = (M + 63) / 64;
    p.gy = (N + 63) / 64;
    const long blocks = (long)p.gx * p.gy;
    long s = (TN_TARGET_WG + blocks - 1) / blocks;
    const long smax_k = (K + TN_BK - 1) / TN_BK;
    if (s > smax_k) s = smax_k;
    const long smax_mem = (long)(std::min(cap, (size_t)4 << 20) / ((size_t)M * N));
    if (s > smax_mem) s = smax_mem;
    if (s < 1) s = 1;
    int kchunk = (int)((K + s - 1) / s);
    kchunk = ((kchunk + TN_BK - 1) / TN_BK) * TN_BK;
    p.kchunk = kchunk;
    p.splits = (K + kchunk - 1) / kchunk;  // <= s
    return p;
}

bool use_nn_sk(bool trans_a, int N, int K) { return !trans_a && K <= SK_MAXK && N <= 512; }
bool use_tn_lk(bool trans_a, int M, int N, int K)
{
    return trans_a && M <= TN_MAXMN && N <= TN_MAXMN && K >= 4 * TN_BK;
}

template <typename TA, typename TB, typename TC>
void launch_nn_sk(int M, int N, int K, double alpha, const TA* A, int lda, const TB* B, int ldb,
                  double beta, const TC* Cin, int ldcin, TC* C, int ldc, hipStream_t s,
                  const int* flags = nullptr, uint64_t seed = 0, uint64_t sid = 0)
{
    // a workgroup per 16-row strip and group of 4 NTW column tiles; for a
    // short C the column tiles are spread over more workgroups (one per wave)
    const int ntiles = (N + 15) / 16, strips = (M + 15) / 16;
    int ntw = (ntiles + 3) / 4, gy = 1;
    if (strips < 192 && ntw > 1) {
        ntw = 1;
        gy = (ntiles + 3) / 4;
    }
    dim3 grid(strips, gy), block(256);
#define BLWS_NNSK_CASE(V)                                                                       \
    case V:                                                                                     \
        hipLaunchKernelGGL((gemm_nn_sk_kernel<TA, TB, TC, V>), grid, block, 0, s, M, N, K, alpha, \
                           A, lda, B, ldb, beta, Cin, ldcin, C, ldc, flags, seed, sid);         \
        break;
    switch (ntw) {
        BLWS_NNSK_CASE(1)
        BLWS_NNSK_CASE(2)
        BLWS_NNSK_CASE(3)
        BLWS_NNSK_CASE(4)
        BLWS_NNSK_CASE(5)
        BLWS_NNSK_CASE(6)
        BLWS_NNSK_CASE(7)
        default:
            BLWS_NNSK_CASE(8)
    }
#undef BLWS_NNSK_CASE
}

}  // namespace

size_t gemm_partial_elems(int M, int N, int K)
{
    Plan p = make_plan(M, N, K);
    size_t e = p.splits > 1 ? (size_t)p.splits * M * N : 0;
    if (use_tn_lk(true, M, N, K)) {
        const TnPlan q = make_tn_plan(M, N, K);
        const size_t et = (size_t)q.splits * M * N;
        if (et > e) e = et;
    }
    return e;
}

bool wproduct_groupable(const WProduct& w)
{
    if (w.prec != 0 || w.M <= 0 || w.N <= 0 || w.K <= 0) return false;
    if (use_nn_sk(w.trans, w.N, w.K)) return false;
    if (use_tn_lk(w.trans, w.M, w.N, w.K) && w.partial && w.partial_elems >= (size_t)w.M * w.N)
        return false;
    const Plan p = make_plan(w.M, w.N, w.K);
    return p.splits == 1 || (w.partial && w.partial_elems >= (size_t)p.splits * w.M * w.N);
}

void gemm_f64_grouped(const WProduct* ps, int n, hipStream_t s)
{
    BLWS_REQUIRE(n >= 1 && n <= GROUP_MAX, BLWS_EINVAL, "gemm_f64_grouped: bad problem count");
    GroupF64 g{};
    GroupRedF64 r{};
    g.n = n;
    int blocks = 0, rblocks = 0, nr = 0;
    for (int q = 0; q < n; ++q) {
        const WProduct& w = ps[q];
        BLWS_REQUIRE(wproduct_groupable(w), BLWS_EINVAL, "gemm_f64_grouped: problem not groupable");
        const Plan p = make_plan(w.M, w.N, w.K);
        GroupF64::Prob& P = g.p[q];
        P.M = w.M;
        P.N = w.N;
        P.K = w.K;
        P.kchunk = p.kchunk;
        P.gx = p.gx;
        P.gy = p.gy;
        P.nt = p.nt;
        P.trans = w.trans ? 1 : 0;
        P.lda = w.lda;
        P.ldb = w.ldb;
        P.ldc = w.ldc;
        P.splits = p.splits;
        P.A = (const double*)w.A;
        P.B = (const double*)w.B;
        P.C = (double*)w.C;
        P.partial = (double*)w.partial;
        g.start[q] = blocks;
        blocks += p.gx * p.gy * p.splits;
        if (p.splits > 1) {
            const size_t total = (size_t)w.M * w.N;
            int nb = (int)((total + 255) / 256);
            if (nb > 2048) nb = 2048;
            r.p[nr] = GroupRedF64::Prob{w.M, w.N, p.splits, w.ldc, (const double*)w.partial,
                                        (double*)w.C};
            r.start[nr] = rblocks;
            rblocks += nb;
            ++nr;
        }
    }
    g.start[n] = blocks;
    hipLaunchKernelGGL(gemm_f64_grouped_kernel, dim3(blocks), dim3(NTHREADS), 0, s, g);
    if (nr > 0) {
        r.n = nr;
        r.start[nr] = rblocks;
        hipLaunchKernelGGL(splitk_reduce_grouped_kernel, dim3(rblocks), dim3(256), 0, s, r);
    }
}

template <typename TA, typename TB, typename TC>
void gemm(Timer* tm, const char* family, bool trans_a, int M, int N, int K, double alpha,
          const TA* A, int lda, const TB* B, int ldb, double beta, const TC* Cin, int ldcin,
          TC* C, int ldc, double* partial, size_t partial_elems, hipStream_t s)
{
    if (M <= 0 || N <= 0) return;
    if (K <= 0) {
        // C = beta * Cin: a split-K reduce over zero partials
        hipLaunchKernelGGL((splitk_reduce_kernel<TC>), dim3(256), dim3(256), 0, s, M, N, 0, 0.0,
                           (const double*)nullptr, beta, Cin, ldcin, C, ldc);
        return;
    }
    if (use_nn_sk(trans_a, N, K)) {
        TimedLaunch tl(tm, family, s, 2.0 * M * N * (double)K,
                       8.0 * ((double)M * K + (double)K * N + (double)M * N));
        launch_nn_sk<TA, TB, TC>(M, N, K, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc, s);
        return;
    }
    if (use_tn_lk(trans_a, M, N, K) && partial && partial_elems >= (size_t)M * N) {
        const TnPlan q = make_tn_plan(M, N, K, partial_elems);
        TimedLaunch tl(tm, family, s, 2.0 * M * N * (double)K,
                       8.0 * ((double)M * K + (double)K * N + (double)M * N));
        hipLaunchKernelGGL((gemm_tn_lk_kernel<TA, TB>), dim3(q.gx, q.gy, q.splits), dim3(256), 0,
                           s, M, N, K, q.kchunk, A, lda, B, ldb, partial);
        splitk_reduce<TC>(M, N, q.splits, alpha, partial, beta, Cin, ldcin, C, ldc, s);
        return;
    }
    Plan p = make_plan(M, N, K);
    const bool split = p.splits > 1;
    BLWS_REQUIRE(!split || (partial && partial_elems >= (size_t)p.splits * M * N), BLWS_ENOMEM,
                 "gemm: split-K scratch too small");
    TimedLaunch tl(tm, family, s, 2.0 * M * N * (double)K,
                   8.0 * ((double)M * K + (double)K * N + (double)M * N));
    if (trans_a)
        launch_nt<TA, TB, TC, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc,
                                     split ? partial : nullptr, s);
    else
        launch_nt<TA, TB, TC, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc,
                                      split ? partial : nullptr, s);
    if (split) splitk_reduce<TC>(M, N, p.splits, alpha, partial, beta, Cin, ldcin, C, ldc, s);
}

template <typename T>
void gemm_apply_flagged(Timer* tm, int M, int N, const T* X, int ldx, const double* R, int ldr,
                        T* C, int ldc, const int* flags, uint64_t seed, uint64_t sid,
                        hipStream_t s)
{
    if (M <= 0 || N <= 0) return;
    BLWS_REQUIRE(use_nn_sk(false, N, N), BLWS_EUNSUPPORTED, "gemm_apply_flagged: width");
    TimedLaunch tl(tm, "gemm_ts", s, 2.0 * M * N * (double)N,
                   8.0 * ((double)M * N + (double)N * N + (double)M * N));
    launch_nn_sk<T, double, T>(M, N, N, 1.0, X, ldx, R, ldr, 0.0, (const T*)nullptr, 0, C, ldc, s,
                               flags, seed, sid);
}
template void gemm_apply_flagged<double>(Timer*, int, int, const double*, int, const double*, int,
                                         double*, int, const int*, uint64_t, uint64_t, hipStream_t);
template void gemm_apply_flagged<float>(Timer*, int, int, const float*, int, const double*, int,
                                        float*, int, const int*, uint64_t, uint64_t, hipStream_t);

#define BLWS_GEMM_INST(TA, TB, TC)                                                           \
    template void gemm<TA, TB, TC>(Timer*, const char*, bool, int, int, int, double, const TA*, \
                                   int, const TB*, int, double, const TC*, int, TC*, int,     \
                                   double*, size_t, hipStream_t);
BLWS_GEMM_INST(double, double, double)
BLWS_GEMM_INST(float, float, float)
BLWS_GEMM_INST(float, float, double)
BLWS_GEMM_INST(float, double, float)
#undef BLWS_GEMM_INST

}  // namespace blws
