// Block products W X and W^T X in FP32 and BF16 on CDNA4 matrix cores.
//
// The products of the Lanczos block with W (Algorithm 2) are the only work of
// the BLWS step that touches the big matrix. In the FP32 and BF16 precision
// modes they run on v_mfma_f32_16x16x4f32 (FP32 inputs) or
// v_mfma_f32_16x16x32_bf16 (W kept as a BF16 copy, the block rounded to BF16
// on the way into LDS), accumulating in FP32. Tiling as the FP64 kernel: a
// workgroup owns 64 rows of C (four wavefronts x 16) and 16 * NT columns;
// long K is split across workgroups and the FP32 partials are summed in a
// fixed order (in FP64) by a second kernel.
#include "blws_common.h"

namespace blws {
namespace {

constexpr int LBM = 64;
constexpr int LNTHREADS = 256;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16 with round-to-nearest-even (finite inputs; NaN stays NaN).
__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (unsigned short)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <typename T>
__device__ __forceinline__ unsigned short to_bf(T v);
template <>
__device__ __forceinline__ unsigned short to_bf<float>(float v) { return f2bf(v); }
template <>
__device__ __forceinline__ unsigned short to_bf<unsigned short>(unsigned short v) { return v; }

template <typename T>
__device__ __forceinline__ float to_f(T v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }

// FP32 mode: A, B float; LDS k-major; BK = 32 (8 MFMA steps of k = 4). One
// 64 x 16 nt block (nt <= NT, uniform) of C over the K range of split bz: the
// body of the single-problem kernel and of the grouped one (As: 32 x 65,
// Bs: 32 x ldbs floats of LDS). An element's products are accumulated in the
// same order whatever nt is.
template <bool TRANS, int NT>
__device__ __forceinline__ void gemm_f32_block(float* As, float* Bs, int ldbs, int bx, int by,
                                               int bz, int nt, int M, int N, int K, int kchunk,
                                               const float* __restrict__ A, int lda,
                                               const float* __restrict__ B, int ldb,
                                               float* __restrict__ C, int ldc,
                                               float* __restrict__ partial)
{
    constexpr int BK = 32, LDA_S = LBM + 1;
    const int BN = 16 * nt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = bx * LBM, c0 = by * BN;
    const int kb = bz * kchunk;
    const int ke = min(K, kb + kchunk);
    f4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};

    // the next stage's tiles load into registers while the current one is used
    constexpr int NB = (BK * 16 * NT + LNTHREADS - 1) / LNTHREADS;
    float ra[8], rb[NB];
    auto fetch = [&](int k0) {
        if (!TRANS) {
            const int row = tid >> 2, kq = (tid & 3) * 8;
            const int gr = r0 + row;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gk = k0 + kq + u;
                ra[u] = (gr < M && gk < ke) ? A[(size_t)gr * lda + gk] : 0.f;
            }
        } else {
            const int kr = tid >> 3, rq = (tid & 7) * 8;
            const int gk = k0 + kr;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gr = r0 + rq + u;
                ra[u] = (gr < M && gk < ke) ? A[(size_t)gk * lda + gr] : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + LNTHREADS * u;
            const int kr = e / BN, cc = e - kr * BN;
            const int gk = k0 + kr, gc = c0 + cc;
            rb[u] = (e < BK * BN && gk < ke && gc < N) ? B[(size_t)gk * ldb + gc] : 0.f;
        }
    };
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        if (!TRANS) {
            const int row = tid >> 2, kq = (tid & 3) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) As[(kq + u) * LDA_S + row] = ra[u];
        } else {
            const int kr = tid >> 3, rq = (tid & 7) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) As[kr * LDA_S + rq + u] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + LNTHREADS * u;
            const int kr = e / BN, cc = e - kr * BN;
            if (e < BK * BN) Bs[kr * ldbs + cc] = rb[u];
        }
        __syncthreads();
        if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const float a = As[(kk * 4 + (lane >> 4)) * LDA_S + wave * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if (j >= nt) break;  // uniform
                const float bv = Bs[(kk * 4 + (lane >> 4)) * ldbs + j * 16 + (lane & 15)];
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // FP32 16x16 tile (measured on gfx950): register i of lane l holds row
    // 4 (l / 16) + i, column l % 16.
    const int rbase = r0 + wave * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        if (j >= nt) break;
        const int col = c0 + j * 16 + (lane & 15);
        if (col >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rbase + i;
            if (row >= M) continue;
            if (partial)
                partial[((size_t)bz * M + row) * N + col] = acc[j][i];
            else
                C[(size_t)row * ldc + col] = acc[j][i];
        }
    }
}

template <bool TRANS, int NT>
__global__ __launch_bounds__(LNTHREADS) void gemm_f32_kernel(int M, int N, int K, int kchunk,
                                                             const float* __restrict__ A, int lda,
                                                             const float* __restrict__ B, int ldb,
                                                             float* __restrict__ C, int ldc,
                                                             float* __restrict__ partial)
{
    __shared__ float As[32 * (LBM + 1)];
    __shared__ float Bs[32 * (16 * NT + 1)];
    gemm_f32_block<TRANS, NT>(As, Bs, 16 * NT + 1, blockIdx.x, blockIdx.y, blockIdx.z, NT, M, N, K,
                              kchunk, A, lda, B, ldb, C, ldc, partial);
}

// BF16 mode: A is BF16 bits (the W copy), B float rounded to BF16 into LDS.
// LDS row-major in k (8 consecutive k per lane fragment); BK = 64 (2 MFMA
// steps of k = 32). As: 64 x 72, Bs: 16 nt x 72 shorts of LDS.
//
// X3 (split-precision BF16 x 3): A = A_hi + A_lo (two BF16 copies) and each
// B element b = b_hi + b_lo with b_hi = bf16(b), b_lo = bf16(b - b_hi), split
// on the way into LDS (Al, Bl beside As, Bs); each k-step accumulates
// A_lo B_hi, A_hi B_lo, then A_hi B_hi in FP32 (the A_lo B_lo term, below
// 2^-18 of |A||B|, is dropped): about 16 significant bits per product in
// place of 8, at three BF16 MFMAs per step.
constexpr int BF_BK = 64, BF_LDK = BF_BK + 8;
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <bool TRANS, int NT, bool X3 = false>
__device__ __forceinline__ void gemm_bf16_block(unsigned short* As, unsigned short* Bs,
                                                unsigned short* Al, unsigned short* Bl, int bx,
                                                int by, int bz, int nt, int M, int N, int K,
                                                int kchunk, const unsigned short* __restrict__ A,
                                                const unsigned short* __restrict__ Alo, int lda,
                                                const float* __restrict__ B, int ldb,
                                                float* __restrict__ C, int ldc,
                                                float* __restrict__ partial)
{
    constexpr int BK = BF_BK, LDK = BF_LDK;
    const int BN = 16 * nt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = bx * LBM, c0 = by * BN;
    const int kb = bz * kchunk;
    const int ke = min(K, kb + kchunk);
    f4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};

    // the next stage's tiles load into registers while the current one is used
    constexpr int NB = (BK * 16 * NT + LNTHREADS - 1) / LNTHREADS;
    unsigned short ra[16], rl[X3 ? 16 : 1];
    float rb[NB];  // rounded to BF16 when stored to LDS, not as it arrives
    auto fetch = [&](int k0) {
        if (!TRANS) {
            const int row = tid >> 2, kq = (tid & 3) * 16;
            const int gr = r0 + row;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int gk = k0 + kq + u;
                const bool in = gr < M && gk < ke;
                ra[u] = in ? A[(size_t)gr * lda + gk] : (unsigned short)0;
                if constexpr (X3) rl[u] = in ? Alo[(size_t)gr * lda + gk] : (unsigned short)0;
            }
        } else {
            const int kr = tid >> 2, rq = (tid & 3) * 16;
            const int gk = k0 + kr;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int gr = r0 + rq + u;
                const bool in = gr < M && gk < ke;
                ra[u] = in ? A[(size_t)gk * lda + gr] : (unsigned short)0;
                if constexpr (X3) rl[u] = in ? Alo[(size_t)gk * lda + gr] : (unsigned short)0;
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + LNTHREADS * u;
            const int kr = e / BN, cc = e - kr * BN;
            const int gk = k0 + kr, gc = c0 + cc;
            rb[u] = (e < BK * BN && gk < ke && gc < N) ? B[(size_t)gk * ldb + gc] : 0.f;
        }
    };
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        if (!TRANS) {
            const int row = tid >> 2, kq = (tid & 3) * 16;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                As[row * LDK + kq + u] = ra[u];
                if constexpr (X3) Al[row * LDK + kq + u] = rl[u];
            }
        } else {
            const int kr = tid >> 2, rq = (tid & 3) * 16;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                As[(rq + u) * LDK + kr] = ra[u];
                if constexpr (X3) Al[(rq + u) * LDK + kr] = rl[u];
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + LNTHREADS * u;
            const int kr = e / BN, cc = e - kr * BN;
            if (e < BK * BN) {
                const unsigned short hi = f2bf(rb[u]);
                Bs[cc * LDK + kr] = hi;
                if constexpr (X3) Bl[cc * LDK + kr] = f2bf(rb[u] - bf2f(hi));
            }
        }
        __syncthreads();
        if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 32; ++kk) {
            const int ao = (wave * 16 + (lane & 15)) * LDK + kk * 32 + 8 * (lane >> 4);
            const s8 a = *(const s8*)&As[ao];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if (j >= nt) break;  // uniform
                const int bo = (j * 16 + (lane & 15)) * LDK + kk * 32 + 8 * (lane >> 4);
                const s8 bv = *(const s8*)&Bs[bo];
                if constexpr (X3) {
                    const s8 al = *(const s8*)&Al[ao];
                    const s8 bl = *(const s8*)&Bl[bo];
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bv, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[j], 0, 0, 0);
                }
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int rbase = r0 + wave * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        if (j >= nt) break;
        const int col = c0 + j * 16 + (lane & 15);
        if (col >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rbase + i;
            if (row >= M) continue;
            if (partial)
                partial[((size_t)bz * M + row) * N + col] = acc[j][i];
            else
                C[(size_t)row * ldc + col] = acc[j][i];
        }
    }
}

template <bool TRANS, int NT>
__global__ __launch_bounds__(LNTHREADS) void gemm_bf16_kernel(
    int M, int N, int K, int kchunk, const unsigned short* __restrict__ A, int lda,
    const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
    float* __restrict__ partial)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[LBM * BF_LDK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[16 * NT * BF_LDK];
    gemm_bf16_block<TRANS, NT>(As, Bs, nullptr, nullptr, blockIdx.x, blockIdx.y, blockIdx.z, NT,
                               M, N, K, kchunk, A, nullptr, lda, B, ldb, C, ldc, partial);
}

template <bool TRANS, int NT>
__global__ __launch_bounds__(LNTHREADS) void gemm_bf16x3_kernel(
    int M, int N, int K, int kchunk, const unsigned short* __restrict__ A,
    const unsigned short* __restrict__ Alo, int lda, const float* __restrict__ B, int ldb,
    float* __restrict__ C, int ldc, float* __restrict__ partial)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[LBM * BF_LDK];
    __shared__ __attribute__((aligned(16))) unsigned short Al[LBM * BF_LDK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[16 * NT * BF_LDK];
    __shared__ __attribute__((aligned(16))) unsigned short Bl[16 * NT * BF_LDK];
    gemm_bf16_block<TRANS, NT, true>(As, Bs, Al, Bl, blockIdx.x, blockIdx.y, blockIdx.z, NT, M, N,
                                     K, kchunk, A, Alo, lda, B, ldb, C, ldc, partial);
}

// FP32 partial sums of split s, added in split order in FP64
__device__ __forceinline__ double sum_splits_f32(const float* partial, size_t total, size_t e, int S)
{
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += (double)partial[(size_t)s * total + e];
    return acc;
}

__global__ void reduce_f32_kernel(int M, int N, int S, const float* partial, float* C, int ldc)
{
    const size_t total = (size_t)M * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const double acc = sum_splits_f32(partial, total, e, S);
        const int row = (int)(e / N), col = (int)(e - (size_t)row * N);
        C[(size_t)row * ldc + col] = (float)acc;
    }
}

// Grouped W-products (FP32 or BF16, one precision per launch): problem q owns
// blocks start[q] .. start[q + 1] - 1, with the block grid and K split it has
// alone, so its results are the same bits.
constexpr int GROUP_MAX = GEMM_GROUP_MAX;
struct GroupLp {
    int n;
    int start[GROUP_MAX + 1];
    struct Prob {
        int M, N, K, kchunk, gx, gy, nt, trans, lda, ldb, ldc, splits;
        const void* A;
        const float* B;
        float *C, *partial;
    } p[GROUP_MAX];
};

__device__ __forceinline__ int group_find(const int* start, int n, int blk)
{
    int q = 0;
    while (q + 1 < n && blk >= start[q + 1]) ++q;
    return q;
}

__device__ __forceinline__ void group_block(const GroupLp& g, int& q, int& bx, int& by, int& bz)
{
    q = group_find(g.start, g.n, blockIdx.x);
    const GroupLp::Prob& P = g.p[q];
    const int l = blockIdx.x - g.start[q], per = P.gx * P.gy;
    bz = l / per;
    const int rem = l - bz * per;
    by = rem / P.gx;
    bx = rem - by * P.gx;
}

__global__ __launch_bounds__(LNTHREADS) void gemm_f32_grouped_kernel(GroupLp g)
{
    __shared__ float As[32 * (LBM + 1)];
    __shared__ float Bs[32 * (16 * 8 + 1)];
    int q, bx, by, bz;
    group_block(g, q, bx, by, bz);
    const GroupLp::Prob& P = g.p[q];
    float* part = P.splits > 1 ? P.partial : nullptr;
    if (P.trans)
        gemm_f32_block<true, 8>(As, Bs, 16 * 8 + 1, bx, by, bz, P.nt, P.M, P.N, P.K, P.kchunk,
                                (const float*)P.A, P.lda, P.B, P.ldb, P.C, P.ldc, part);
    else
        gemm_f32_block<false, 8>(As, Bs, 16 * 8 + 1, bx, by, bz, P.nt, P.M, P.N, P.K, P.kchunk,
                                 (const float*)P.A, P.lda, P.B, P.ldb, P.C, P.ldc, part);
}

__global__ __launch_bounds__(LNTHREADS) void gemm_bf16_grouped_kernel(GroupLp g)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[LBM * BF_LDK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[16 * 8 * BF_LDK];
    int q, bx, by, bz;
    group_block(g, q, bx, by, bz);
    const GroupLp::Prob& P = g.p[q];
    float* part = P.splits > 1 ? P.partial : nullptr;
    if (P.trans)
        gemm_bf16_block<true, 8>(As, Bs, nullptr, nullptr, bx, by, bz, P.nt, P.M, P.N, P.K,
                                 P.kchunk, (const unsigned short*)P.A, nullptr, P.lda, P.B, P.ldb,
                                 P.C, P.ldc, part);
    else
        gemm_bf16_block<false, 8>(As, Bs, nullptr, nullptr, bx, by, bz, P.nt, P.M, P.N, P.K,
                                  P.kchunk, (const unsigned short*)P.A, nullptr, P.lda, P.B, P.ldb,
                                  P.C, P.ldc, part);
}

struct GroupRedLp {
    int n;
    int start[GROUP_MAX + 1];
    struct Prob {
        int M, N, S, ldc;
        const float* partial;
        float* C;
    } p[GROUP_MAX];
};

__global__ void reduce_f32_grouped_kernel(GroupRedLp g)
{
    const int q = group_find(g.start, g.n, blockIdx.x);
    const GroupRedLp::Prob& P = g.p[q];
    const int nb = g.start[q + 1] - g.start[q], lb = blockIdx.x - g.start[q];
    const size_t total = (size_t)P.M * P.N;
    for (size_t e = lb * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)nb * blockDim.x) {
        const double acc = sum_splits_f32(P.partial, total, e, P.S);
        const int row = (int)(e / P.N), col = (int)(e - (size_t)row * P.N);
        P.C[(size_t)row * P.ldc + col] = (float)acc;
    }
}

// Hi[r][c] = bf16(X[r][c]), Lo[r][c] = bf16(X[r][c] - Hi[r][c]) (rows x cols, the
// same ld for all three)
__global__ void split_bf16x2_kernel(int rows, int cols, const float* __restrict__ X, int ld,
                                    unsigned short* __restrict__ Hi,
                                    unsigned short* __restrict__ Lo)
{
    const long long total = (long long)rows * cols;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / cols), c = (int)(e - (long long)r * cols);
        const size_t i = (size_t)r * ld + c;
        const float x = X[i];
        const unsigned short h = f2bf(x);
        Hi[i] = h;
        Lo[i] = f2bf(x - bf2f(h));
    }
}

__global__ void to_bf16_kernel(long long count, const float* __restrict__ X,
                               unsigned short* __restrict__ Y)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        Y[e] = f2bf(X[e]);
}

struct PlanLp {
    int nt, gy, gx, splits, kchunk;
};

PlanLp make_plan_lp(int M, int N, int K, int BK)
{
    PlanLp p;
    p.nt = N >= 128 ? 8 : (N + 15) / 16;
    if (p.nt < 1) p.nt = 1;
    p.gy = (N + 16 * p.nt - 1) / (16 * p.nt);
    p.gx = (M + LBM - 1) / LBM;
    const long tiles = (long)p.gx * p.gy;
    const long target = plan_target(BK == 64 ? 2 : 1, M, N, K, 512);
    long s = (target + tiles - 1) / tiles;
    const long smax_k = (K + 4 * BK - 1) / (4 * BK);
    if (s > smax_k) s = smax_k;
    const long smax_mem = (8L << 20) / ((long)M * N > 0 ? (long)M * N : 1);
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

}  // namespace

size_t gemm_lp_partial_elems(int M, int N, int K)
{
    const PlanLp p1 = make_plan_lp(M, N, K, 32), p2 = make_plan_lp(M, N, K, 64);
    const int s = p1.splits > p2.splits ? p1.splits : p2.splits;
    return s > 1 ? (size_t)s * M * N : 0;
}

void gemm_lp(Timer* tm, const char* family, bool bf16, bool trans_a, int M, int N, int K,
             const void* A, int lda, const float* B, int ldb, float* C, int ldc, float* partial,
             size_t partial_elems, hipStream_t s, const unsigned short* A_lo)
{
    if (M <= 0 || N <= 0) return;
    BLWS_REQUIRE(K > 0, BLWS_EINVAL, "gemm_lp: K must be positive");
    BLWS_REQUIRE(!A_lo || bf16, BLWS_EINVAL, "gemm_lp: a low BF16 half needs the BF16 mode");
    const PlanLp p = make_plan_lp(M, N, K, bf16 ? 64 : 32);
    const bool split = p.splits > 1;
    BLWS_REQUIRE(!split || (partial && partial_elems >= (size_t)p.splits * M * N), BLWS_ENOMEM,
                 "gemm_lp: split-K scratch too small");
    TimedLaunch tl(tm, family, s, (A_lo ? 6.0 : 2.0) * M * N * (double)K,
                   (A_lo ? 4.0 : bf16 ? 2.0 : 4.0) * (double)M * K +
                       4.0 * ((double)K * N + (double)M * N));
    dim3 grid(p.gx, p.gy, p.splits), block(LNTHREADS);
    float* part = split ? partial : nullptr;
#define BLWS_LP_CASE(NTV)                                                                      \
    case NTV:                                                                                  \
        if (A_lo) {                                                                            \
            if (trans_a)                                                                       \
                hipLaunchKernelGGL((gemm_bf16x3_kernel<true, NTV>), grid, block, 0, s, M, N,   \
                                   K, p.kchunk, (const unsigned short*)A, A_lo, lda, B, ldb, C, \
                                   ldc, part);                                                 \
            else                                                                               \
                hipLaunchKernelGGL((gemm_bf16x3_kernel<false, NTV>), grid, block, 0, s, M, N,  \
                                   K, p.kchunk, (const unsigned short*)A, A_lo, lda, B, ldb, C, \
                                   ldc, part);                                                 \
        } else if (bf16) {                                                                     \
            if (trans_a)                                                                       \
                hipLaunchKernelGGL((gemm_bf16_kernel<true, NTV>), grid, block, 0, s, M, N, K,  \
                                   p.kchunk, (const unsigned short*)A, lda, B, ldb, C, ldc,     \
                                   part);                                                      \
            else                                                                               \
                hipLaunchKernelGGL((gemm_bf16_kernel<false, NTV>), grid, block, 0, s, M, N, K, \
                                   p.kchunk, (const unsigned short*)A, lda, B, ldb, C, ldc,     \
                                   part);                                                      \
        } else {                                                                               \
            if (trans_a)                                                                       \
                hipLaunchKernelGGL((gemm_f32_kernel<true, NTV>), grid, block, 0, s, M, N, K,   \
                                   p.kchunk, (const float*)A, lda, B, ldb, C, ldc, part);       \
            else                                                                               \
                hipLaunchKernelGGL((gemm_f32_kernel<false, NTV>), grid, block, 0, s, M, N, K,  \
                                   p.kchunk, (const float*)A, lda, B, ldb, C, ldc, part);       \
        }                                                                                      \
        break;
    switch (p.nt) {
        BLWS_LP_CASE(1)
        BLWS_LP_CASE(2)
        BLWS_LP_CASE(3)
        BLWS_LP_CASE(4)
        BLWS_LP_CASE(5)
        BLWS_LP_CASE(6)
        BLWS_LP_CASE(7)
        default:
            BLWS_LP_CASE(8)
    }
#undef BLWS_LP_CASE
    if (split) {
        const size_t total = (size_t)M * N;
        int blocks = (int)((total + 255) / 256);
        if (blocks > 2048) blocks = 2048;
        hipLaunchKernelGGL(reduce_f32_kernel, dim3(blocks), dim3(256), 0, s, M, N, p.splits,
                           partial, C, ldc);
    }
}

bool wproduct_lp_groupable(const WProduct& w)
{
    if ((w.prec != 1 && w.prec != 2) || w.M <= 0 || w.N <= 0 || w.K <= 0) return false;
    const PlanLp p = make_plan_lp(w.M, w.N, w.K, w.prec == 2 ? 64 : 32);
    return p.splits == 1 || (w.partial && w.partial_elems >= (size_t)p.splits * w.M * w.N);
}

void gemm_lp_grouped(const WProduct* ps, int n, hipStream_t s)
{
    BLWS_REQUIRE(n >= 1 && n <= GEMM_GROUP_MAX, BLWS_EINVAL, "gemm_lp_grouped: bad problem count");
    const int prec = ps[0].prec;
    GroupLp g{};
    GroupRedLp r{};
    g.n = n;
    int blocks = 0, rblocks = 0, nr = 0;
    for (int q = 0; q < n; ++q) {
        const WProduct& w = ps[q];
        BLWS_REQUIRE(w.prec == prec && wproduct_lp_groupable(w), BLWS_EINVAL,
                     "gemm_lp_grouped: problem not groupable");
        const PlanLp p = make_plan_lp(w.M, w.N, w.K, prec == 2 ? 64 : 32);
        GroupLp::Prob& P = g.p[q];
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
        P.A = w.A;
        P.B = (const float*)w.B;
        P.C = (float*)w.C;
        P.partial = (float*)w.partial;
        g.start[q] = blocks;
        blocks += p.gx * p.gy * p.splits;
        if (p.splits > 1) {
            const size_t total = (size_t)w.M * w.N;
            int nb = (int)((total + 255) / 256);
            if (nb > 2048) nb = 2048;
            r.p[nr] = GroupRedLp::Prob{w.M, w.N, p.splits, w.ldc, (const float*)w.partial,
                                       (float*)w.C};
            r.start[nr] = rblocks;
            rblocks += nb;
            ++nr;
        }
    }
    g.start[n] = blocks;
    if (prec == 2)
        hipLaunchKernelGGL(gemm_bf16_grouped_kernel, dim3(blocks), dim3(LNTHREADS), 0, s, g);
    else
        hipLaunchKernelGGL(gemm_f32_grouped_kernel, dim3(blocks), dim3(LNTHREADS), 0, s, g);
    if (nr > 0) {
        r.n = nr;
        r.start[nr] = rblocks;
        hipLaunchKernelGGL(reduce_f32_grouped_kernel, dim3(rblocks), dim3(256), 0, s, r);
    }
}

void split_bf16x2(int rows, int cols, const float* X, int ld, unsigned short* Hi,
                  unsigned short* Lo, hipStream_t s)
{
    const long long total = (long long)rows * cols;
    if (total <= 0) return;
    long long blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(split_bf16x2_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rows, cols, X,
                       ld, Hi, Lo);
    HIP_TRY(hipGetLastError());
}

void to_bf16(long long count, const float* X, unsigned short* Y, hipStream_t s)
{
    if (count <= 0) return;
    long long blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, X, Y);
}

}  // namespace blws
