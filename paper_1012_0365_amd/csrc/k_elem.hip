// Passes over the dense m x n state of the RPCA solver.
//
// The fused epilogue rebuilds each 64 x 64 tile of A = U_r diag(S_r - eps) V_r^T
// (Eq. (4) on the Ritz pairs above the threshold) with MFMA tiles of depth r,
// and applies the inexact-ALM update to the same tile while it is in registers:
// soft-thresholding of E, the multiplier and residual, and the next W. A is
// never written to memory during the solve. Reductions (residual norm, norms
// of D, nonzero count) are two-pass and summed in a fixed order.
#include "blws_common.h"

namespace blws {
namespace {

constexpr int TILE = 64;
constexpr int EBK = 16;

typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ double rd(const T* p)
{
    return (double)(*p);
}

// FP32 -> BF16 bits, round to nearest even (the BF16 copy of W).
__device__ __forceinline__ unsigned short bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (unsigned short)((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) tot += sh[w];
    }
    return tot;  // valid in thread 0
}

// MODE 0: ALM epilogue. MODE 1: reconstruction only (A_out).
template <typename T, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void svt_tile_kernel(
    int m, int n, int b, const T* __restrict__ U, int ldu, const T* __restrict__ V, int ldv,
    const double* __restrict__ S, double eps, double lam, double mu, double mu_next,
    const T* __restrict__ D, int ldd, T* __restrict__ Y, T* __restrict__ E, int lde,
    T* __restrict__ W, unsigned short* __restrict__ Wh, unsigned short* __restrict__ Wl,
    T* __restrict__ A_out, int lda, double* __restrict__ partials)
{
    __shared__ double Us[EBK][TILE + 1];
    __shared__ double Vs[EBK][TILE + 1];
    __shared__ double red[8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = blockIdx.x * TILE, r0 = blockIdx.y * TILE;

    // r = #{S_k > eps}: the Ritz values are sorted, so count in parallel.
    int cnt = 0;
    for (int k = tid; k < b; k += blockDim.x) cnt += S[k] > eps;
    __shared__ int rsh;
    if (tid == 0) rsh = 0;
    __syncthreads();
    if (cnt) atomicAdd(&rsh, cnt);
    __syncthreads();
    const int rank = rsh;

    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};

    // FP64 16x16 tile: register i of lane l holds row (l / 16) + 4 i, column l % 16
    const int rbase = r0 + wave * 16 + (lane >> 4);
    // 64 rows x EBK ranks of U (scaled by S_k - eps) and of V per chunk: thread
    // (rr, kk) holds rows rr + 16 q, q < 4, of rank kk, the next chunk loaded
    // into registers (clamped in range) while the current one is used
    static_assert(TILE * EBK == 4 * 256, "four staged values per thread and matrix");
    const int kk = tid % EBK, rr = tid / EBK;
    double ur[4], vr[4], sk = 0.0;
    auto fetch = [&](int k0) {
        const int k = min(k0 + kk, rank - 1);
        sk = S[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ur[q] = rd(U + (size_t)min(r0 + rr + 16 * q, m - 1) * ldu + k);
            vr[q] = rd(V + (size_t)min(c0 + rr + 16 * q, n - 1) * ldv + k);
        }
    };
    auto stage = [&](int ch) {
        const bool kin = ch * EBK + kk < rank;
        const double th = kin ? sk - eps : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rr + 16 * q;
            Us[kk][row] = (kin && r0 + row < m) ? ur[q] * th : 0.0;
            Vs[kk][row] = (kin && c0 + row < n) ? vr[q] : 0.0;
        }
    };
    auto products = [&]() {
#pragma unroll
        for (int k4 = 0; k4 < EBK / 4; ++k4) {
            const double a = Us[k4 * 4 + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double bv = Vs[k4 * 4 + (lane >> 4)][j * 16 + (lane & 15)];
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[j], 0, 0, 0);
            }
        }
    };
    const int nch = (rank + EBK - 1) / EBK;
    if (nch > 0) fetch(0);
    for (int ch = 0; ch + 1 < nch; ++ch) {
        stage(ch);
        __syncthreads();
        fetch((ch + 1) * EBK);
        products();
        __syncthreads();
    }
    if (nch > 0) {
        stage(nch - 1);
        __syncthreads();
        products();
    }
    double zz = 0.0;
    const double thr = lam / mu;
    // the lane's 16 elements in two halves of eight; each half's D and Y are
    // loaded together (from clamped in-range addresses) before any is used
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double dv[2][4], yv[2][4];
        if (MODE == 0) {
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = min(rbase + 4 * i, m - 1);
                    const int col = min(c0 + (2 * h + jj) * 16 + (lane & 15), n - 1);
                    dv[jj][i] = rd(D + (size_t)row * ldd + col);
                    yv[jj][i] = rd(Y + (size_t)row * n + col);
                }
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int j = 2 * h + jj;
            const int col = c0 + j * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = rbase + 4 * i;
                if (row >= m || col >= n) continue;
                const double a = acc[j][i];
                if (MODE == 1) {
                    A_out[(size_t)row * lda + col] = (T)a;
                    continue;
                }
                const double d = dv[jj][i];
                const size_t ye = (size_t)row * n + col;
                const double y = yv[jj][i];
                const double t = d - a + y / mu;
                const double e = t > thr ? t - thr : (t < -thr ? t + thr : 0.0);
                const double z = d - a - e;
                const double y2 = y + mu * z;
                E[(size_t)row * lde + col] = (T)e;
                Y[ye] = (T)y2;
                const T wn = (T)(d - e + y2 / mu_next);
                W[ye] = wn;
                if (Wh) {
                    const unsigned short h = bf16_rne((float)wn);
                    Wh[ye] = h;
                    // low half of the split-precision copy: W - W_hi in BF16
                    if (Wl) Wl[ye] = bf16_rne((float)wn - __uint_as_float((unsigned)h << 16));
                }
                if (A_out) A_out[(size_t)row * lda + col] = (T)a;
                zz += z * z;
            }
        }
    }
    if (MODE == 0) {
        const double tot = block_sum(zz, red);
        if (tid == 0) partials[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
    }
}

constexpr int RED_BLOCKS = 1024;

template <typename T>
__global__ __launch_bounds__(256) void norms_kernel(int m, int n, const T* X, int ldx,
                                                    double* part)
{
    __shared__ double sh[8];
    __shared__ double shm[8];
    double s2 = 0.0, mx = 0.0;
    const size_t total = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
        const double v = rd(X + (size_t)i * ldx + j);
        s2 += v * v;
        mx = fmax(mx, fabs(v));
    }
    for (int off = 32; off > 0; off >>= 1) {
        s2 += __shfl_xor(s2, off, 64);
        mx = fmax(mx, __shfl_xor(mx, off, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[wave] = s2;
        shm[wave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a += sh[w];
            b = fmax(b, shm[w]);
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void norms_final_kernel(int nb, const double* part, double* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nb; ++i) {
            a += part[2 * i];
            b = fmax(b, part[2 * i + 1]);
        }
        out[0] = a;
        out[1] = b;
    }
}

template <typename T>
__global__ void rpca_init_kernel(int m, int n, const T* D, int ldd, double J, double mu, T* Y,
                                 T* E, int lde, T* W)
{
    const size_t total = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
        const double d = rd(D + (size_t)i * ldd + j);
        const double y = d / J;
        Y[e] = (T)y;
        E[(size_t)i * lde + j] = (T)0.0;
        W[e] = (T)(d - 0.0 + (double)(T)y / mu);
    }
}

__global__ void sum_partials_kernel(int count, const double* p, double* out)
{
    // one wavefront sums in a fixed order: lane-strided partial sums, then a
    // fixed shuffle tree
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += 64) s += p[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[0] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void nnz_kernel(int m, int n, const T* X, int ldx,
                                                  long long* part)
{
    __shared__ long long sh[4];
    long long c = 0;
    const size_t total = (size_t)m * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
        c += X[(size_t)i * ldx + j] != (T)0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void nnz_final_kernel(int nb, const long long* part, long long* out)
{
    if (threadIdx.x == 0) {
        long long c = 0;
        for (int i = 0; i < nb; ++i) c += part[i];
        out[0] = c;
    }
}

}  // namespace

size_t norms_scratch_elems() { return 2 * RED_BLOCKS; }

template <typename T>
void norms(int m, int n, const T* X, int ldx, double* out, double* scratch, hipStream_t s)
{
    hipLaunchKernelGGL((norms_kernel<T>), dim3(RED_BLOCKS), dim3(256), 0, s, m, n, X, ldx,
                       scratch);
    hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(64), 0, s, RED_BLOCKS, scratch, out);
}

template <typename T>
void rpca_init(int m, int n, const T* D, int ldd, double J, double mu, T* Y, T* E, int lde,
               T* W, hipStream_t s)
{
    hipLaunchKernelGGL((rpca_init_kernel<T>), dim3(2048), dim3(256), 0, s, m, n, D, ldd, J, mu,
                       Y, E, lde, W);
}

size_t alm_partials(int m, int n)
{
    return (size_t)((n + TILE - 1) / TILE) * ((m + TILE - 1) / TILE);
}

template <typename T>
void alm_epilogue(Timer* tm, int m, int n, int b, const T* U, int ldu, const T* V, int ldv,
                  const double* S, double eps, double lam, double mu, double mu_next, const T* D,
                  int ldd, T* Y, T* E, int lde, T* W, unsigned short* Wh, T* A_out, int lda,
                  double* partials, hipStream_t s, unsigned short* Wl)
{
    dim3 grid((n + TILE - 1) / TILE, (m + TILE - 1) / TILE);
    // algorithmic traffic: read D, Y; write E, Y, W (A itself is never stored)
    TimedLaunch tl(tm, "alm_epilogue", s, 2.0 * m * (double)n * b,
                   5.0 * sizeof(T) * (double)m * n);
    hipLaunchKernelGGL((svt_tile_kernel<T, 0>), grid, dim3(256), 0, s, m, n, b, U, ldu, V, ldv, S,
                       eps, lam, mu, mu_next, D, ldd, Y, E, lde, W, Wh, Wl, A_out, lda,
                       partials);
}

template <typename T>
void svt_reconstruct(Timer* tm, int m, int n, int b, const T* U, int ldu, const T* V, int ldv,
                     const double* S, double eps, T* A, int lda, hipStream_t s)
{
    dim3 grid((n + TILE - 1) / TILE, (m + TILE - 1) / TILE);
    TimedLaunch tl(tm, "svt_reconstruct", s, 2.0 * m * (double)n * b,
                   sizeof(T) * (double)m * n);
    hipLaunchKernelGGL((svt_tile_kernel<T, 1>), grid, dim3(256), 0, s, m, n, b, U, ldu, V, ldv, S,
                       eps, 0.0, 1.0, 1.0, (const T*)nullptr, 0, (T*)nullptr, (T*)nullptr, 0,
                       (T*)nullptr, (unsigned short*)nullptr, (unsigned short*)nullptr, A, lda,
                       (double*)nullptr);
}

// The per-iteration readback gathered by one kernel: the summed partials, and
// two device counters copied beside them (rank may be null: then 0).
__global__ void iter_readback_kernel(int count, const double* p, const int* rank, const int* err,
                                     double* zz, int* rank_out, int* err_out)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += 64) s += p[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) {
        zz[0] = s;
        rank_out[0] = rank ? rank[0] : 0;
        err_out[0] = err[0];
    }
}

void iter_readback(int count, const double* partials, const int* rank, const int* err, double* zz,
                   int* rank_out, int* err_out, hipStream_t s)
{
    hipLaunchKernelGGL(iter_readback_kernel, dim3(1), dim3(64), 0, s, count, partials, rank, err,
                       zz, rank_out, err_out);
}

void sum_partials(int count, const double* partials, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, count, partials, out);
}

template <typename T>
void count_nonzeros(int m, int n, const T* X, int ldx, long long* out, long long* scratch,
                    hipStream_t s)
{
    hipLaunchKernelGGL((nnz_kernel<T>), dim3(RED_BLOCKS), dim3(256), 0, s, m, n, X, ldx, scratch);
    hipLaunchKernelGGL(nnz_final_kernel, dim3(1), dim3(64), 0, s, RED_BLOCKS, scratch, out);
}

#define BLWS_ELEM_INST(T)                                                                     \
    template void norms<T>(int, int, const T*, int, double*, double*, hipStream_t);             \
    template void rpca_init<T>(int, int, const T*, int, double, double, T*, T*, int, T*,         \
                               hipStream_t);                                                   \
    template void alm_epilogue<T>(Timer*, int, int, int, const T*, int, const T*, int,          \
                                  const double*, double, double, double, double, const T*, int, \
                                  T*, T*, int, T*, unsigned short*, T*, int, double*,           \
                                  hipStream_t, unsigned short*);                                \
    template void svt_reconstruct<T>(Timer*, int, int, int, const T*, int, const T*, int,       \
                                     const double*, double, T*, int, hipStream_t);             \
    template void count_nonzeros<T>(int, int, const T*, int, long long*, long long*,            \
                                    hipStream_t);
BLWS_ELEM_INST(double)
BLWS_ELEM_INST(float)
#undef BLWS_ELEM_INST

}  // namespace blws
