// Kernels of the matrix-completion operator.
//
// In the ALM for matrix completion the matrix whose SVT is taken is low rank
// plus sparse, W = U_r diag(theta) V_r^T + S_Omega (Sec. 2, Eq. (2) and its
// ALM host), and is never formed: its products with a block are a sparse-dense
// product over Omega plus two skinny GEMMs with the factors. W^T products use a
// transposed copy of the pattern (column pointers, row indices and, for each
// position, the index of the value in CSR order), built once per solve in a
// fixed order so that every sum runs in the same order on every call.
//
// The per-iteration update over Omega (A_Omega from the factors, the multiplier
// and residual, the next sparse part) is one fused pass.
#include <limits.h>

#include "blws_common.h"

namespace blws {
namespace {

constexpr int SEG_LDS = 4096;  // column segments up to this length sort in LDS

__global__ void csr_check_kernel(int m, int n, int nnz, const int* row_ptr, const int* col_idx,
                                 int* flag)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    int bad = 0;
    for (int i = tid; i <= m; i += stride) {
        const int a = row_ptr[i];
        if (a < 0 || a > nnz) bad |= 1;
        if (i == 0 && a != 0) bad |= 1;
        if (i == m && a != nnz) bad |= 1;
        if (i < m && row_ptr[i + 1] < a) bad |= 1;
    }
    for (int e = tid; e < nnz; e += stride) {
        const int c = col_idx[e];
        if (c < 0 || c >= n) bad |= 2;
    }
    if (bad) atomicOr(flag, bad);
}

__global__ void col_count_kernel(int nnz, const int* col_idx, int* cnt)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x)
        atomicAdd(&cnt[col_idx[e]], 1);
}

// Exclusive scan of cnt[0..n) into ptr[0..n] and the largest count into
// maxcnt[0], by one workgroup of 1024 threads in chunks.
__global__ __launch_bounds__(1024) void scan_kernel(int n, const int* cnt, int* ptr, int* maxcnt)
{
    __shared__ int sh[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    int mx = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + t;
        const int v = i < n ? cnt[i] : 0;
        mx = v > mx ? v : mx;
        sh[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int add = t >= off ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += add;
            __syncthreads();
        }
        const int incl = sh[t];
        if (i < n) ptr[i] = carry + incl - v;
        __syncthreads();
        if (t == 1023) carry += incl;
        __syncthreads();
    }
    if (t == 0) ptr[n] = carry;
    sh[t] = mx;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (t < off && sh[t + off] > sh[t]) sh[t] = sh[t + off];
        __syncthreads();
    }
    if (t == 0) maxcnt[0] = sh[0];
}

// Scatter CSR positions into their columns (order within a column arbitrary;
// the segment sort below fixes it).
__global__ void csc_scatter_kernel(int nnz, const int* col_idx, const int* col_ptr, int* cursor,
                                   int* perm)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
        const int c = col_idx[e];
        perm[col_ptr[c] + atomicAdd(&cursor[c], 1)] = e;
    }
}

__global__ void row_of_kernel(int m, const int* row_ptr, int* row_of)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) row_of[e] = i;
}

// Sort each column's CSR positions ascending (= by row, CSR being row-major),
// from perm into out, and record the row of each position. One workgroup per
// column: bitonic sort in LDS, or counting ranks for long columns.
__global__ __launch_bounds__(256) void seg_sort_kernel(int n, const int* col_ptr, const int* perm,
                                                        const int* row_of, int* out, int* csc_row)
{
    __shared__ int key[SEG_LDS];
    const int j = blockIdx.x;
    if (j >= n) return;
    const int a = col_ptr[j], L = col_ptr[j + 1] - a;
    if (L <= SEG_LDS) {
        int P = 1;
        while (P < L) P <<= 1;
        for (int t = threadIdx.x; t < P; t += 256) key[t] = t < L ? perm[a + t] : INT_MAX;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1)
            for (int h = k >> 1; h > 0; h >>= 1) {
                for (int t = threadIdx.x; t < P; t += 256) {
                    const int u = t ^ h;
                    if (u > t) {
                        const int x = key[t], y = key[u];
                        const bool up = (t & k) == 0;
                        if ((x > y) == up && x != y) {
                            key[t] = y;
                            key[u] = x;
                        }
                    }
                }
                __syncthreads();
            }
        for (int t = threadIdx.x; t < L; t += 256) {
            const int e = key[t];
            out[a + t] = e;
            csc_row[a + t] = row_of[e];
        }
    } else {
        for (int t = threadIdx.x; t < L; t += 256) {
            const int e = perm[a + t];
            int rank = 0;
            for (int u = 0; u < L; ++u) rank += perm[a + u] < e;
            out[a + rank] = e;
            csc_row[a + rank] = row_of[e];
        }
    }
}

// out (rows x c, ldo) = sum over the entries of each row of val * X[idx, :].
// One wavefront per row; lanes over the c columns (c <= 512); entries fetched
// 64 at a time and broadcast; sums in FP64 in entry order. With `perm` the
// value of position e is val[perm[e]] (the transposed pattern).
template <typename T, int QN>
__global__ __launch_bounds__(256) void spmm_kernel(int rows, int c, const int* ptr,
                                                   const int* idx, const int* perm, const T* val,
                                                   const T* X, int ldx, T* out, int ldo)
{
    // QN = ceil(c / 64) chunks of 64 columns, one value per lane each; the
    // rows of X for eight samples are loaded before any is used (the gathers,
    // mostly from L2 and the last-level cache, are what the kernel waits on)
    constexpr int G = 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave;
    if (i >= rows) return;  // no barriers below
    const int a = ptr[i], z = ptr[i + 1];
    bool live[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) live[q] = lane + 64 * q < c;
    double acc[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) acc[q] = 0.0;
    for (int base = a; base < z; base += 64) {
        const int e = base + lane;
        int col = 0;
        double v = 0.0;
        if (e < z) {
            col = idx[e];
            v = (double)val[perm ? perm[e] : e];
        }
        const int cnt = (z - base) < 64 ? (z - base) : 64;
        int t = 0;
        for (; t + G <= cnt; t += G) {
            T xv[G][QN];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const T* xr = X + (size_t)__shfl(col, t + u, 64) * ldx + lane;
#pragma unroll
                for (int q = 0; q < QN; ++q) xv[u][q] = live[q] ? xr[64 * q] : T(0);
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const double vv = __shfl(v, t + u, 64);
#pragma unroll
                for (int q = 0; q < QN; ++q) acc[q] += vv * (double)xv[u][q];
            }
        }
        for (; t < cnt; ++t) {
            const T* xr = X + (size_t)__shfl(col, t, 64) * ldx + lane;
            const double vv = __shfl(v, t, 64);
#pragma unroll
            for (int q = 0; q < QN; ++q)
                if (live[q]) acc[q] += vv * (double)xr[64 * q];
        }
    }
#pragma unroll
    for (int q = 0; q < QN; ++q)
        if (live[q]) out[(size_t)i * ldo + lane + 64 * q] = (T)acc[q];
}

// C (r x c, ldc) row k *= (S[k] - eps): the coefficients theta of the low-rank part.
__global__ void lr_scale_kernel(int r, int c, const double* S, double eps, double* C, int ldc)
{
    const int k = blockIdx.x;
    if (k >= r) return;
    const double th = S[k] - eps;
    for (int j = threadIdx.x; j < c; j += blockDim.x) C[(size_t)k * ldc + j] *= th;
}

// Fused update over Omega, one wavefront per row i:
//   a_e  = sum_{k < r} (U[i][k] (S[k] - eps)) V[col_e][k]     (A on Omega)
//   z    = d_e - a_e;  y_e += mu z;  s_e = d_e + y_e / mu_next - a_e
// and per-workgroup partial sums of z^2. r = min(*rank_dev, rmax).
template <typename T>
__global__ __launch_bounds__(256) void mc_update_kernel(
    int m, const int* row_ptr, const int* col_idx, const T* d, T* y, T* sv, const T* U, int ldu,
    const T* V, int ldv, const double* S, double eps, const int* rank_dev, int rmax, double mu,
    double mu_next, int need, double* part)
{
    __shared__ double coef[4][512];
    __shared__ double red[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave;
    if (rank_dev[0] >= need) {  // the host repeats the thresholding first
        if (threadIdx.x == 0) part[blockIdx.x] = 0.0;
        return;
    }
    int r = rank_dev[0];
    if (r > rmax) r = rmax;
    if (r < 0) r = 0;
    if (i < m)
        for (int k = lane; k < r; k += 64) coef[wave][k] = (double)U[(size_t)i * ldu + k] * (S[k] - eps);
    __syncthreads();
    double zz = 0.0;
    if (i < m) {
        const int a = row_ptr[i], z = row_ptr[i + 1];
        // V's rows four values per load where they are 16-byte aligned (FP32,
        // ldv and V's base multiples of 4 values); the sum runs in the same order
        const bool vec4 = sizeof(T) == 4 && (ldv & 3) == 0 && (((uintptr_t)V) & 15) == 0;
        const int r4 = vec4 ? (r & ~3) : 0;
        for (int e = a + lane; e < z; e += 64) {
            const T* vr = V + (size_t)col_idx[e] * ldv;
            double s = 0.0;
            for (int k = 0; k < r4; k += 4) {
                const float4 q = *(const float4*)(vr + k);
                s += coef[wave][k] * (double)q.x;
                s += coef[wave][k + 1] * (double)q.y;
                s += coef[wave][k + 2] * (double)q.z;
                s += coef[wave][k + 3] * (double)q.w;
            }
            for (int k = r4; k < r; ++k) s += coef[wave][k] * (double)vr[k];
            const double dd = (double)d[e];
            const double zv = dd - s;
            const T yn = (T)((double)y[e] + mu * zv);
            y[e] = yn;
            if (sv) sv[e] = (T)(dd + (double)yn / mu_next - s);
            zz += zv * zv;
        }
    }
    for (int off = 32; off > 0; off >>= 1) zz += __shfl_xor(zz, off, 64);
    if (lane == 0) red[wave] = zz;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

template <typename T>
__global__ void scale_copy_kernel(int nnz, double alpha, const T* d, T* y)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x)
        y[e] = (T)(alpha * (double)d[e]);
}

template <typename T>
__global__ void mc_init_kernel(int nnz, const T* d, T* y, T* sv)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
        y[e] = (T)0;
        sv[e] = d[e];
    }
}

// Sout[k] = S[k] - eps for k < r (the singular values of the returned A).
__global__ void theta_out_kernel(int r, const double* S, double eps, double* Sout)
{
    for (int k = threadIdx.x; k < r; k += blockDim.x) Sout[k] = S[k] - eps;
}

int grid_for(long long work, int block)
{
    long long g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

void csr_check(int m, int n, int nnz, const int* row_ptr, const int* col_idx, int* flag,
               hipStream_t s)
{
    zero_bytes(flag, sizeof(int), s);
    hipLaunchKernelGGL(csr_check_kernel, dim3(grid_for((long long)nnz + m + 1, 256)), dim3(256),
                       0, s, m, n, nnz, row_ptr, col_idx, flag);
}

size_t csc_scratch_ints(int n, int nnz) { return 2 * (size_t)(n + 1) + 2 * (size_t)nnz + 4; }

void csc_build(int m, int n, int nnz, const int* row_ptr, const int* col_idx, int* col_ptr,
               int* csc_row, int* csc_perm, int* maxcnt, int* scratch, hipStream_t s)
{
    int* cnt = scratch;                   // n + 1
    int* cursor = cnt + (n + 1);          // n + 1
    int* perm = cursor + (n + 1);         // nnz
    int* row_of = perm + nnz;             // nnz
    zero_bytes(cnt, 2 * (size_t)(n + 1) * sizeof(int), s);
    if (nnz > 0)
        hipLaunchKernelGGL(col_count_kernel, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz,
                           col_idx, cnt);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, n, cnt, col_ptr, maxcnt);
    if (nnz == 0) return;
    hipLaunchKernelGGL(csc_scatter_kernel, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz,
                       col_idx, col_ptr, cursor, perm);
    hipLaunchKernelGGL(row_of_kernel, dim3(grid_for(m, 256)), dim3(256), 0, s, m, row_ptr,
                       row_of);
    hipLaunchKernelGGL(seg_sort_kernel, dim3(n), dim3(256), 0, s, n, col_ptr, perm, row_of,
                       csc_perm, csc_row);
}

template <typename T>
void spmm(Timer* tm, const char* family, int rows, int c, const int* ptr, const int* idx,
          const int* perm, const T* val, const T* X, int ldx, T* out, int ldo, long long nnz,
          hipStream_t s)
{
    if (rows <= 0 || c <= 0) return;
    BLWS_REQUIRE(c <= 512, BLWS_EUNSUPPORTED, "spmm: more than 512 columns");
    TimedLaunch tl(tm, family, s, 2.0 * (double)nnz * c,
                   (double)nnz * (sizeof(int) + sizeof(T) + (perm ? sizeof(int) : 0) +
                                  (double)c * sizeof(T)) +
                       (double)rows * c * sizeof(T));
    const dim3 grid((rows + 3) / 4);
    switch ((c + 63) / 64) {
#define BLWS_SPMM_CASE(Q)                                                                      \
    case Q:                                                                                    \
        hipLaunchKernelGGL((spmm_kernel<T, Q>), grid, dim3(256), 0, s, rows, c, ptr, idx, perm, \
                           val, X, ldx, out, ldo);                                             \
        break;
        BLWS_SPMM_CASE(1)
        BLWS_SPMM_CASE(2)
        BLWS_SPMM_CASE(3)
        BLWS_SPMM_CASE(4)
        BLWS_SPMM_CASE(5)
        BLWS_SPMM_CASE(6)
        BLWS_SPMM_CASE(7)
        BLWS_SPMM_CASE(8)
#undef BLWS_SPMM_CASE
    }
}

void lr_scale(int r, int c, const double* S, double eps, double* C, int ldc, hipStream_t s)
{
    if (r <= 0 || c <= 0) return;
    hipLaunchKernelGGL(lr_scale_kernel, dim3(r), dim3(64), 0, s, r, c, S, eps, C, ldc);
}

size_t mc_partials(int m) { return (size_t)(m + 3) / 4; }

template <typename T>
void mc_update(Timer* tm, int m, long long nnz, const int* row_ptr, const int* col_idx,
               const T* d, T* y, T* sv, const T* U, int ldu, const T* V, int ldv, const double* S,
               double eps, const int* rank_dev, int rmax, double mu, double mu_next, int need,
               double* partials, hipStream_t s)
{
    BLWS_REQUIRE(rmax <= 512, BLWS_EUNSUPPORTED, "mc_update: rank above 512");
    TimedLaunch tl(tm, "mc_update", s, 2.0 * (double)nnz * rmax,
                   (double)nnz * (sizeof(int) + 5.0 * sizeof(T)));
    hipLaunchKernelGGL((mc_update_kernel<T>), dim3((m + 3) / 4), dim3(256), 0, s, m, row_ptr,
                       col_idx, d, y, sv, U, ldu, V, ldv, S, eps, rank_dev, rmax, mu, mu_next,
                       need, partials);
}

template <typename T>
void scale_copy(long long nnz, double alpha, const T* d, T* y, hipStream_t s)
{
    if (nnz <= 0) return;
    hipLaunchKernelGGL((scale_copy_kernel<T>), dim3(grid_for(nnz, 256)), dim3(256), 0, s,
                       (int)nnz, alpha, d, y);
}

template <typename T>
void mc_init(long long nnz, const T* d, T* y, T* sv, hipStream_t s)
{
    if (nnz <= 0) return;
    hipLaunchKernelGGL((mc_init_kernel<T>), dim3(grid_for(nnz, 256)), dim3(256), 0, s, (int)nnz,
                       d, y, sv);
}

void theta_out(int r, const double* S, double eps, double* Sout, hipStream_t s)
{
    if (r <= 0) return;
    hipLaunchKernelGGL(theta_out_kernel, dim3(1), dim3(256), 0, s, r, S, eps, Sout);
}

#define BLWS_INST_SPARSE(T)                                                                   \
    template void spmm<T>(Timer*, const char*, int, int, const int*, const int*, const int*,    \
                          const T*, const T*, int, T*, int, long long, hipStream_t);           \
    template void mc_update<T>(Timer*, int, long long, const int*, const int*, const T*, T*,   \
                               T*, const T*, int, const T*, int, const double*, double,         \
                               const int*, int, double, double, int, double*, hipStream_t);     \
    template void mc_init<T>(long long, const T*, T*, T*, hipStream_t);                        \
    template void scale_copy<T>(long long, double, const T*, T*, hipStream_t);
BLWS_INST_SPARSE(double)
BLWS_INST_SPARSE(float)

}  // namespace blws
