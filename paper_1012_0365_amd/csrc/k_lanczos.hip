// Kernels of the literal block Lanczos procedure on the augmented matrix
// [[0, W], [W^T, 0]] (Algorithms 2 and 3; the start-block ablations of
// Sec. 4.1): the diagonal blocks M_l, the block tridiagonal T_k, and its
// eigenvalues from the SVD of a shifted copy.
//
// T_k is symmetric but indefinite (its eigenvalues come in near +-sigma
// pairs, Theorem 1), so its EVD is taken from the SVD of T_k + c I with c at
// least the spectral radius (Gershgorin: the largest absolute row sum). The
// shifted matrix is positive semidefinite, its singular values are
// lambda_i + c in the same decreasing order and its left singular vectors are
// the eigenvectors; the absolute error of each lambda_i is that of the SVD,
// a rounding unit of c ~ ||T_k||, as for any backward-stable symmetric EVD.
#include "blws_common.h"

namespace blws {
namespace {

// M (c x c) = S + S^T
__global__ void lz_sym_kernel(int c, const double* __restrict__ S, double* __restrict__ M)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c * c) return;
    const int i = e / c, j = e - i * c;
    M[e] = S[(size_t)i * c + j] + S[(size_t)j * c + i];
}

// Bt (c x c) = B^T
__global__ void lz_transpose_kernel(int c, const double* __restrict__ B, double* __restrict__ Bt)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c * c) return;
    const int i = e / c, j = e - i * c;
    Bt[e] = B[(size_t)j * c + i];
}

// Entry (i, j) of T_k: block (l, l) = M_l, block (l + 1, l) = B_l, block
// (l, l + 1) = B_l^T, zero elsewhere (K = k c).
__device__ __forceinline__ double lz_t(int c, int k, const double* Ms, const double* Bs, int i,
                                       int j)
{
    const int li = i / c, lj = j / c, a = i - li * c, e = j - lj * c;
    if (li == lj) return Ms[((size_t)li * c + a) * c + e];
    if (li == lj + 1) return Bs[((size_t)lj * c + a) * c + e];
    if (lj == li + 1) return Bs[((size_t)li * c + e) * c + a];
    return 0.0;
}

// shift = max_i sum_j |T_ij| over the nonzero blocks of row i; one workgroup.
__global__ __launch_bounds__(1024) void lz_shift_kernel(int k, int c, const double* __restrict__ Ms,
                                                        const double* __restrict__ Bs,
                                                        double* __restrict__ shift)
{
    __shared__ double red[1024];
    const int K = k * c;
    double best = 0.0;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        const int l = i / c;
        const int j0 = (l > 0 ? l - 1 : 0) * c, j1 = (l + 1 < k ? l + 2 : k) * c;
        double sum = 0.0;
        for (int j = j0; j < j1; ++j) sum += fabs(lz_t(c, k, Ms, Bs, i, j));
        best = fmax(best, sum);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    // a zero T_k still gets a positive shift (the SVD then sees c I)
    if (threadIdx.x == 0) *shift = red[0] > 0.0 ? red[0] : 1.0;
}

// T (K x K, ld K) = T_k + shift I
__global__ void lz_assemble_kernel(int k, int c, const double* __restrict__ Ms,
                                   const double* __restrict__ Bs, const double* __restrict__ shift,
                                   double* __restrict__ T)
{
    const int K = k * c;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)K * K) return;
    const int i = (int)(e / K), j = (int)(e - (long long)i * K);
    T[e] = lz_t(c, k, Ms, Bs, i, j) + (i == j ? *shift : 0.0);
}

// lambda_i = sigma_i(T_k + shift I) - shift, i < b
__global__ void lz_eigvals_kernel(int b, const double* __restrict__ sig,
                                  const double* __restrict__ shift, double* __restrict__ lam)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b) lam[i] = sig[i] - *shift;
}

}  // namespace

void lanczos_sym(int c, const double* S, double* M, hipStream_t s)
{
    const int total = c * c;
    hipLaunchKernelGGL(lz_sym_kernel, dim3((total + 255) / 256), dim3(256), 0, s, c, S, M);
    HIP_TRY(hipGetLastError());
}

void lanczos_transpose(int c, const double* B, double* Bt, hipStream_t s)
{
    const int total = c * c;
    hipLaunchKernelGGL(lz_transpose_kernel, dim3((total + 255) / 256), dim3(256), 0, s, c, B, Bt);
    HIP_TRY(hipGetLastError());
}

void lanczos_assemble(int k, int c, const double* Ms, const double* Bs, double* shift, double* T,
                      hipStream_t s)
{
    hipLaunchKernelGGL(lz_shift_kernel, dim3(1), dim3(1024), 0, s, k, c, Ms, Bs, shift);
    HIP_TRY(hipGetLastError());
    const long long total = (long long)k * c * k * c;
    hipLaunchKernelGGL(lz_assemble_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       k, c, Ms, Bs, shift, T);
    HIP_TRY(hipGetLastError());
}

void lanczos_eigvals(int b, const double* sig, const double* shift, double* lam, hipStream_t s)
{
    hipLaunchKernelGGL(lz_eigvals_kernel, dim3((b + 255) / 256), dim3(256), 0, s, b, sig, shift,
                       lam);
    HIP_TRY(hipGetLastError());
}

}  // namespace blws
