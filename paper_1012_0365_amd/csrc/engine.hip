// Host side of libblws: workspace, the BLWS step, the inexact-ALM RPCA loop,
// kernel timing and the C ABI declared in include/blws.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <type_traits>
#include <vector>

#include "blws_common.h"

namespace blws {

// ---------------------------------------------------------------------------
// Timing
// ---------------------------------------------------------------------------
struct Timer {
    bool on = false;
    struct Family {
        std::vector<hipEvent_t> start, stop;
        double flops = 0.0, bytes = 0.0;
        long long launches = 0;
    };
    std::map<std::string, Family> fam;
    void clear()
    {
        for (auto& kv : fam) {
            for (auto e : kv.second.start) (void)hipEventDestroy(e);
            for (auto e : kv.second.stop) (void)hipEventDestroy(e);
        }
        fam.clear();
    }
};

TimedLaunch::TimedLaunch(Timer* timer, const char* family, hipStream_t s, double flops,
                         double bytes)
    : t(timer && timer->on ? timer : nullptr), slot(-1), stream(s), fam(family)
{
    if (!t) return;
    Timer::Family& f = t->fam[family];
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(a, s));
    f.start.push_back(a);
    f.stop.push_back(b);
    f.flops += flops;
    f.bytes += bytes;
    f.launches += 1;
    slot = (int)f.stop.size() - 1;
}

TimedLaunch::~TimedLaunch()
{
    if (!t || slot < 0) return;
    (void)hipEventRecord(t->fam[fam].stop[slot], stream);
}

namespace {

constexpr double CHOL_ETA = 1e-13;  // scaled pivot below which a column is dependent

// ---------------------------------------------------------------------------
// Workspace: one device allocation per context, carved into sub-buffers.
// ---------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct Context {
    int device = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* host_pinned = nullptr;  // small readback area
    std::string last_error;
    Timer timer;
    uint64_t fix_calls = 0;  // stream ids for breakdown replacement draws

    void ensure(size_t bytes)
    {
        if (bytes <= ws_bytes) return;
        HIP_TRY(hipDeviceSynchronize());
        if (ws) HIP_TRY(hipFree(ws));
        ws = nullptr;
        ws_bytes = 0;
        size_t want = bytes + (bytes >> 3);
        hipError_t e = hipMalloc(&ws, want);
        if (e != hipSuccess) {
            ws = nullptr;
            throw BlwsError{BLWS_ENOMEM, "workspace allocation failed"};
        }
        ws_bytes = want;
    }
};

namespace {

// Scratch of one BLWS step at block width b on an m x n matrix.
template <typename T>
struct StepWs {
    T *UF, *PH, *VG, *Qb, *T1, *T2, *R;
    double *Cp, *Gr, *Ri, *Bm, *UB, *VB, *Sall, *svd, *chol, *partial, *D1, *D2;
    int *flags, *nflag;
    size_t partial_elems;

    void carve(Carver& c, int m, int n, int b)
    {
        const int b2 = 2 * b, mx = m > n ? m : n;
        UF = c.take<T>((size_t)m * b2);
        PH = c.take<T>((size_t)m * b2);
        VG = c.take<T>((size_t)n * b2);
        Qb = c.take<T>((size_t)n * b);
        T1 = c.take<T>((size_t)mx * b);
        T2 = c.take<T>((size_t)mx * b);
        R = c.take<T>((size_t)mx * b);
        Cp = c.take<double>((size_t)b * b);
        Gr = c.take<double>((size_t)b * b);
        Ri = c.take<double>((size_t)b * b);
        Bm = c.take<double>((size_t)b2 * b2);
        UB = c.take<double>((size_t)b2 * b2);
        VB = c.take<double>((size_t)b2 * b2);
        Sall = c.take<double>((size_t)b2);
        {
            size_t e1 = small_svd_jacobi_scratch_elems(b2), e2 = small_svd_gk_scratch_elems(b2);
            svd = c.take<double>(e1 > e2 ? e1 : e2);
        }
        D1 = c.take<double>((size_t)b2 * b);
        D2 = c.take<double>((size_t)b2 * b);
        chol = c.take<double>(chol_scratch_elems(b) + 1);
        flags = c.take<int>((size_t)b);
        nflag = c.take<int>(4);
        size_t pe = 0;
        const int shapes[][3] = {{m, b, n},  {n, b, m},   {b, b, m},  {b, b, n},
                                 {b2, b2, m}, {m, b, b2}, {n, b, b2}, {m, b, b},
                                 {n, b, b}};
        for (auto& sh : shapes) {
            size_t e = gemm_partial_elems(sh[0], sh[1], sh[2]);
            if (e > pe) pe = e;
            // the FP32 / BF16 W-product kernels keep FP32 partials in the same buffer
            e = (gemm_lp_partial_elems(sh[0], sh[1], sh[2]) + 1) / 2;
            if (e > pe) pe = e;
        }
        partial_elems = pe;
        partial = c.take<double>(pe + 1);
    }
};

// Scratch of one orthonormalisation: T1, T2 (rows x 128), Cp (b x 128, b the
// widest block projected against), Gr, Ri (128 x 128), the Cholesky scratch,
// the breakdown flags (nflag[0] counts them) and the split-K partials.
template <typename T>
struct OrthWs {
    T *T1, *T2;
    double *Cp, *Gr, *Ri, *chol, *partial;
    size_t partial_elems;
    int *flags, *nflag;
};

constexpr int ORTH_CHUNK = 128;  // widest Cholesky-QR block (register Cholesky)

// dst (rows x c, ld c) = src minus its components in span(X_0), span(X_1), ...,
// block after block (each X_q rows x bx[q], orthonormal columns).
template <typename T>
void project_out(Context& cx, const OrthWs<T>& w, hipStream_t s, int rows, int nx,
                 const T* const* X, const int* ldx, const int* bx, const T* src, int lds, T* dst,
                 int c)
{
    Timer* tm = &cx.timer;
    if (nx == 0) {
        copy2d<T, T>(rows, c, src, lds, dst, c, s);
        return;
    }
    const T* cur = src;
    int ldcur = lds;
    for (int q = 0; q < nx; ++q) {
        gemm<T, T, double>(tm, "gemm_ts", true, bx[q], c, rows, 1.0, X[q], ldx[q], cur, ldcur, 0.0,
                           (const double*)nullptr, 0, w.Cp, c, w.partial, w.partial_elems, s);
        gemm<T, double, T>(tm, "gemm_ts", false, rows, c, bx[q], -1.0, X[q], ldx[q], w.Cp, c, 1.0,
                           cur, ldcur, dst, c, w.partial, w.partial_elems, s);
        cur = dst;
        ldcur = c;
    }
}

// One block of at most ORTH_CHUNK columns: project In out of the X blocks,
// then two Cholesky-QR passes, the X blocks projected out again between them.
// Columns found dependent in the first pass are replaced by counter-based
// random draws, which the second projection and pass orthonormalise.
template <typename T>
void orth_chunk(Context& cx, const OrthWs<T>& w, hipStream_t s, int rows, int nx,
                const T* const* X, const int* ldx, const int* bx, const T* In, int ldin, int c,
                T* Out, int ldout, uint64_t seed)
{
    Timer* tm = &cx.timer;
    project_out<T>(cx, w, s, rows, nx, X, ldx, bx, In, ldin, w.T1, c);
    T* cur = w.T1;
    for (int pass = 0; pass < 2; ++pass) {
        gemm<T, T, double>(tm, "gemm_ts", true, c, c, rows, 1.0, cur, c, cur, c, 0.0,
                           (const double*)nullptr, 0, w.Gr, c, w.partial, w.partial_elems, s);
        chol_inv(tm, c, w.Gr, c, w.Ri, w.flags, w.nflag, CHOL_ETA, w.chol, s);
        T* dst = (pass == 0) ? w.T2 : Out;
        const int ldd = (pass == 0) ? c : ldout;
        gemm<T, double, T>(tm, "gemm_ts", false, rows, c, c, 1.0, cur, c, w.Ri, c, 0.0,
                           (const T*)nullptr, 0, dst, ldd, w.partial, w.partial_elems, s);
        if (pass == 0) {
            fill_flagged<T>(rows, c, w.T2, c, w.flags, seed, (1ULL << 20) + (++cx.fix_calls), s);
            if (nx > 0) {
                project_out<T>(cx, w, s, rows, nx, X, ldx, bx, w.T2, c, w.T1, c);
                cur = w.T1;
            } else {
                cur = w.T2;
            }
        }
    }
}

// Orthonormalise `In` (rows x c, ldin) against the orthonormal block X (rows x b0,
// may be null) into Out: the QR step of the block Lanczos procedure
// (Algorithm 2). Blocks of ORTH_CHUNK columns are orthonormalised in turn,
// each against X and the blocks before it (block Gram-Schmidt), so that every
// Cholesky factorisation is at most ORTH_CHUNK wide. In may equal Out.
template <typename T>
void orth_against(Context& cx, const OrthWs<T>& w, hipStream_t s, int rows, int b0, const T* X,
                  int ldx, const T* In, int ldin, int c, T* Out, int ldout, uint64_t seed)
{
    for (int c0 = 0; c0 < c; c0 += ORTH_CHUNK) {
        const int cc = (c - c0) < ORTH_CHUNK ? (c - c0) : ORTH_CHUNK;
        const T* Xs[2];
        int lds[2], bs[2], nx = 0;
        if (X && b0 > 0) {
            Xs[nx] = X;
            lds[nx] = ldx;
            bs[nx++] = b0;
        }
        if (c0 > 0) {
            Xs[nx] = Out;
            lds[nx] = ldout;
            bs[nx++] = c0;
        }
        orth_chunk<T>(cx, w, s, rows, nx, Xs, lds, bs, In + c0, ldin, cc, Out + c0, ldout, seed);
    }
}

template <typename T>
void orth_against(Context& cx, StepWs<T>& sw, hipStream_t s, int rows, int b0, const T* X,
                  int ldx, const T* In, int ldin, int c, T* Out, int ldout, uint64_t seed)
{
    const OrthWs<T> w{sw.T1, sw.T2, sw.Cp, sw.Gr, sw.Ri, sw.chol, sw.partial, sw.partial_elems,
                      sw.flags, sw.nflag};
    orth_against<T>(cx, w, s, rows, b0, X, ldx, In, ldin, c, Out, ldout, seed);
}

// SVD of the small projected matrix: the top nv values and vectors, by the
// Golub-Kahan path (N <= 512), whose leading vectors are then polished to
// orthonormal by Cholesky-QR (inverse iteration leaves the vectors of close
// values only nearly orthogonal). The one-sided Jacobi kernel serves larger N.
// nflag[1] is set if the cooperative bidiagonalisation timed out.
void small_svd_dispatch(Context& cx, hipStream_t s, int N, int nv, const double* B, int ldb,
                        double* UB, double* S, double* VB, double* svd_scratch,
                        const OrthWs<double>& w, uint64_t seed)
{
    TimedLaunch tl(&cx.timer, "small_svd", s, 0.0, 0.0);
    if (small_svd_gk_supported(N)) {
        small_svd_gk(&cx.timer, N, nv, B, ldb, UB, S, VB, svd_scratch, w.nflag + 1, s);
        orth_against<double>(cx, w, s, N, 0, nullptr, 0, UB, N, nv, UB, N, seed);
        orth_against<double>(cx, w, s, N, 0, nullptr, 0, VB, N, nv, VB, N, seed);
    } else {
        small_svd_jacobi(&cx.timer, N, B, ldb, UB, S, VB, svd_scratch, s);
    }
}

// The matrix whose SVT is taken, seen only through its products with blocks.
// Dense (RPCA: W stored), or low rank plus sparse (matrix completion:
// W = Ul diag(S - eps) Vl^T + S_Omega with the low-rank part of rank r, never
// formed).
template <typename T>
struct McOp {
    int nnz = 0;
    const int *row_ptr = nullptr, *col_idx = nullptr;                   // CSR pattern
    const int *col_ptr = nullptr, *csc_row = nullptr, *csc_perm = nullptr;  // transposed
    const T* sval = nullptr;  // sparse part, CSR order
    int r = 0;                // rank of the low-rank part
    const T *Ul = nullptr, *Vl = nullptr;
    int ldl = 0;
    const double* S = nullptr;  // theta_k = S[k] - eps
    double eps = 0.0;
    double* coef = nullptr;  // r x c scratch
};

template <typename T>
struct Op {
    const T* W = nullptr;
    int ldw = 0;
    const McOp<T>* mc = nullptr;
    const unsigned short* Wh = nullptr;  // BF16 copy of W (ld ldw): products in BF16
};

// out (rows x c) = W X (trans = false: X is n x c, rows = m) or W^T X
// (trans = true: X is m x c, rows = n).
template <typename T>
void op_apply(Context& cx, StepWs<T>& w, hipStream_t s, const Op<T>& op, int m, int n,
              bool trans, const T* X, int ldx, int c, T* out, int ldo)
{
    Timer* tm = &cx.timer;
    const int rows = trans ? n : m, inner = trans ? m : n;
    if (op.W) {
        if constexpr (std::is_same<T, float>::value) {
            // FP32 or BF16 matrix cores, FP32 accumulation
            const bool bf = op.Wh != nullptr;
            gemm_lp(tm, "gemm_w", bf, trans, rows, c, inner,
                    bf ? (const void*)op.Wh : (const void*)op.W, op.ldw, X, ldx, out, ldo,
                    (float*)w.partial, 2 * w.partial_elems, s);
        } else {
            gemm<T, T, T>(tm, "gemm_w", trans, rows, c, inner, 1.0, op.W, op.ldw, X, ldx, 0.0,
                          (const T*)nullptr, 0, out, ldo, w.partial, w.partial_elems, s);
        }
        return;
    }
    const McOp<T>& mc = *op.mc;
    if (!trans)
        spmm<T>(tm, "spmm", m, c, mc.row_ptr, mc.col_idx, nullptr, mc.sval, X, ldx, out, ldo,
                mc.nnz, s);
    else
        spmm<T>(tm, "spmm", n, c, mc.col_ptr, mc.csc_row, mc.csc_perm, mc.sval, X, ldx, out, ldo,
                mc.nnz, s);
    if (mc.r > 0) {
        // W X = Ul (theta o (Vl^T X)) + S X;  W^T X = Vl (theta o (Ul^T X)) + S^T X
        const T* L = trans ? mc.Ul : mc.Vl;
        const T* Rf = trans ? mc.Vl : mc.Ul;
        gemm<T, T, double>(tm, "gemm_lr", true, mc.r, c, inner, 1.0, L, mc.ldl, X, ldx, 0.0,
                           (const double*)nullptr, 0, mc.coef, c, w.partial, w.partial_elems, s);
        lr_scale(mc.r, c, mc.S, mc.eps, mc.coef, c, s);
        gemm<T, double, T>(tm, "gemm_lr", false, rows, c, mc.r, 1.0, Rf, mc.ldl, mc.coef, c, 1.0,
                           out, ldo, out, ldo, w.partial, w.partial_elems, s);
    }
}

// One BLWS step (Algorithms 2-3, k = 2) on W from the orthonormal block
// (U, V); on return U, V hold the top-b Ritz vectors and S the Ritz values.
//
// The augmented matrix [[0, W], [W^T, 0]] (Theorem 1) is never formed: its
// product with the start block splits into W V and W^T U; the new block is
// the orthonormalised part of [W V; W^T U] outside span(U) x span(V); the
// Rayleigh-Ritz matrix on the two blocks is, up to a permutation,
// [[0, B], [B^T, 0]] with B = [U, F]^T W [V, G] = [U, F]^T [W V, W G], whose
// SVD gives the Ritz values and vectors.
template <typename T>
void svt_step(Context& cx, StepWs<T>& w, hipStream_t s, int m, int n, const Op<T>& W,
              double eps, int b, T* U, int ldu, T* V, int ldv, double* S, int* rank_dev,
              uint64_t seed)
{
    Timer* tm = &cx.timer;
    const int b2 = 2 * b;
    copy2d<T, T>(m, b, U, ldu, w.UF, b2, s);
    copy2d<T, T>(n, b, V, ldv, w.VG, b2, s);
    // products with the start block: P = W V, Q = W^T U
    op_apply<T>(cx, w, s, W, m, n, false, V, ldv, b, w.PH, b2);
    op_apply<T>(cx, w, s, W, m, n, true, U, ldu, b, w.Qb, b);
    // new block: F = orth(P - U U^T P), G = orth(Q - V V^T Q)
    orth_against<T>(cx, w, s, m, b, U, ldu, w.PH, b2, b, w.UF + b, b2, seed);
    orth_against<T>(cx, w, s, n, b, V, ldv, w.Qb, b, b, w.VG + b, b2, seed);
    // the last product of the pass: H = W G
    op_apply<T>(cx, w, s, W, m, n, false, w.VG + b, b2, b, w.PH + b, b2);
    // B = [U, F]^T [P, H] in FP64
    gemm<T, T, double>(tm, "gemm_ts", true, b2, b2, m, 1.0, w.UF, b2, w.PH, b2, 0.0,
                       (const double*)nullptr, 0, w.Bm, b2, w.partial, w.partial_elems, s);
    {
        const OrthWs<double> ow{w.D1, w.D2, w.Cp, w.Gr, w.Ri, w.chol, w.partial,
                                w.partial_elems, w.flags, w.nflag};
        small_svd_dispatch(cx, s, b2, b, w.Bm, b2, w.UB, w.Sall, w.VB, w.svd, ow, seed);
    }
    // Ritz vectors [U, F] U_B(:, 1:b), [V, G] V_B(:, 1:b)
    gemm<T, double, T>(tm, "gemm_ts", false, m, b, b2, 1.0, w.UF, b2, w.UB, b2, 0.0,
                       (const T*)nullptr, 0, U, ldu, w.partial, w.partial_elems, s);
    gemm<T, double, T>(tm, "gemm_ts", false, n, b, b2, 1.0, w.VG, b2, w.VB, b2, 0.0,
                       (const T*)nullptr, 0, V, ldv, w.partial, w.partial_elems, s);
    copy2d<double, double>(1, b, w.Sall, b2, S, b, s);
    if (rank_dev) count_above(b, S, eps, rank_dev, s);
}

// Cold block: V = orth(random n x b) refined by pow_steps power half-step
// pairs V <- orth(W^T orth(W V)); U = orth(random m x b) drawn independently.
// (A U tied to V by U = orth(W V) would put W V inside span(U) and leave the
// first Lanczos step without new left directions; likewise on the right.)
template <typename T>
void cold_block(Context& cx, StepWs<T>& w, hipStream_t s, int m, int n, const Op<T>& W, int b,
                int pow_steps, uint64_t seed, uint64_t stream_v, T* U, int ldu, T* V, int ldv)
{
    fill_uniform<T>(n, b, w.Qb, b, seed, stream_v, s);
    orth_against<T>(cx, w, s, n, 0, (const T*)nullptr, 0, w.Qb, b, b, V, ldv, seed);
    for (int t = 0; t < pow_steps; ++t) {
        op_apply<T>(cx, w, s, W, m, n, false, V, ldv, b, w.PH, b);
        orth_against<T>(cx, w, s, m, 0, (const T*)nullptr, 0, w.PH, b, b, U, ldu, seed);
        op_apply<T>(cx, w, s, W, m, n, true, U, ldu, b, w.Qb, b);
        orth_against<T>(cx, w, s, n, 0, (const T*)nullptr, 0, w.Qb, b, b, V, ldv, seed);
    }
    fill_uniform<T>(m, b, w.PH, b, seed, stream_v + 1, s);
    orth_against<T>(cx, w, s, m, 0, (const T*)nullptr, 0, w.PH, b, b, U, ldu, seed);
}

// Grow the warm block X (rows x b_old, ld) to b_new columns with random
// columns orthonormalised against it; shrinking keeps the leading columns.
template <typename T>
void grow_block(Context& cx, StepWs<T>& w, hipStream_t s, int rows, int b_old, int b_new, T* X,
                int ldx, uint64_t seed, uint64_t stream_id)
{
    if (b_new <= b_old) return;
    const int c = b_new - b_old;
    fill_uniform<T>(rows, c, w.R, c, seed, stream_id, s);
    orth_against<T>(cx, w, s, rows, b_old, X, ldx, w.R, c, c, X + b_old, ldx, seed);
}

// Block width for a predicted rank sv: rounded up, at most floor(p / 2) and
// b_max. Beyond b_soft the block grows only as far as the previous count of
// values above the threshold (svp) requires, without the prediction's margin.
int block_width(int sv, int svp, const blws_alm_opts& o, int p)
{
    const int want = ((sv + o.b_round - 1) / o.b_round) * o.b_round;
    int b = want;
    if (b > o.b_soft) {
        const int need = ((svp + 1 + o.b_round - 1) / o.b_round) * o.b_round;
        b = need > o.b_soft ? need : o.b_soft;
        if (b > want) b = want;
    }
    if (b > p / 2) b = p / 2;
    if (b > o.b_max) b = o.b_max;
    if (b < 1) b = 1;
    return b;
}

int predict_rank(int svp, int sv, double step_frac, int p)
{
    if (svp < sv) return (svp + 1 < p) ? svp + 1 : p;
    int v = svp + (int)std::lround(step_frac * p);
    return v < p ? v : p;
}

struct Readback {
    double zz;
    double pad;
    int rank;
    int nflag;
    long long nnz;
    int svd_err;
    int pad2;
};

template <typename T>
int rpca_solve_t(Context& cx, hipStream_t s, int m, int n, const T* D, int ldd, double lambda,
                 const blws_alm_opts& o, T* A, int lda, T* E, int lde, blws_solve_info* info,
                 bool ladder = false)
{
    auto t0 = std::chrono::steady_clock::now();
    const int p = m < n ? m : n;
    const int bmax = (p / 2 < o.b_max) ? p / 2 : o.b_max;
    if (lambda <= 0.0) lambda = 1.0 / std::sqrt((double)(m > n ? m : n));
    const size_t mn = (size_t)m * n;

    // workspace layout
    StepWs<T> w;
    unsigned short* Wh = nullptr;  // BF16 copy of W (precision ladder)
    auto layout = [&](Carver& c, T*& Y, T*& Wb, T*& U, T*& V, double*& S, double*& part,
                      double*& scal, int*& rank_dev, long long*& nnz_scr, Readback*& rb) {
        w.carve(c, m, n, bmax);
        Y = c.take<T>(mn);
        Wb = c.take<T>(mn);
        Wh = c.take<unsigned short>(ladder ? mn : 1);
        U = c.take<T>((size_t)m * bmax);
        V = c.take<T>((size_t)n * bmax);
        S = c.take<double>(bmax);
        size_t np = alm_partials(m, n);
        if (np < norms_scratch_elems()) np = norms_scratch_elems();
        part = c.take<double>(np);
        scal = c.take<double>(16);
        rank_dev = c.take<int>(4);
        nnz_scr = c.take<long long>(1024);
        rb = c.take<Readback>(1);
    };
    T *Y, *Wb, *U, *V;
    double *S, *part, *scal;
    int* rank_dev;
    long long* nnz_scr;
    Readback* rb;
    {
        Carver dry(nullptr);
        layout(dry, Y, Wb, U, V, S, part, scal, rank_dev, nnz_scr, rb);
        cx.ensure(dry.off + 256);
    }
    Carver c(cx.ws);
    layout(c, Y, Wb, U, V, S, part, scal, rank_dev, nnz_scr, rb);
    Readback* hrb = (Readback*)cx.host_pinned;
    HIP_TRY(hipMemsetAsync(w.nflag, 0, 4 * sizeof(int), s));

    // ||D||_F and ||D||_inf
    norms<T>(m, n, D, ldd, scal, part, s);
    HIP_TRY(hipMemcpyAsync(hrb, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double dnorm = std::sqrt(((double*)hrb)[0]);
    const double dinf = ((double*)hrb)[1];
    BLWS_REQUIRE(std::isfinite(dnorm) && std::isfinite(dinf), BLWS_ENUMERIC,
                 "rpca_solve: D holds NaN or Inf");
    if (dnorm == 0.0) {
        copy2d<T, T>(m, n, D, ldd, A, lda, s);  // D = 0: A = E = 0
        copy2d<T, T>(m, n, D, ldd, E, lde, s);
        HIP_TRY(hipStreamSynchronize(s));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return BLWS_OK;
    }

    // ||D||_2 by BLWS steps from a cold block (generator stream 3)
    const int bs = bmax < 16 ? bmax : 16;
    const Op<T> opD{D, ldd, nullptr};
    cold_block<T>(cx, w, s, m, n, opD, bs, o.pow_steps, o.seed, 3, U, bs, V, bs);
    double s1 = 0.0, prev = 0.0;
    for (int t = 0; t < o.norm_steps; ++t) {
        svt_step<T>(cx, w, s, m, n, opD, 0.0, bs, U, bs, V, bs, S, nullptr, o.seed);
        HIP_TRY(hipMemcpyAsync(hrb, S, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        s1 = ((double*)hrb)[0];
        BLWS_REQUIRE(std::isfinite(s1), BLWS_ENUMERIC, "rpca_solve: ||D||_2 is not finite");
        if (t > 0 && std::fabs(s1 - prev) <= o.norm_rtol * s1) break;
        prev = s1;
    }

    const double J = s1 > dinf / lambda ? s1 : dinf / lambda;
    double mu = o.mu0_scale / s1;
    const double mu_bar = mu * o.mu_max_factor;
    rpca_init<T>(m, n, D, ldd, J, mu, Y, E, lde, Wb, s);
    if constexpr (std::is_same<T, float>::value)
        if (ladder) to_bf16((long long)mn, Wb, Wh, s);

    int sv = o.sv0, b = 0, svp = 0, it = 0;
    double rel = INFINITY, rel_prev = INFINITY, eps = 0.0;
    const int np = (int)alm_partials(m, n);
    // precision ladder: BF16 products while the residual is at or above
    // ladder_tol (or until it stops decreasing), FP32 afterwards
    bool bf = ladder, last_bf = false, refined = false;
    int iters_bf = 0;
    Op<T> opW{Wb, n, nullptr, nullptr};
    for (it = 1; it <= o.max_iter; ++it) {
        eps = 1.0 / mu;
        opW.Wh = bf ? Wh : nullptr;
        last_bf = bf;
        iters_bf += bf ? 1 : 0;
        const int bn = block_width(sv, svp, o, p);
        if (b == 0) {
            cold_block<T>(cx, w, s, m, n, opW, bn, o.pow_steps, o.seed, 1, U, bmax, V, bmax);
        } else if (bn > b) {
            grow_block<T>(cx, w, s, m, b, bn, U, bmax, o.seed, 1000 + 2 * (uint64_t)it);
            grow_block<T>(cx, w, s, n, b, bn, V, bmax, o.seed, 1000 + 2 * (uint64_t)it + 1);
        }
        b = bn;
        svt_step<T>(cx, w, s, m, n, opW, eps, b, U, bmax, V, bmax, S, rank_dev, o.seed);
        const double mu_next = (o.rho * mu < mu_bar) ? o.rho * mu : mu_bar;
        alm_epilogue<T>(&cx.timer, m, n, b, U, bmax, V, bmax, S, eps, lambda, mu, mu_next, D, ldd,
                        Y, E, lde, Wb, bf ? Wh : nullptr, (T*)nullptr, 0, part, s);
        sum_partials(np, part, &rb->zz, s);
        HIP_TRY(hipMemcpyAsync(&rb->rank, rank_dev, sizeof(int), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(&rb->svd_err, w.nflag + 1, sizeof(int), hipMemcpyDeviceToDevice,
                               s));
        HIP_TRY(hipMemcpyAsync(hrb, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        BLWS_REQUIRE(hrb->svd_err == 0, BLWS_EDEVICE,
                     "small SVD: a device-wide barrier wait timed out");
        svp = hrb->rank;
        BLWS_REQUIRE(std::isfinite(hrb->zz), BLWS_ENUMERIC, "rpca_solve: residual is not finite");
        sv = predict_rank(svp, sv, o.sv_step_frac, p);
        mu = mu_next;
        rel = std::sqrt(hrb->zz) / dnorm;
        if (bf && (rel < o.ladder_tol || (it >= 3 && rel >= rel_prev))) bf = false;
        rel_prev = rel;
        if (rel < o.tol) {
            if (last_bf) {
                // refinement: the last iterate came from BF16 products; one more
                // ALM step with FP32 products (FP64 Rayleigh-Ritz, FP64
                // reconstruction)
                refined = true;
                eps = 1.0 / mu;
                opW.Wh = nullptr;
                svt_step<T>(cx, w, s, m, n, opW, eps, b, U, bmax, V, bmax, S, rank_dev, o.seed);
                const double mu_n2 = (o.rho * mu < mu_bar) ? o.rho * mu : mu_bar;
                alm_epilogue<T>(&cx.timer, m, n, b, U, bmax, V, bmax, S, eps, lambda, mu, mu_n2,
                                D, ldd, Y, E, lde, Wb, nullptr, (T*)nullptr, 0, part, s);
                sum_partials(np, part, &rb->zz, s);
                HIP_TRY(hipMemcpyAsync(&rb->rank, rank_dev, sizeof(int), hipMemcpyDeviceToDevice,
                                       s));
                HIP_TRY(hipMemcpyAsync(hrb, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                svp = hrb->rank;
                rel = std::sqrt(hrb->zz) / dnorm;
                mu = mu_n2;
            }
            break;
        }
    }
    // ALM steps taken (the refinement step included)
    const int steps = (it > o.max_iter ? o.max_iter : it) + (refined ? 1 : 0);
    svt_reconstruct<T>(&cx.timer, m, n, b, U, bmax, V, bmax, S, eps, A, lda, s);
    count_nonzeros<T>(m, n, E, lde, &rb->nnz, nnz_scr, s);
    HIP_TRY(hipMemcpyAsync(&rb->nflag, w.nflag, sizeof(int), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(hrb, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->status = rel < o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
        info->iters = steps;
        info->rank = svp;
        info->b_final = b;
        info->fallbacks = hrb->nflag;
        info->nnz_E = hrb->nnz;
        info->iters_bf16 = iters_bf;
        info->refined = refined ? 1 : 0;
        info->rel_residual = rel;
        info->norm2_D = s1;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rel < o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
}

template <typename T>
void svt_call_t(Context& cx, hipStream_t s, int m, int n, const T* W, int ldw, double eps, int b,
                T* U, int ldu, T* V, int ldv, int warm, double* S, int* rank_dev, T* A, int lda,
                const blws_svt_opts& o)
{
    StepWs<T> w;
    {
        Carver dry(nullptr);
        w.carve(dry, m, n, b);
        cx.ensure(dry.off + 256);
    }
    Carver c(cx.ws);
    w.carve(c, m, n, b);
    HIP_TRY(hipMemsetAsync(w.nflag, 0, 4 * sizeof(int), s));
    const Op<T> op{W, ldw, nullptr};
    if (!warm) cold_block<T>(cx, w, s, m, n, op, b, o.pow_steps, o.seed, 1, U, ldu, V, ldv);
    svt_step<T>(cx, w, s, m, n, op, eps, b, U, ldu, V, ldv, S, rank_dev, o.seed);
    if (A) svt_reconstruct<T>(&cx.timer, m, n, b, U, ldu, V, ldv, S, eps, A, lda, s);
}

// Inexact ALM for matrix completion: W = A + P_Omega(D + Y/mu - A), A = T_{1/mu}(W),
// Y_Omega += mu (d - A_Omega), with A kept as the factors of the last BLWS step
// and W applied as low rank plus sparse (never formed).
template <typename T>
int mc_solve_t(Context& cx, hipStream_t s, int m, int n, int nnz, const int* row_ptr,
               const int* col_idx, const T* d, const blws_alm_opts& o, int r_cap, T* Uout,
               int ldu, double* Sout, T* Vout, int ldv, blws_solve_info* info)
{
    auto t0 = std::chrono::steady_clock::now();
    const int p = m < n ? m : n;
    const int bmax = (p / 2 < o.b_max) ? p / 2 : o.b_max;

    StepWs<T> w;
    T *U, *V, *y, *sv;
    double *S, *coef, *part, *scal;
    int *col_ptr, *csc_row, *csc_perm, *csc_scr, *flag, *rank_dev;
    Readback* rb;
    const size_t np = std::max(mc_partials(m), norms_scratch_elems());
    auto layout = [&](Carver& c) {
        w.carve(c, m, n, bmax);
        U = c.take<T>((size_t)m * bmax);
        V = c.take<T>((size_t)n * bmax);
        S = c.take<double>(bmax);
        y = c.take<T>((size_t)nnz + 1);
        sv = c.take<T>((size_t)nnz + 1);
        coef = c.take<double>((size_t)bmax * bmax);
        part = c.take<double>(np);
        scal = c.take<double>(16);
        col_ptr = c.take<int>((size_t)n + 1);
        csc_row = c.take<int>((size_t)nnz + 1);
        csc_perm = c.take<int>((size_t)nnz + 1);
        csc_scr = c.take<int>(csc_scratch_ints(n, nnz));
        flag = c.take<int>(4);
        rank_dev = c.take<int>(4);
        rb = c.take<Readback>(1);
    };
    {
        Carver dry(nullptr);
        layout(dry);
        cx.ensure(dry.off + 256);
    }
    Carver c(cx.ws);
    layout(c);
    Readback* hrb = (Readback*)cx.host_pinned;
    HIP_TRY(hipMemsetAsync(w.nflag, 0, 4 * sizeof(int), s));

    // the pattern must be valid before any kernel indexes with it
    csr_check(m, n, nnz, row_ptr, col_idx, flag, s);
    HIP_TRY(hipMemcpyAsync(&hrb->rank, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    BLWS_REQUIRE(hrb->rank == 0, BLWS_EINVAL,
                 (hrb->rank & 1) ? "mc_solve: row_ptr is not nondecreasing from 0 to nnz"
                                 : "mc_solve: a column index lies outside [0, n)");
    csc_build(m, n, nnz, row_ptr, col_idx, col_ptr, csc_row, csc_perm, flag + 1, csc_scr, s);

    double dnorm = 0.0;
    if (nnz > 0) {
        norms<T>(1, nnz, d, nnz, scal, part, s);
        HIP_TRY(hipMemcpyAsync(hrb, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        dnorm = std::sqrt(((double*)hrb)[0]);
        BLWS_REQUIRE(std::isfinite(dnorm), BLWS_ENUMERIC, "mc_solve: values hold NaN or Inf");
    }
    if (dnorm == 0.0) {
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        HIP_TRY(hipStreamSynchronize(s));
        return BLWS_OK;
    }

    McOp<T> mo;
    mo.nnz = nnz;
    mo.row_ptr = row_ptr;
    mo.col_idx = col_idx;
    mo.col_ptr = col_ptr;
    mo.csc_row = csc_row;
    mo.csc_perm = csc_perm;
    mo.Ul = U;
    mo.Vl = V;
    mo.ldl = bmax;
    mo.S = S;
    mo.coef = coef;
    const Op<T> op{nullptr, 0, &mo};

    // ||D||_2 of the sampled matrix alone, by BLWS steps from a cold block
    mo.sval = d;
    mo.r = 0;
    const int bs = bmax < 16 ? bmax : 16;
    cold_block<T>(cx, w, s, m, n, op, bs, o.pow_steps, o.seed, 3, U, bs, V, bs);
    double s1 = 0.0, prev = 0.0;
    for (int t = 0; t < o.norm_steps; ++t) {
        svt_step<T>(cx, w, s, m, n, op, 0.0, bs, U, bs, V, bs, S, nullptr, o.seed);
        HIP_TRY(hipMemcpyAsync(hrb, S, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        s1 = ((double*)hrb)[0];
        BLWS_REQUIRE(std::isfinite(s1) && s1 > 0.0, BLWS_ENUMERIC,
                     "mc_solve: ||D||_2 is not finite");
        if (t > 0 && std::fabs(s1 - prev) <= o.norm_rtol * s1) break;
        prev = s1;
    }

    double mu = o.mu0_scale / s1;
    const double mu_bar = mu * o.mu_max_factor;
    mc_init<T>(nnz, d, y, sv, s);
    mo.sval = sv;

    int sv_pred = o.sv0, b = 0, svp = 0, it = 0;
    double rel = INFINITY, eps = 0.0, eps_prev = 0.0;
    const int npart = (int)mc_partials(m);
    for (it = 1; it <= o.max_iter; ++it) {
        eps = 1.0 / mu;
        // the current A = U_r diag(S_r - eps_prev) V_r^T of the last step
        mo.r = svp;
        mo.eps = eps_prev;
        const int bn = block_width(sv_pred, svp, o, p);
        if (b == 0) {
            cold_block<T>(cx, w, s, m, n, op, bn, o.pow_steps, o.seed, 1, U, bmax, V, bmax);
        } else if (bn > b) {
            grow_block<T>(cx, w, s, m, b, bn, U, bmax, o.seed, 1000 + 2 * (uint64_t)it);
            grow_block<T>(cx, w, s, n, b, bn, V, bmax, o.seed, 1000 + 2 * (uint64_t)it + 1);
        }
        b = bn;
        svt_step<T>(cx, w, s, m, n, op, eps, b, U, bmax, V, bmax, S, rank_dev, o.seed);
        const double mu_next = (o.rho * mu < mu_bar) ? o.rho * mu : mu_bar;
        mc_update<T>(&cx.timer, m, nnz, row_ptr, col_idx, d, y, sv, U, bmax, V, bmax, S, eps,
                     rank_dev, b, mu, mu_next, part, s);
        sum_partials(npart, part, &rb->zz, s);
        HIP_TRY(hipMemcpyAsync(&rb->rank, rank_dev, sizeof(int), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(&rb->svd_err, w.nflag + 1, sizeof(int), hipMemcpyDeviceToDevice,
                               s));
        HIP_TRY(hipMemcpyAsync(hrb, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        BLWS_REQUIRE(hrb->svd_err == 0, BLWS_EDEVICE,
                     "small SVD: a device-wide barrier wait timed out");
        svp = hrb->rank;
        BLWS_REQUIRE(std::isfinite(hrb->zz), BLWS_ENUMERIC, "mc_solve: residual is not finite");
        sv_pred = predict_rank(svp, sv_pred, o.sv_step_frac, p);
        mu = mu_next;
        eps_prev = eps;
        rel = std::sqrt(hrb->zz) / dnorm;
        if (rel < o.tol) break;
    }
    if (it > o.max_iter) it = o.max_iter;
    const int rc = svp < r_cap ? svp : r_cap;
    if (rc > 0) {
        copy2d<T, T>(m, rc, U, bmax, Uout, ldu, s);
        copy2d<T, T>(n, rc, V, bmax, Vout, ldv, s);
        theta_out(rc, S, eps, Sout, s);
    }
    HIP_TRY(hipMemcpyAsync(&rb->nflag, w.nflag, sizeof(int), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(hrb, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->status = rel < o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
        info->iters = it;
        info->rank = svp;
        info->b_final = b;
        info->fallbacks = hrb->nflag;
        info->nnz_E = 0;
        info->iters_bf16 = 0;
        info->refined = 0;
        info->rel_residual = rel;
        info->norm2_D = s1;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rel < o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
}

int fail(Context* cx, const BlwsError& e)
{
    if (cx) cx->last_error = e.msg;
    return e.status;
}

}  // namespace
}  // namespace blws

using blws::BlwsError;
using blws::Carver;
using blws::Context;

struct blws_ctx_s {
    Context cx;
};

static thread_local std::string g_noctx_error;

#define ABI_BEGIN(ctx)                                                                    \
    if (!(ctx)) return BLWS_EINVAL;                                                        \
    Context& cx = (ctx)->cx;                                                               \
    try {                                                                                  \
        HIP_TRY(hipSetDevice(cx.device));

#define ABI_END                                                                           \
    }                                                                                      \
    catch (const BlwsError& e) { return blws::fail(&cx, e); }                             \
    catch (const std::exception& e) { return blws::fail(&cx, BlwsError{BLWS_EDEVICE, e.what()}); } \
    catch (...) { return blws::fail(&cx, BlwsError{BLWS_EDEVICE, "unknown error"}); }

extern "C" {

int blws_create(blws_ctx* out, int device)
{
    if (!out) return BLWS_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        g_noctx_error = "no such HIP device";
        return BLWS_EDEVICE;
    }
    blws_ctx c = new (std::nothrow) blws_ctx_s();
    if (!c) return BLWS_ENOMEM;
    c->cx.device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc(&c->cx.host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return BLWS_EDEVICE;
    }
    *out = c;
    return BLWS_OK;
}

int blws_destroy(blws_ctx ctx)
{
    if (!ctx) return BLWS_EINVAL;
    (void)hipSetDevice(ctx->cx.device);
    (void)hipDeviceSynchronize();
    ctx->cx.timer.clear();
    if (ctx->cx.ws) (void)hipFree(ctx->cx.ws);
    if (ctx->cx.host_pinned) (void)hipHostFree(ctx->cx.host_pinned);
    delete ctx;
    return BLWS_OK;
}

const char* blws_status_string(int status)
{
    switch (status) {
        case BLWS_OK: return "ok";
        case BLWS_NOT_CONVERGED: return "not converged";
        case BLWS_EINVAL: return "invalid argument";
        case BLWS_ENOMEM: return "out of device memory";
        case BLWS_EDEVICE: return "device error";
        case BLWS_ENUMERIC: return "NaN or Inf encountered";
        case BLWS_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* blws_last_error(blws_ctx ctx)
{
    if (!ctx) return g_noctx_error.c_str();
    return ctx->cx.last_error.c_str();
}

void blws_default_alm_opts(blws_alm_opts* o)
{
    if (!o) return;
    o->tol = 1e-7;
    o->max_iter = 1000;
    o->rho = 1.5;
    o->mu0_scale = 1.25;
    o->mu_max_factor = 1e7;
    o->sv0 = 10;
    o->sv_step_frac = 0.05;
    o->b_round = 16;
    o->pow_steps = 2;
    o->seed = 20101202ULL;
    o->norm_steps = 8;
    o->norm_rtol = 1e-13;
    o->b_max = 256;
    o->b_soft = 112;
    o->ladder_tol = 1e-3;
}

void blws_default_svt_opts(blws_svt_opts* o)
{
    if (!o) return;
    o->pow_steps = 2;
    o->seed = 20101202ULL;
}

int blws_svt(blws_ctx ctx, void* stream, int prec, int m, int n, const void* W, int ldw,
             double eps, int b, void* U, int ldu, void* V, int ldv, int warm, double* S,
             int* rank_dev, void* A, int lda, const blws_svt_opts* opts)
{
    ABI_BEGIN(ctx)
    const int p = m < n ? m : n;
    BLWS_REQUIRE(m >= 2 && n >= 2 && b >= 1 && 2 * b <= p, BLWS_EINVAL,
                 "blws_svt: need m, n >= 2 and 1 <= b <= min(m, n) / 2");
    BLWS_REQUIRE(W && U && V && S, BLWS_EINVAL, "blws_svt: null W, U, V or S");
    BLWS_REQUIRE(ldw >= n && ldu >= b && ldv >= b && (!A || lda >= n), BLWS_EINVAL,
                 "blws_svt: leading dimension too small");
    BLWS_REQUIRE(std::isfinite(eps) && eps >= 0.0, BLWS_EINVAL, "blws_svt: eps must be >= 0");
    BLWS_REQUIRE(2 * b <= 512, BLWS_EUNSUPPORTED, "blws_svt: b above 256");
    blws_svt_opts o;
    blws_default_svt_opts(&o);
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)stream;
    if (prec == BLWS_FP64)
        blws::svt_call_t<double>(cx, s, m, n, (const double*)W, ldw, eps, b, (double*)U, ldu,
                                 (double*)V, ldv, warm, S, rank_dev, (double*)A, lda, o);
    else if (prec == BLWS_FP32)
        blws::svt_call_t<float>(cx, s, m, n, (const float*)W, ldw, eps, b, (float*)U, ldu,
                                (float*)V, ldv, warm, S, rank_dev, (float*)A, lda, o);
    else
        throw BlwsError{BLWS_EUNSUPPORTED, "blws_svt: precision not supported"};
    return BLWS_OK;
    ABI_END
}

int blws_rpca_solve(blws_ctx ctx, void* stream, int prec, int m, int n, const void* D, int ldd,
                    double lambda, const blws_alm_opts* opts, void* A, int lda, void* E, int lde,
                    blws_solve_info* info)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(m >= 2 && n >= 2, BLWS_EINVAL, "blws_rpca_solve: need m, n >= 2");
    BLWS_REQUIRE(D && A && E, BLWS_EINVAL, "blws_rpca_solve: null D, A or E");
    BLWS_REQUIRE(ldd >= n && lda >= n && lde >= n, BLWS_EINVAL,
                 "blws_rpca_solve: leading dimension too small");
    blws_alm_opts o;
    blws_default_alm_opts(&o);
    if (opts) o = *opts;
    BLWS_REQUIRE(o.tol > 0.0 && o.max_iter >= 1 && o.rho >= 1.0 && o.mu0_scale > 0.0 &&
                     o.mu_max_factor >= 1.0 && o.sv0 >= 1 && o.b_round >= 1 &&
                     o.norm_steps >= 1 && o.sv_step_frac >= 0.0 && o.b_max >= 1 &&
                     o.b_soft >= 1 && o.ladder_tol >= 0.0,
                 BLWS_EINVAL, "blws_rpca_solve: bad options");
    BLWS_REQUIRE(o.b_max <= 256, BLWS_EUNSUPPORTED, "blws_rpca_solve: b_max above 256");
    hipStream_t s = (hipStream_t)stream;
    if (prec == BLWS_FP64)
        return blws::rpca_solve_t<double>(cx, s, m, n, (const double*)D, ldd, lambda, o,
                                          (double*)A, lda, (double*)E, lde, info);
    if (prec == BLWS_FP32 || prec == BLWS_BF16)
        return blws::rpca_solve_t<float>(cx, s, m, n, (const float*)D, ldd, lambda, o,
                                         (float*)A, lda, (float*)E, lde, info,
                                         prec == BLWS_BF16);
    throw BlwsError{BLWS_EUNSUPPORTED, "blws_rpca_solve: precision not supported"};
    ABI_END
}

void blws_default_mc_opts(blws_alm_opts* o)
{
    if (!o) return;
    blws_default_alm_opts(o);
    o->tol = 1e-6;
    o->rho = 1.1;
    o->mu0_scale = 1.0;
}

int blws_mc_solve(blws_ctx ctx, void* stream, int prec, int m, int n, int nnz,
                  const int* row_ptr, const int* col_idx, const void* values,
                  const blws_alm_opts* opts, int r_cap, void* U, int ldu, double* S, void* V,
                  int ldv, blws_solve_info* info)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(m >= 2 && n >= 2 && nnz >= 0, BLWS_EINVAL, "blws_mc_solve: need m, n >= 2");
    BLWS_REQUIRE(row_ptr && U && S && V && (nnz == 0 || (col_idx && values)), BLWS_EINVAL,
                 "blws_mc_solve: null pointer argument");
    BLWS_REQUIRE(r_cap >= 1 && ldu >= r_cap && ldv >= r_cap, BLWS_EINVAL,
                 "blws_mc_solve: need r_cap >= 1 and ldu, ldv >= r_cap");
    blws_alm_opts o;
    blws_default_mc_opts(&o);
    if (opts) o = *opts;
    BLWS_REQUIRE(o.tol > 0.0 && o.max_iter >= 1 && o.rho >= 1.0 && o.mu0_scale > 0.0 &&
                     o.mu_max_factor >= 1.0 && o.sv0 >= 1 && o.b_round >= 1 &&
                     o.norm_steps >= 1 && o.sv_step_frac >= 0.0 && o.b_max >= 1 &&
                     o.b_soft >= 1,
                 BLWS_EINVAL, "blws_mc_solve: bad options");
    BLWS_REQUIRE(o.b_max <= 256, BLWS_EUNSUPPORTED, "blws_mc_solve: b_max above 256");
    hipStream_t s = (hipStream_t)stream;
    if (prec == BLWS_FP64)
        return blws::mc_solve_t<double>(cx, s, m, n, nnz, row_ptr, col_idx,
                                        (const double*)values, o, r_cap, (double*)U, ldu, S,
                                        (double*)V, ldv, info);
    if (prec == BLWS_FP32)
        return blws::mc_solve_t<float>(cx, s, m, n, nnz, row_ptr, col_idx, (const float*)values,
                                       o, r_cap, (float*)U, ldu, S, (float*)V, ldv, info);
    throw BlwsError{BLWS_EUNSUPPORTED, "blws_mc_solve: precision not supported"};
    ABI_END
}

int blws_fill_uniform(blws_ctx ctx, void* stream, int rows, int cols, double* X, int ldx,
                      unsigned long long seed, unsigned long long stream_id)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(rows >= 0 && cols >= 0 && cols <= 4096 && X && ldx >= cols, BLWS_EINVAL,
                 "blws_fill_uniform: bad arguments");
    blws::fill_uniform<double>(rows, cols, X, ldx, seed, stream_id, (hipStream_t)stream);
    return BLWS_OK;
    ABI_END
}

int blws_gemm_f64(blws_ctx ctx, void* stream, int trans_a, int M, int N, int K, double alpha,
                  const double* A, int lda, const double* B, int ldb, double beta, double* C,
                  int ldc)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(M >= 0 && N >= 0 && K >= 0 && A && B && C, BLWS_EINVAL,
                 "blws_gemm_f64: bad arguments");
    BLWS_REQUIRE(ldb >= N && ldc >= N && lda >= (trans_a ? M : K), BLWS_EINVAL,
                 "blws_gemm_f64: leading dimension too small");
    const size_t pe = blws::gemm_partial_elems(M, N, K);
    cx.ensure((pe + 1) * sizeof(double) + 256);
    blws::gemm<double, double, double>(&cx.timer, "gemm_diag", trans_a != 0, M, N, K, alpha, A,
                                       lda, B, ldb, beta, C, ldc, C, ldc, (double*)cx.ws, pe + 1,
                                       (hipStream_t)stream);
    return BLWS_OK;
    ABI_END
}

int blws_gemm_lp(blws_ctx ctx, void* stream, int bf16, int trans_a, int M, int N, int K,
                 const void* A, int lda, const float* B, int ldb, float* C, int ldc)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(M >= 0 && N >= 0 && K >= 1 && A && B && C, BLWS_EINVAL,
                 "blws_gemm_lp: bad arguments");
    BLWS_REQUIRE(ldb >= N && ldc >= N && lda >= (trans_a ? M : K), BLWS_EINVAL,
                 "blws_gemm_lp: leading dimension too small");
    const size_t pe = blws::gemm_lp_partial_elems(M, N, K);
    cx.ensure((pe + 1) * sizeof(float) + 256);
    blws::gemm_lp(&cx.timer, "gemm_diag", bf16 != 0, trans_a != 0, M, N, K, A, lda, B, ldb, C,
                  ldc, (float*)cx.ws, pe + 1, (hipStream_t)stream);
    return BLWS_OK;
    ABI_END
}

int blws_small_svd_f64(blws_ctx ctx, void* stream, int N, const double* B, int ldb, double* UB,
                       double* S, double* VB)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(N >= 1 && N <= 512 && B && UB && S && VB && ldb >= N, BLWS_EINVAL,
                 "blws_small_svd_f64: bad arguments");
    double* svd = nullptr;
    auto layout = [&](Carver& c, blws::OrthWs<double>& w) {
        size_t e1 = blws::small_svd_jacobi_scratch_elems(N), e2 = blws::small_svd_gk_scratch_elems(N);
        svd = c.take<double>(e1 > e2 ? e1 : e2);
        w.T1 = c.take<double>((size_t)N * N);
        w.T2 = c.take<double>((size_t)N * N);
        w.Cp = c.take<double>((size_t)N * N);
        w.Gr = c.take<double>((size_t)N * N);
        w.Ri = c.take<double>((size_t)N * N);
        w.chol = c.take<double>(blws::chol_scratch_elems(N) + 1);
        w.flags = c.take<int>((size_t)N);
        w.nflag = c.take<int>(4);
        size_t pe = blws::gemm_partial_elems(N, N, N);
        w.partial_elems = pe;
        w.partial = c.take<double>(pe + 1);
    };
    blws::OrthWs<double> w;
    {
        Carver dry(nullptr);
        layout(dry, w);
        cx.ensure(dry.off + 256);
    }
    Carver c(cx.ws);
    layout(c, w);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemsetAsync(w.nflag, 0, 4 * sizeof(int), s));
    blws::small_svd_dispatch(cx, s, N, N, B, ldb, UB, S, VB, svd, w, 20101202ULL);
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, w.nflag + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    BLWS_REQUIRE(err == 0, BLWS_EDEVICE, "small SVD: a device-wide barrier wait timed out");
    return BLWS_OK;
    ABI_END
}

int blws_cold_block(blws_ctx ctx, void* stream, int prec, int m, int n, const void* W, int ldw,
                    int b, int pow_steps, unsigned long long seed, unsigned long long stream_v,
                    void* U, int ldu, void* V, int ldv)
{
    ABI_BEGIN(ctx)
    const int p = m < n ? m : n;
    BLWS_REQUIRE(m >= 2 && n >= 2 && b >= 1 && 2 * b <= p && W && U && V, BLWS_EINVAL,
                 "blws_cold_block: bad arguments");
    BLWS_REQUIRE(ldw >= n && ldu >= b && ldv >= b && pow_steps >= 0, BLWS_EINVAL,
                 "blws_cold_block: bad leading dimension or pow_steps");
    hipStream_t s = (hipStream_t)stream;
    if (prec == BLWS_FP64) {
        blws::StepWs<double> w;
        Carver dry(nullptr);
        w.carve(dry, m, n, b);
        cx.ensure(dry.off + 256);
        Carver c(cx.ws);
        w.carve(c, m, n, b);
        const blws::Op<double> op{(const double*)W, ldw, nullptr};
        blws::cold_block<double>(cx, w, s, m, n, op, b, pow_steps, seed, stream_v, (double*)U,
                                 ldu, (double*)V, ldv);
    } else if (prec == BLWS_FP32) {
        blws::StepWs<float> w;
        Carver dry(nullptr);
        w.carve(dry, m, n, b);
        cx.ensure(dry.off + 256);
        Carver c(cx.ws);
        w.carve(c, m, n, b);
        const blws::Op<float> op{(const float*)W, ldw, nullptr};
        blws::cold_block<float>(cx, w, s, m, n, op, b, pow_steps, seed, stream_v, (float*)U,
                                ldu, (float*)V, ldv);
    } else {
        throw BlwsError{BLWS_EUNSUPPORTED, "blws_cold_block: precision not supported"};
    }
    return BLWS_OK;
    ABI_END
}

int blws_timing_enable(blws_ctx ctx, int enable)
{
    ABI_BEGIN(ctx)
    HIP_TRY(hipDeviceSynchronize());
    if (enable) cx.timer.clear();
    cx.timer.on = enable != 0;
    return BLWS_OK;
    ABI_END
}

int blws_timing_get(blws_ctx ctx, const char* name, long long* launches, double* ms,
                    double* flops, double* bytes)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(name, BLWS_EINVAL, "blws_timing_get: null name");
    HIP_TRY(hipDeviceSynchronize());
    long long n = 0;
    double t = 0.0, f = 0.0, by = 0.0;
    auto it = cx.timer.fam.find(name);
    if (it != cx.timer.fam.end()) {
        auto& fam = it->second;
        for (size_t i = 0; i < fam.start.size(); ++i) {
            float e = 0.0f;
            HIP_TRY(hipEventElapsedTime(&e, fam.start[i], fam.stop[i]));
            t += e;
        }
        n = fam.launches;
        f = fam.flops;
        by = fam.bytes;
    }
    if (launches) *launches = n;
    if (ms) *ms = t;
    if (flops) *flops = f;
    if (bytes) *bytes = by;
    return BLWS_OK;
    ABI_END
}

}  // extern "C"
