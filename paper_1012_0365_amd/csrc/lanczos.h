// The start-block ablations of Sec. 4.1 on the GPU: one SVT step by
// Algorithms 2 and 3 taken literally on the augmented matrix
// W~ = [[0, W], [W^T, 0]] (Theorem 1), from one of four start blocks and with
// k blocks, FP64.
//
//   BLWS_START_SPLIT  X_1 = blockdiag(U, V)     2b columns (the default step's
//                                               reading, here without its
//                                               zero-block skipping)
//   BLWS_START_AUG    X_1 = (U; V) / sqrt(2)    b columns (the start written
//                                               for BLWS in Sec. 4.1)
//   BLWS_START_LEFT   X_1 = (U; 0)              b columns (the standard
//   BLWS_START_RIGHT  X_1 = (0; V)              half-information starts)
//
// W~ is never formed: a block X = (X_top; X_bot) of N = m + n rows maps to
// W~ X = (W X_bot; W^T X_top), and M_l = X_l^T W~ X_l = S + S^T with
// S = X_top^T (W X_bot), so the last block needs only W X_bot (2k - 1 products
// in all). The start block is orthonormalised (Algorithm 2 takes an
// orthogonal X_1); each new block X_{l+1} is orthonormalised against all
// earlier blocks (block reorthogonalisation, which changes nothing in exact
// arithmetic) and B_l = X_{l+1}^T R_l. Algorithm 3: eigenpairs of the block
// tridiagonal T_k from the SVD of T_k + c I (positive semidefinite for c at
// least the spectral radius); the top b Ritz vectors Y = Q_k Z(:, 1:b) give
// U = sqrt(2) Y_top and V = sqrt(2) Y_bot (an eigenvector of W~ for
// sigma > 0 is (u; v) / sqrt(2)) and S the top b Ritz values.
#pragma once

#include "step.h"

namespace blws {
namespace {

constexpr int LZ_START_SPLIT = 0, LZ_START_AUG = 1, LZ_START_LEFT = 2, LZ_START_RIGHT = 3;

inline int lz_cols(int start, int b) { return start == LZ_START_SPLIT ? 2 * b : b; }

// Scratch of one literal block-Lanczos step (FP64).
struct LanczosWs {
    double *Q, *WX, *R, *Sm, *Ms, *Bs, *Bt, *Tm, *shift, *UB, *VB, *Sall, *svd;
    double *T1, *T2, *Cp, *Gr, *Ri, *chol, *partial, *D1, *D2, *xv;
    int *flags, *nflag;
    size_t partial_elems;

    void carve(Carver& cv, int m, int n, int b, int start, int k)
    {
        const int N = m + n, c = lz_cols(start, b), K = k * c, w = ORTH_CHUNK;
        Q = cv.take<double>((size_t)N * K);
        WX = cv.take<double>((size_t)N * c);
        R = cv.take<double>((size_t)N * c);
        Sm = cv.take<double>((size_t)c * c);
        Ms = cv.take<double>((size_t)k * c * c);
        Bs = cv.take<double>((size_t)k * c * c);
        Bt = cv.take<double>((size_t)c * c);
        Tm = cv.take<double>((size_t)K * K);
        shift = cv.take<double>(2);
        UB = cv.take<double>((size_t)K * K);
        VB = cv.take<double>((size_t)K * K);
        Sall = cv.take<double>((size_t)K);
        svd = cv.take<double>(small_svd_gk_scratch_elems(K));
        T1 = cv.take<double>((size_t)N * w);
        T2 = cv.take<double>((size_t)N * w);
        Cp = cv.take<double>((size_t)K * w);
        Gr = cv.take<double>((size_t)w * w);
        Ri = cv.take<double>((size_t)w * w);
        chol = cv.take<double>(chol_scratch_elems(w) + 1);
        D1 = cv.take<double>((size_t)K * w);
        D2 = cv.take<double>((size_t)K * w);
        xv = cv.take<double>((size_t)N);
        flags = cv.take<int>((size_t)2 * w);
        nflag = cv.take<int>(4);
        size_t pe = 0;
        const int shapes[][3] = {{m, c, n}, {n, c, m}, {c, c, m}, {N, c, c}, {c, c, N},
                                 {K, w, N}, {N, w, K}, {w, w, N}, {N, w, w}, {K, w, K},
                                 {w, w, K}, {K, w, w}, {m, b, K}, {n, b, K}};
        for (auto& sh : shapes) {
            const size_t e = gemm_partial_elems(sh[0], sh[1], sh[2]);
            if (e > pe) pe = e;
        }
        partial_elems = pe;
        partial = cv.take<double>(pe + 1);
    }
};

inline size_t lanczos_ws_bytes(int m, int n, int b, int start, int k)
{
    Carver dry(nullptr);
    LanczosWs w;
    w.carve(dry, m, n, b, start, k);
    return dry.off + 256;
}

// One SVT step by the literal procedure (see above) on the dense W (FP64).
// U (m x b, ldu) and V (n x b, ldv): the previous subspaces on entry, the Ritz
// vectors sqrt(2) Y_top, sqrt(2) Y_bot on exit; S (b) the top b Ritz values;
// rank_dev (may be null) = #{S_i > eps}. Requires k * columns(start) <= 1024
// and <= m + n.
inline void lanczos_step(Context& cx, LanczosWs& w, hipStream_t s, int m, int n,
                         const Op<double>& W, double eps, int b, int start, int k, double* U,
                         int ldu, double* V, int ldv, double* S, int* rank_dev, uint64_t seed)
{
    Timer* tm = &cx.timer;
    const int N = m + n, c = lz_cols(start, b), K = k * c;
    const OrthWs<double> ow{w.T1, w.T2, w.Cp, w.Gr, w.Ri, w.chol, w.partial, w.partial_elems,
                            w.flags, w.nflag, w.xv};
    StepWs<double> pw{};  // op_apply reads only the split-K partials
    pw.partial = w.partial;
    pw.partial_elems = w.partial_elems;
    // the start block X_1 in the first c columns of Q (N x K, ld K): rows
    // 0 .. m-1 the top half, rows m .. N-1 the bottom half
    zero_bytes(w.Q, sizeof(double) * (size_t)N * K, s);
    if (start == LZ_START_SPLIT) {
        copy2d<double, double>(m, b, U, ldu, w.Q, K, s);
        copy2d<double, double>(n, b, V, ldv, w.Q + (size_t)m * K + b, K, s);
    } else {
        // (U; V) / sqrt(2) spans what (U; V) spans: the orthonormalisation
        // below makes the scale moot
        if (start != LZ_START_RIGHT) copy2d<double, double>(m, b, U, ldu, w.Q, K, s);
        if (start != LZ_START_LEFT) copy2d<double, double>(n, b, V, ldv, w.Q + (size_t)m * K, K, s);
    }
    orth_against<double>(cx, ow, s, N, 0, nullptr, 0, w.Q, K, c, w.Q, K, seed);
    for (int l = 0; l < k; ++l) {
        double* X = w.Q + (size_t)l * c;  // X_l: top rows X, bottom rows X + m K
        double* Ml = w.Ms + (size_t)l * c * c;
        // W~ X_l = (W X_bot; W^T X_top); the last block needs the top half only
        op_apply<double>(cx, pw, s, W, m, n, false, X + (size_t)m * K, K, c, w.WX, c);
        if (l + 1 < k)
            op_apply<double>(cx, pw, s, W, m, n, true, X, K, c, w.WX + (size_t)m * c, c);
        // M_l = S + S^T, S = X_top^T (W X_bot)
        gemm<double, double, double>(tm, "gemm_ts", true, c, c, m, 1.0, X, K, w.WX, c, 0.0,
                                     (const double*)nullptr, 0, w.Sm, c, w.partial,
                                     w.partial_elems, s);
        lanczos_sym(c, w.Sm, Ml, s);
        if (l + 1 == k) break;
        // R_l = W~ X_l - X_l M_l - X_{l-1} B_{l-1}^T
        gemm<double, double, double>(tm, "gemm_ts", false, N, c, c, -1.0, X, K, Ml, c, 1.0, w.WX,
                                     c, w.R, c, w.partial, w.partial_elems, s);
        if (l > 0)
            gemm<double, double, double>(tm, "gemm_ts", false, N, c, c, -1.0, X - c, K, w.Bt, c,
                                         1.0, w.R, c, w.R, c, w.partial, w.partial_elems, s);
        // (X_{l+1}, B_l) = qr(R_l), X_{l+1} orthogonal to X_1 .. X_l
        double* Xn = X + c;
        orth_against<double>(cx, ow, s, N, (l + 1) * c, w.Q, K, w.R, c, c, Xn, K, seed);
        double* Bl = w.Bs + (size_t)l * c * c;
        gemm<double, double, double>(tm, "gemm_ts", true, c, c, N, 1.0, Xn, K, w.R, c, 0.0,
                                     (const double*)nullptr, 0, Bl, c, w.partial, w.partial_elems,
                                     s);
        lanczos_transpose(c, Bl, w.Bt, s);
    }
    // Algorithm 3: eigenpairs of T_k via the SVD of T_k + shift I
    lanczos_assemble(k, c, w.Ms, w.Bs, w.shift, w.Tm, s);
    {
        const OrthWs<double> sw{w.D1, w.D2, w.Cp, w.Gr, w.Ri, w.chol, w.partial, w.partial_elems,
                                w.flags, w.nflag, w.xv};
        small_svd_dispatch(cx, s, K, b, w.Tm, K, w.UB, w.Sall, w.VB, w.svd, sw, seed);
    }
    lanczos_eigvals(b, w.Sall, w.shift, S, s);
    // Ritz vectors Y = Q_k Z(:, 1:b): U = sqrt(2) Y_top, V = sqrt(2) Y_bot
    const double r2 = std::sqrt(2.0);
    gemm<double, double, double>(tm, "gemm_ts", false, m, b, K, r2, w.Q, K, w.UB, K, 0.0,
                                 (const double*)nullptr, 0, U, ldu, w.partial, w.partial_elems, s);
    gemm<double, double, double>(tm, "gemm_ts", false, n, b, K, r2, w.Q + (size_t)m * K, K, w.UB,
                                 K, 0.0, (const double*)nullptr, 0, V, ldv, w.partial,
                                 w.partial_elems, s);
    if (rank_dev) count_above(b, S, eps, rank_dev, s);
}

}  // namespace
}  // namespace blws
