// Internal: the inexact-ALM solvers (robust PCA and matrix completion, each
// iteration one BLWS step) as resumable jobs.
//
// A job is a sequence of ticks. Each tick queues GPU work on the job's stream
// and ends with an asynchronous copy of a small Readback record into the
// context's pinned host area. Once that copy has landed, advance() runs the
// host logic of the iteration (the rank rule and block width, mu, the
// stopping test, the precision ladder) and queues the next tick. The blocking
// solver calls synchronise between ticks; the request server interleaves the
// ticks of many jobs on their own streams. Both run the same code, so a
// result does not depend on how it was scheduled.
#pragma once

#include <climits>
#include <memory>
#include <string>

#include "lanczos.h"
#include "step.h"

namespace blws {
namespace {

struct Job {
    virtual ~Job() {}
    // Device workspace the job needs (bytes, carving included).
    virtual size_t workspace_bytes() = 0;
    // Carve cx's workspace and queue the first tick.
    virtual void start(Context& cx, hipStream_t s) = 0;
    // The last tick's readback has landed: process it, queue the next tick or
    // the final work (then done = true; the caller waits for the stream).
    virtual void advance(Context& cx, hipStream_t s) = 0;
    bool done = false;
    int status = BLWS_OK;
    blws_solve_info info{};
    // set by a tick that queued work after its readback: the readback is
    // complete once this event is (else once the stream is idle)
    hipEvent_t readback_done = nullptr;
};

// Wait for the work queued on s by polling it: a blocking wait can add a
// thread wake-up to every tick of a solve.
inline void poll_stream(hipStream_t s)
{
    for (;;) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) HIP_TRY(e);
        std::this_thread::yield();
    }
}

inline void poll_event(hipEvent_t e)
{
    for (;;) {
        const hipError_t r = hipEventQuery(e);
        if (r == hipSuccess) return;
        if (r != hipErrorNotReady) HIP_TRY(r);
        std::this_thread::yield();
    }
}

inline void run_blocking(Job& job, Context& cx, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    cx.fix_calls = 0;
    cx.fix_calls_aux = 0;
    cx.ensure(job.workspace_bytes());
    // the solve may queue work ahead of its readbacks: off again on every
    // exit, and nothing of it left running (an error can end the loop early)
    struct Spec {
        Context& cx;
        hipStream_t s;
        Spec(Context& c, hipStream_t st) : cx(c), s(st)
        {
            cx.speculate = !cx.single_stream && !cx.group;
        }
        ~Spec()
        {
            cx.speculate = false;
            (void)hipStreamSynchronize(s);
        }
    } spec(cx, s);
    job.start(cx, s);
    while (!job.done) {
        if (job.readback_done)
            poll_event(job.readback_done);
        else
            poll_stream(s);
        job.readback_done = nullptr;
        job.advance(cx, s);
    }
    HIP_TRY(hipStreamSynchronize(s));
    job.info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

inline double next_mu(const blws_alm_opts& o, double mu, double mu_bar)
{
    return (o.rho * mu < mu_bar) ? o.rho * mu : mu_bar;
}

// ---------------------------------------------------------------------------
// Robust PCA: W = D - E + Y/mu; A = T_{1/mu}(W) by one BLWS step;
// E = S_{lambda/mu}(D - A + Y/mu); Y += mu (D - A - E); mu <- min(rho mu, mu_bar).
// Y0 = D / max(||D||_2, ||D||_inf / lambda), mu0 = mu0_scale / ||D||_2, with
// ||D||_2 from BLWS steps on D from a cold block (generator stream 3).
// ---------------------------------------------------------------------------
template <typename T>
struct RpcaJob : Job {
    // problem
    int m, n, ldd, lda, lde;
    const T* D;
    T *A, *E;
    double lambda;
    blws_alm_opts o;
    bool ladder;
    // derived
    int p, bmax;
    size_t mn;
    // workspace
    StepWs<T> w;
    bool abl = false;  // each SVT by the literal block Lanczos (Sec. 4.1 ablations)
    LanczosWs lw;
    T *Y = nullptr, *Wb = nullptr, *U = nullptr, *V = nullptr;
    unsigned short *Wh = nullptr, *Wl = nullptr;
    double *S = nullptr, *part = nullptr, *scal = nullptr;
    int* rank_dev = nullptr;
    long long* nnz_scr = nullptr;
    Readback* rb = nullptr;
    // state
    enum Phase { NORMS, SPEC, ALM, REFINE, FINISH } phase = NORMS;
    double dnorm = 0.0, s1 = 0.0, prev = 0.0, mu = 0.0, mu_bar = 0.0, mu_next = 0.0;
    double rel = INFINITY, rel_prev = INFINITY, rel_old = INFINITY, eps = 0.0;
    int t = 0, sv = 0, b = 0, svp = 0, it = 0, iters_bf = 0, iters_x3 = 0, np = 0;
    // precision ladder: BF16 products (bf), then split-precision BF16 x 3
    // products (x3, when ladder3_tol > 0), then FP32; last_red: the last
    // iterate came from reduced-precision products
    bool bf = false, x3 = false, x3_on = false, last_red = false, refined = false;
    // the next iteration's products already queued (after the readback) for
    // block width spec_b and products in BF16 (spec_bf) or BF16 x 3 (spec_x3)
    bool spec = false, spec_bf = false, spec_x3 = false;
    int spec_b = 0, prev_b = 0;

    RpcaJob(int m_, int n_, const T* D_, int ldd_, double lambda_, const blws_alm_opts& o_, T* A_,
            int lda_, T* E_, int lde_, bool ladder_)
        : m(m_), n(n_), ldd(ldd_), lda(lda_), lde(lde_), D(D_), A(A_), E(E_), lambda(lambda_),
          o(o_), ladder(ladder_)
    {
        p = m < n ? m : n;
        bmax = (p / 2 < o.b_max) ? p / 2 : o.b_max;
        abl = o.svt_start != LZ_START_SPLIT || o.k_blocks != 2;
        if (abl) {  // k blocks of lz_cols(start, b) columns: at most 1024 and m + n
            const int lim = (m + n < 1024 ? m + n : 1024) / (o.k_blocks * lz_cols(o.svt_start, 1));
            if (bmax > lim) bmax = lim;
        }
        if (lambda <= 0.0) lambda = 1.0 / std::sqrt((double)(m > n ? m : n));
        mn = (size_t)m * n;
        sv = o.sv0;
        bf = ladder;
        x3_on = ladder && o.ladder3_tol > 0.0;
        np = (int)alm_partials(m, n);
    }

    void layout(Carver& c)
    {
        w.carve(c, m, n, bmax);
        if (abl) {
            lw.carve(c, m, n, bmax, o.svt_start, o.k_blocks);
            lw.nflag = w.nflag;  // one breakdown / timeout record for the job
        }
        Y = c.take<T>(mn);
        Wb = c.take<T>(mn);
        Wh = c.take<unsigned short>(ladder ? mn : 1);
        Wl = c.take<unsigned short>(x3_on ? mn : 1);
        U = c.take<T>((size_t)m * bmax);
        V = c.take<T>((size_t)n * bmax);
        S = c.take<double>(bmax);
        size_t npart = alm_partials(m, n);
        if (npart < norms_scratch_elems()) npart = norms_scratch_elems();
        part = c.take<double>(npart);
        scal = c.take<double>(16);
        rank_dev = c.take<int>(4);
        nnz_scr = c.take<long long>(1024);
        rb = c.take<Readback>(1);
    }

    size_t workspace_bytes() override
    {
        Carver dry(nullptr);
        layout(dry);
        return dry.off + 256;
    }

    void start(Context& cx, hipStream_t s) override
    {
        Carver c(cx.ws);
        layout(c);
        zero_bytes(w.nflag, 4 * sizeof(int), s);
        // ||D||_F and ||D||_inf
        norms<T>(m, n, D, ldd, scal, part, s);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               s));
        phase = NORMS;
    }

    void spec_step(Context& cx, hipStream_t s)
    {
        const int bs = bmax < 16 ? bmax : 16;
        const Op<T> opD{D, ldd, nullptr, nullptr};
        svt_step<T>(cx, w, s, m, n, opD, 0.0, bs, U, bs, V, bs, S, nullptr, o.seed);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, S, sizeof(double), hipMemcpyDeviceToHost, s));
    }

    void queue_readback(Context& cx, hipStream_t s)
    {
        iter_readback(np, part, rank_dev, w.nflag + 1, &rb->zz, &rb->rank, &rb->svd_err, s);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
    }

    // one ALM iteration (refine = the FP32 step after a BF16 last iterate)
    void queue_iteration(Context& cx, hipStream_t s, bool refine)
    {
        eps = 1.0 / mu;
        // the products queued ahead are this iteration's when the width and
        // the product precision came out as assumed
        const bool have = spec && !refine && !abl && block_width(sv, o, p) == spec_b &&
                          spec_b == b && bf == spec_bf && (!bf && x3) == spec_x3;
        spec = false;
        if (!refine) {
            const int bn = block_width(sv, o, p);
            const Op<T> opW0{Wb, n, nullptr, nullptr};
            if (b == 0) {
                cold_block<T>(cx, w, s, m, n, opW0, bn, o.pow_steps, o.seed, 1, U, bmax, V, bmax);
            } else if (bn > b) {
                grow_block<T>(cx, w, s, m, b, bn, U, bmax, o.seed, 1000 + 2 * (uint64_t)it);
                grow_block<T>(cx, w, s, n, b, bn, V, bmax, o.seed, 1000 + 2 * (uint64_t)it + 1);
            }
            prev_b = b;
            b = bn;
            last_red = bf || x3;
            iters_bf += bf ? 1 : 0;
            iters_x3 += (!bf && x3) ? 1 : 0;
        }
        const bool use_bf = !refine && bf, use_x3 = !refine && !bf && x3;
        const Op<T> opW{Wb, n, nullptr, (use_bf || use_x3) ? Wh : nullptr,
                        use_x3 ? Wl : nullptr};
        bool lz = false;
        if constexpr (std::is_same<T, double>::value) {
            if (abl) {
                lanczos_step(cx, lw, s, m, n, opW, eps, b, o.svt_start, o.k_blocks, U, bmax, V,
                             bmax, S, rank_dev, o.seed);
                lz = true;
            }
        }
        if (!lz) {
            if (!have) svt_step_products<T>(cx, w, s, m, n, opW, b, U, bmax, V, bmax, o.seed);
            svt_step_finish<T>(cx, w, s, m, n, eps, b, U, bmax, V, bmax, S, rank_dev, o.seed);
        }
        mu_next = next_mu(o, mu, mu_bar);
        // the copies the next iteration's products may read
        alm_epilogue<T>(&cx.timer, m, n, b, U, bmax, V, bmax, S, eps, lambda, mu, mu_next, D, ldd,
                        Y, E, lde, Wb, (use_bf || use_x3) ? Wh : nullptr, (T*)nullptr, 0, part, s,
                        ((use_bf || use_x3) && x3_on) ? Wl : nullptr);
        queue_readback(cx, s);
        // While the host reads this iteration's result, the GPU can already
        // run the next one's products: they read W, U and V as this iteration
        // leaves them and write only the step's scratch, so they are simply
        // queued again when the result changes the width or the precision
        // (or are left unused when the solve stops).
        // Only where it is likely to be used: the width unchanged since the
        // last iteration (the rank rule has settled) and, by the residual's
        // last ratio, neither a stop nor a precision switch expected next.
        const double guess = rel_old > 0.0 && std::isfinite(rel_old) ? rel * (rel / rel_old) : rel;
        const bool likely = b == prev_b && guess >= o.tol && !(bf && guess < o.ladder_tol) &&
                            !(!bf && x3 && guess < o.ladder3_tol);
        if (cx.speculate && !abl && !refine && likely) {
            if (!cx.ev_rb) HIP_TRY(hipEventCreateWithFlags(&cx.ev_rb, hipEventDisableTiming));
            HIP_TRY(hipEventRecord(cx.ev_rb, s));
            readback_done = cx.ev_rb;
            const Op<T> opN{Wb, n, nullptr, (bf || x3) ? Wh : nullptr, (!bf && x3) ? Wl : nullptr};
            svt_step_products<T>(cx, w, s, m, n, opN, b, U, bmax, V, bmax, o.seed);
            spec = true;
            spec_b = b;
            spec_bf = bf;
            spec_x3 = !bf && x3;
        }
    }

    void queue_finish(Context& cx, hipStream_t s)
    {
        svt_reconstruct<T>(&cx.timer, m, n, b, U, bmax, V, bmax, S, eps, A, lda, s);
        count_nonzeros<T>(m, n, E, lde, &rb->nnz, nnz_scr, s);
        HIP_TRY(hipMemcpyAsync(&rb->nflag, w.nflag, sizeof(int), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
        phase = FINISH;
    }

    void read_iteration(const Readback* hrb)
    {
        BLWS_REQUIRE(hrb->svd_err == 0, BLWS_EDEVICE,
                     "small SVD: a device-wide barrier wait timed out");
        svp = hrb->rank;
        BLWS_REQUIRE(std::isfinite(hrb->zz), BLWS_ENUMERIC, "rpca_solve: residual is not finite");
        rel = std::sqrt(hrb->zz) / dnorm;
        mu = mu_next;
    }

    void advance(Context& cx, hipStream_t s) override
    {
        const Readback* hrb = (const Readback*)cx.host_pinned;
        switch (phase) {
            case NORMS: {
                dnorm = std::sqrt(((const double*)hrb)[0]);
                const double dinf = ((const double*)hrb)[1];
                BLWS_REQUIRE(std::isfinite(dnorm) && std::isfinite(dinf), BLWS_ENUMERIC,
                             "rpca_solve: D holds NaN or Inf");
                if (dnorm == 0.0) {  // D = 0: A = E = 0
                    copy2d<T, T>(m, n, D, ldd, A, lda, s);
                    copy2d<T, T>(m, n, D, ldd, E, lde, s);
                    std::memset(&info, 0, sizeof(info));
                    done = true;
                    return;
                }
                dinf_ = dinf;
                const int bs = bmax < 16 ? bmax : 16;
                const Op<T> opD{D, ldd, nullptr, nullptr};
                cold_block<T>(cx, w, s, m, n, opD, bs, o.pow_steps, o.seed, 3, U, bs, V, bs);
                prev = 0.0;
                t = 0;
                spec_step(cx, s);
                phase = SPEC;
                return;
            }
            case SPEC: {
                s1 = ((const double*)hrb)[0];
                BLWS_REQUIRE(std::isfinite(s1), BLWS_ENUMERIC, "rpca_solve: ||D||_2 is not finite");
                const bool conv = t > 0 && std::fabs(s1 - prev) <= o.norm_rtol * s1;
                prev = s1;
                ++t;
                if (!conv && t < o.norm_steps) {
                    spec_step(cx, s);
                    return;
                }
                const double J = s1 > dinf_ / lambda ? s1 : dinf_ / lambda;
                mu = o.mu0_scale / s1;
                mu_bar = mu * o.mu_max_factor;
                rpca_init<T>(m, n, D, ldd, J, mu, Y, E, lde, Wb, s);
                if constexpr (std::is_same<T, float>::value) {
                    if (x3_on)
                        split_bf16x2(m, n, Wb, n, Wh, Wl, s);
                    else if (ladder)
                        to_bf16((long long)mn, Wb, Wh, s);
                }
                it = 1;
                queue_iteration(cx, s, false);
                phase = ALM;
                return;
            }
            case ALM: {
                read_iteration(hrb);
                sv = predict_rank(svp, sv, o.sv_step_frac, p);
                if (x3 && (rel < o.ladder3_tol || rel >= rel_prev)) x3 = false;
                if (bf && (rel < o.ladder_tol || (it >= 3 && rel >= rel_prev))) {
                    bf = false;
                    x3 = x3_on && rel >= o.ladder3_tol;
                }
                rel_old = rel_prev;
                rel_prev = rel;
                if (rel < o.tol) {
                    if (last_red) {
                        // the last iterate came from BF16 or BF16 x 3 products: one
                        // more ALM step with FP32 products (FP64 Rayleigh-Ritz and
                        // reconstruction)
                        refined = true;
                        queue_iteration(cx, s, true);
                        phase = REFINE;
                        return;
                    }
                    queue_finish(cx, s);
                    return;
                }
                if (it >= o.max_iter) {
                    queue_finish(cx, s);
                    return;
                }
                ++it;
                queue_iteration(cx, s, false);
                return;
            }
            case REFINE: {
                read_iteration(hrb);
                queue_finish(cx, s);
                return;
            }
            case FINISH: {
                info.status = rel < o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
                info.iters = it + (refined ? 1 : 0);
                info.rank = svp;
                info.b_final = b;
                info.fallbacks = hrb->nflag;
                info.nnz_E = hrb->nnz;
                info.rel_residual = rel;
                info.norm2_D = s1;
                info.iters_bf16 = iters_bf;
                info.iters_bf16x3 = iters_x3;
                info.refined = refined ? 1 : 0;
                status = info.status;
                done = true;
                return;
            }
        }
    }
    double dinf_ = 0.0;  // ||D||_inf, for Y0
};

// ---------------------------------------------------------------------------
// Matrix completion: W = A + P_Omega(D + Y/mu - A), A = T_{1/mu}(W) by one BLWS
// step, Y_Omega += mu (d - A_Omega), A kept as the factors of the last step
// and W applied as low rank plus sparse (never formed). mu0 = mu0_scale /
// ||P_Omega(M)||_2, Y0 = 0.
// ---------------------------------------------------------------------------
template <typename T>
struct McJob : Job {
    int m, n, nnz, r_cap, ldu, ldv;
    const int *row_ptr, *col_idx;
    const T* d;
    T *Uout, *Vout;
    double* Sout;
    blws_alm_opts o;
    int p, bmax;
    // workspace
    StepWs<T> w;
    T *U = nullptr, *V = nullptr, *y = nullptr, *sv = nullptr;
    double *S = nullptr, *coef = nullptr, *part = nullptr, *scal = nullptr;
    int *col_ptr = nullptr, *csc_row = nullptr, *csc_perm = nullptr, *csc_scr = nullptr;
    int *flag = nullptr, *rank_dev = nullptr;
    Readback* rb = nullptr;
    McOp<T> mo;
    // state
    enum Phase { CHECK, NORMS, SPEC, ALM, FINISH } phase = CHECK;
    double dnorm = 0.0, s1 = 0.0, prev = 0.0, mu = 0.0, mu_bar = 0.0, mu_next = 0.0;
    double rel = INFINITY, eps = 0.0, eps_prev = 0.0;
    int t = 0, sv_pred = 0, b = 0, svp = 0, it = 0, npart = 0;

    McJob(int m_, int n_, int nnz_, const int* rp, const int* ci, const T* d_,
          const blws_alm_opts& o_, int r_cap_, T* U_, int ldu_, double* S_, T* V_, int ldv_)
        : m(m_), n(n_), nnz(nnz_), r_cap(r_cap_), ldu(ldu_), ldv(ldv_), row_ptr(rp), col_idx(ci),
          d(d_), Uout(U_), Vout(V_), Sout(S_), o(o_)
    {
        p = m < n ? m : n;
        bmax = (p / 2 < o.b_max) ? p / 2 : o.b_max;
        sv_pred = o.sv0;
        npart = (int)mc_partials(m);
    }

    void layout(Carver& c)
    {
        const size_t np = std::max(mc_partials(m), norms_scratch_elems());
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
    }

    size_t workspace_bytes() override
    {
        Carver dry(nullptr);
        layout(dry);
        return dry.off + 256;
    }

    void start(Context& cx, hipStream_t s) override
    {
        Carver c(cx.ws);
        layout(c);
        zero_bytes(w.nflag, 4 * sizeof(int), s);
        // the pattern must be valid before any kernel indexes with it
        csr_check(m, n, nnz, row_ptr, col_idx, flag, s);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        phase = CHECK;
    }

    void spec_step(Context& cx, hipStream_t s)
    {
        const int bs = bmax < 16 ? bmax : 16;
        const Op<T> op{nullptr, 0, &mo, nullptr};
        svt_step<T>(cx, w, s, m, n, op, 0.0, bs, U, bs, V, bs, S, nullptr, o.seed);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, S, sizeof(double), hipMemcpyDeviceToHost, s));
    }

    void queue_iteration(Context& cx, hipStream_t s)
    {
        eps = 1.0 / mu;
        // the current A = U_r diag(S_r - eps_prev) V_r^T of the last step
        mo.r = svp;
        mo.eps = eps_prev;
        const Op<T> op{nullptr, 0, &mo, nullptr};
        const int bn = block_width(sv_pred, o, p);
        if (b == 0) {
            cold_block<T>(cx, w, s, m, n, op, bn, o.pow_steps, o.seed, 1, U, bmax, V, bmax);
        } else if (bn > b) {
            grow_block<T>(cx, w, s, m, b, bn, U, bmax, o.seed, 1000 + 2 * (uint64_t)it);
            grow_block<T>(cx, w, s, n, b, bn, V, bmax, o.seed, 1000 + 2 * (uint64_t)it + 1);
        }
        b = bn;
        svt_step<T>(cx, w, s, m, n, op, eps, b, U, bmax, V, bmax, S, rank_dev, o.seed);
        mu_next = next_mu(o, mu, mu_bar);
        mc_update<T>(&cx.timer, m, nnz, row_ptr, col_idx, d, y, sv, U, bmax, V, bmax, S, eps,
                     rank_dev, b, mu, mu_next, INT_MAX, part, s);
        iter_readback(npart, part, rank_dev, w.nflag + 1, &rb->zz, &rb->rank, &rb->svd_err, s);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
    }

    void queue_finish(Context& cx, hipStream_t s)
    {
        const int rc = svp < r_cap ? svp : r_cap;
        if (rc > 0) {
            copy2d<T, T>(m, rc, U, bmax, Uout, ldu, s);
            copy2d<T, T>(n, rc, V, bmax, Vout, ldv, s);
            theta_out(rc, S, eps, Sout, s);
        }
        HIP_TRY(hipMemcpyAsync(&rb->nflag, w.nflag, sizeof(int), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
        phase = FINISH;
    }

    void finish_empty()
    {
        std::memset(&info, 0, sizeof(info));
        done = true;
    }

    void advance(Context& cx, hipStream_t s) override
    {
        const Readback* hrb = (const Readback*)cx.host_pinned;
        switch (phase) {
            case CHECK: {
                const int bad = *(const int*)hrb;
                BLWS_REQUIRE(bad == 0, BLWS_EINVAL,
                             (bad & 1) ? "mc_solve: row_ptr is not nondecreasing from 0 to nnz"
                                       : "mc_solve: a column index lies outside [0, n)");
                csc_build(m, n, nnz, row_ptr, col_idx, col_ptr, csc_row, csc_perm, flag + 1,
                          csc_scr, s);
                if (nnz == 0) {
                    finish_empty();
                    return;
                }
                norms<T>(1, nnz, d, nnz, scal, part, s);
                HIP_TRY(hipMemcpyAsync(cx.host_pinned, scal, 2 * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
                phase = NORMS;
                return;
            }
            case NORMS: {
                dnorm = std::sqrt(((const double*)hrb)[0]);
                BLWS_REQUIRE(std::isfinite(dnorm), BLWS_ENUMERIC, "mc_solve: values hold NaN or Inf");
                if (dnorm == 0.0) {
                    finish_empty();
                    return;
                }
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
                // ||D||_2 of the sampled matrix alone, by BLWS steps from a cold block
                mo.sval = d;
                mo.r = 0;
                const int bs = bmax < 16 ? bmax : 16;
                const Op<T> op{nullptr, 0, &mo, nullptr};
                cold_block<T>(cx, w, s, m, n, op, bs, o.pow_steps, o.seed, 3, U, bs, V, bs);
                prev = 0.0;
                t = 0;
                spec_step(cx, s);
                phase = SPEC;
                return;
            }
            case SPEC: {
                s1 = ((const double*)hrb)[0];
                BLWS_REQUIRE(std::isfinite(s1) && s1 > 0.0, BLWS_ENUMERIC,
                             "mc_solve: ||D||_2 is not finite");
                const bool conv = t > 0 && std::fabs(s1 - prev) <= o.norm_rtol * s1;
                prev = s1;
                ++t;
                if (!conv && t < o.norm_steps) {
                    spec_step(cx, s);
                    return;
                }
                mu = o.mu0_scale / s1;
                mu_bar = mu * o.mu_max_factor;
                mc_init<T>(nnz, d, y, sv, s);
                mo.sval = sv;
                it = 1;
                queue_iteration(cx, s);
                phase = ALM;
                return;
            }
            case ALM: {
                BLWS_REQUIRE(hrb->svd_err == 0, BLWS_EDEVICE,
                             "small SVD: a device-wide barrier wait timed out");
                svp = hrb->rank;
                BLWS_REQUIRE(std::isfinite(hrb->zz), BLWS_ENUMERIC,
                             "mc_solve: residual is not finite");
                sv_pred = predict_rank(svp, sv_pred, o.sv_step_frac, p);
                mu = mu_next;
                eps_prev = eps;
                rel = std::sqrt(hrb->zz) / dnorm;
                if (rel < o.tol || it >= o.max_iter) {
                    queue_finish(cx, s);
                    return;
                }
                ++it;
                queue_iteration(cx, s);
                return;
            }
            case FINISH: {
                info.status = rel < o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
                info.iters = it;
                info.rank = svp;
                info.b_final = b;
                info.fallbacks = hrb->nflag;
                info.nnz_E = 0;
                info.iters_bf16 = 0;
                info.refined = 0;
                info.rel_residual = rel;
                info.norm2_D = s1;
                status = info.status;
                done = true;
                return;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Matrix completion by the SVT algorithm (the MC host of the experiments):
// Y_0 = k0 delta P_Omega(M), k0 = ceil(tau / (delta ||P_Omega(M)||_2)); each
// iteration X_k = T_tau(Y_{k-1}) by BLWS on the purely sparse W = Y_{k-1},
// then Y_k = Y_{k-1} + delta P_Omega(M - X_k), until ||P_Omega(M - X_k)||_F /
// ||P_Omega(M)||_F <= tol. The thresholding asks for s = r_{k-1} + 1 values;
// while all s Ritz values exceed tau it asks for rank_step more, each time a
// BLWS step warm-started from the block just computed (widened when s
// outgrows it). The update kernel skips its writes when the step is to be
// repeated, so one readback per step decides both.
// ---------------------------------------------------------------------------
template <typename T>
struct McSvtJob : Job {
    int m, n, nnz, r_cap, ldu, ldv;
    const int *row_ptr, *col_idx;
    const T* d;
    T *Uout, *Vout;
    double* Sout;
    blws_svt_mc_opts o;
    double tau = 0.0, delta = 0.0;
    int p, bmax;
    StepWs<T> w;
    T *U = nullptr, *V = nullptr, *y = nullptr;
    double *S = nullptr, *coef = nullptr, *part = nullptr, *scal = nullptr;
    int *col_ptr = nullptr, *csc_row = nullptr, *csc_perm = nullptr, *csc_scr = nullptr;
    int *flag = nullptr, *rank_dev = nullptr;
    Readback* rb = nullptr;
    McOp<T> mo;
    enum Phase { CHECK, NORMS, SPEC, STEP, FINISH } phase = CHECK;
    double dnorm = 0.0, s1 = 0.0, prev = 0.0, rel = INFINITY;
    int t = 0, sreq = 1, b = 0, r = 0, it = 0, npart = 0;

    McSvtJob(int m_, int n_, int nnz_, const int* rp, const int* ci, const T* d_,
             const blws_svt_mc_opts& o_, int r_cap_, T* U_, int ldu_, double* S_, T* V_, int ldv_)
        : m(m_), n(n_), nnz(nnz_), r_cap(r_cap_), ldu(ldu_), ldv(ldv_), row_ptr(rp), col_idx(ci),
          d(d_), Uout(U_), Vout(V_), Sout(S_), o(o_)
    {
        p = m < n ? m : n;
        bmax = (p / 2 < o.b_max) ? p / 2 : o.b_max;
        tau = o.tau > 0.0 ? o.tau : 5.0 * std::sqrt((double)m * (double)n);
        delta = o.delta > 0.0 ? o.delta : 1.2 * (double)m * (double)n / (nnz > 0 ? nnz : 1);
        npart = (int)mc_partials(m);
    }

    void layout(Carver& c)
    {
        const size_t np = std::max(mc_partials(m), norms_scratch_elems());
        w.carve(c, m, n, bmax);
        U = c.take<T>((size_t)m * bmax);
        V = c.take<T>((size_t)n * bmax);
        S = c.take<double>(bmax);
        y = c.take<T>((size_t)nnz + 1);
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
    }

    size_t workspace_bytes() override
    {
        Carver dry(nullptr);
        layout(dry);
        return dry.off + 256;
    }

    void start(Context& cx, hipStream_t s) override
    {
        Carver c(cx.ws);
        layout(c);
        zero_bytes(w.nflag, 4 * sizeof(int), s);
        csr_check(m, n, nnz, row_ptr, col_idx, flag, s);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        phase = CHECK;
    }

    void spec_step(Context& cx, hipStream_t s)
    {
        const int bs = bmax < 16 ? bmax : 16;
        const Op<T> op{nullptr, 0, &mo, nullptr};
        svt_step<T>(cx, w, s, m, n, op, 0.0, bs, U, bs, V, bs, S, nullptr, o.seed);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, S, sizeof(double), hipMemcpyDeviceToHost, s));
    }

    // one thresholding of W = Y at the request sreq, and the update (skipped
    // on the device when all sreq values exceed tau and sreq can still grow)
    void queue_step(Context& cx, hipStream_t s)
    {
        const Op<T> op{nullptr, 0, &mo, nullptr};
        int bn = ((sreq + o.b_round - 1) / o.b_round) * o.b_round;
        bn = std::max(1, std::min(bn, bmax));
        if (b == 0) {
            cold_block<T>(cx, w, s, m, n, op, bn, o.pow_steps, o.seed, 1, U, bmax, V, bmax);
        } else if (bn > b) {
            // generator streams by iteration (the repeated requests of one
            // iteration draw from its streams), as in the ALM solvers
            grow_block<T>(cx, w, s, m, b, bn, U, bmax, o.seed, 1000 + 2 * (uint64_t)it);
            grow_block<T>(cx, w, s, n, b, bn, V, bmax, o.seed, 1000 + 2 * (uint64_t)it + 1);
        }
        b = bn;
        svt_step<T>(cx, w, s, m, n, op, tau, b, U, bmax, V, bmax, S, rank_dev, o.seed);
        // the request can still grow unless it reached min(m, n) or the block its cap
        const int need = (sreq >= p || b >= bmax) ? INT_MAX : sreq;
        mc_update<T>(&cx.timer, m, nnz, row_ptr, col_idx, d, y, (T*)nullptr, U, bmax, V, bmax, S,
                     tau, rank_dev, b, delta, delta, need, part, s);
        iter_readback(npart, part, rank_dev, w.nflag + 1, &rb->zz, &rb->rank, &rb->svd_err, s);
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
        last_need = need;
    }
    int last_need = INT_MAX;

    void queue_finish(Context& cx, hipStream_t s)
    {
        const int rc = r < r_cap ? r : r_cap;
        if (rc > 0) {
            copy2d<T, T>(m, rc, U, bmax, Uout, ldu, s);
            copy2d<T, T>(n, rc, V, bmax, Vout, ldv, s);
            theta_out(rc, S, tau, Sout, s);
        }
        HIP_TRY(hipMemcpyAsync(&rb->nflag, w.nflag, sizeof(int), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(cx.host_pinned, rb, sizeof(Readback), hipMemcpyDeviceToHost, s));
        phase = FINISH;
    }

    void advance(Context& cx, hipStream_t s) override
    {
        const Readback* hrb = (const Readback*)cx.host_pinned;
        switch (phase) {
            case CHECK: {
                const int bad = *(const int*)hrb;
                BLWS_REQUIRE(bad == 0, BLWS_EINVAL,
                             (bad & 1) ? "mc_svt_solve: row_ptr is not nondecreasing from 0 to nnz"
                                       : "mc_svt_solve: a column index lies outside [0, n)");
                csc_build(m, n, nnz, row_ptr, col_idx, col_ptr, csc_row, csc_perm, flag + 1,
                          csc_scr, s);
                if (nnz == 0) {
                    std::memset(&info, 0, sizeof(info));
                    done = true;
                    return;
                }
                norms<T>(1, nnz, d, nnz, scal, part, s);
                HIP_TRY(hipMemcpyAsync(cx.host_pinned, scal, 2 * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
                phase = NORMS;
                return;
            }
            case NORMS: {
                dnorm = std::sqrt(((const double*)hrb)[0]);
                BLWS_REQUIRE(std::isfinite(dnorm), BLWS_ENUMERIC,
                             "mc_svt_solve: values hold NaN or Inf");
                if (dnorm == 0.0) {
                    std::memset(&info, 0, sizeof(info));
                    done = true;
                    return;
                }
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
                mo.r = 0;  // W = Y is purely sparse
                mo.sval = d;
                const int bs = bmax < 16 ? bmax : 16;
                const Op<T> op{nullptr, 0, &mo, nullptr};
                cold_block<T>(cx, w, s, m, n, op, bs, o.pow_steps, o.seed, 3, U, bs, V, bs);
                prev = 0.0;
                t = 0;
                spec_step(cx, s);
                phase = SPEC;
                return;
            }
            case SPEC: {
                s1 = ((const double*)hrb)[0];
                BLWS_REQUIRE(std::isfinite(s1) && s1 > 0.0, BLWS_ENUMERIC,
                             "mc_svt_solve: ||P_Omega(M)||_2 is not finite");
                const bool conv = t > 0 && std::fabs(s1 - prev) <= o.norm_rtol * s1;
                prev = s1;
                ++t;
                if (!conv && t < o.norm_steps) {
                    spec_step(cx, s);
                    return;
                }
                const double k0 = std::ceil(tau / (delta * s1));
                scale_copy<T>(nnz, k0 * delta, d, y, s);
                mo.sval = y;
                it = 1;
                sreq = 1;
                queue_step(cx, s);
                phase = STEP;
                return;
            }
            case STEP: {
                BLWS_REQUIRE(hrb->svd_err == 0, BLWS_EDEVICE,
                             "small SVD: a device-wide barrier wait timed out");
                const int svp = hrb->rank;
                if (svp >= last_need) {  // every requested value above tau: ask for more
                    sreq += o.rank_step;
                    queue_step(cx, s);
                    return;
                }
                BLWS_REQUIRE(std::isfinite(hrb->zz), BLWS_ENUMERIC,
                             "mc_svt_solve: residual is not finite");
                r = svp;
                rel = std::sqrt(hrb->zz) / dnorm;
                if (rel <= o.tol || it >= o.max_iter) {
                    queue_finish(cx, s);
                    return;
                }
                ++it;
                sreq = r + 1;
                queue_step(cx, s);
                return;
            }
            case FINISH: {
                info.status = rel <= o.tol ? BLWS_OK : BLWS_NOT_CONVERGED;
                info.iters = it;
                info.rank = r;
                info.b_final = b;
                info.fallbacks = hrb->nflag;
                info.nnz_E = 0;
                info.iters_bf16 = 0;
                info.refined = 0;
                info.rel_residual = rel;
                info.norm2_D = s1;
                status = info.status;
                done = true;
                return;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Argument checks and job construction, shared by the blocking solvers and the
// request server (errors are thrown as BlwsError before any work is queued).
// ---------------------------------------------------------------------------
inline void check_alm_opts(const blws_alm_opts& o, const std::string& who)
{
    BLWS_REQUIRE(o.tol > 0.0 && o.max_iter >= 1 && o.rho >= 1.0 && o.mu0_scale > 0.0 &&
                     o.mu_max_factor >= 1.0 && o.sv0 >= 1 && o.b_round >= 1 &&
                     o.norm_steps >= 1 && o.sv_step_frac >= 0.0 && o.b_max >= 1 &&
                     o.ladder_tol >= 0.0 && o.ladder3_tol >= 0.0,
                 BLWS_EINVAL, who + ": bad options");
    BLWS_REQUIRE(o.b_max <= 512, BLWS_EUNSUPPORTED, who + ": b_max above 512");
    BLWS_REQUIRE(o.svt_start >= LZ_START_SPLIT && o.svt_start <= LZ_START_RIGHT &&
                     o.k_blocks >= 1,
                 BLWS_EINVAL, who + ": bad svt_start or k_blocks");
}

// The Sec. 4.1 ablations (svt_start, k_blocks) run in FP64 robust PCA only.
inline bool alm_opts_ablation(const blws_alm_opts& o)
{
    return o.svt_start != LZ_START_SPLIT || o.k_blocks != 2;
}

inline std::unique_ptr<Job> make_rpca_job(int prec, int m, int n, const void* D, int ldd,
                                          double lambda, const blws_alm_opts* opts, void* A,
                                          int lda, void* E, int lde, const std::string& who)
{
    BLWS_REQUIRE(m >= 2 && n >= 2, BLWS_EINVAL, who + ": need m, n >= 2");
    BLWS_REQUIRE(D && A && E, BLWS_EINVAL, who + ": null D, A or E");
    BLWS_REQUIRE(ldd >= n && lda >= n && lde >= n, BLWS_EINVAL,
                 who + ": leading dimension too small");
    BLWS_REQUIRE(std::isfinite(lambda), BLWS_EINVAL, who + ": lambda must be finite");
    blws_alm_opts o;
    blws_default_alm_opts(&o);
    if (opts) o = *opts;
    check_alm_opts(o, who);
    BLWS_REQUIRE(prec == BLWS_FP64 || !alm_opts_ablation(o), BLWS_EUNSUPPORTED,
                 who + ": svt_start / k_blocks ablations run in FP64 only");
    if (prec == BLWS_FP64)
        return std::unique_ptr<Job>(new RpcaJob<double>(m, n, (const double*)D, ldd, lambda, o,
                                                        (double*)A, lda, (double*)E, lde, false));
    if (prec == BLWS_FP32 || prec == BLWS_BF16)
        return std::unique_ptr<Job>(new RpcaJob<float>(m, n, (const float*)D, ldd, lambda, o,
                                                       (float*)A, lda, (float*)E, lde,
                                                       prec == BLWS_BF16));
    throw BlwsError{BLWS_EUNSUPPORTED, who + ": precision not supported"};
}

inline std::unique_ptr<Job> make_mc_job(int prec, int m, int n, int nnz, const int* row_ptr,
                                        const int* col_idx, const void* values,
                                        const blws_alm_opts* opts, int r_cap, void* U, int ldu,
                                        double* S, void* V, int ldv, const std::string& who)
{
    BLWS_REQUIRE(m >= 2 && n >= 2 && nnz >= 0, BLWS_EINVAL, who + ": need m, n >= 2");
    BLWS_REQUIRE(row_ptr && U && S && V && (nnz == 0 || (col_idx && values)), BLWS_EINVAL,
                 who + ": null pointer argument");
    BLWS_REQUIRE(r_cap >= 1 && ldu >= r_cap && ldv >= r_cap, BLWS_EINVAL,
                 who + ": need r_cap >= 1 and ldu, ldv >= r_cap");
    blws_alm_opts o;
    blws_default_mc_opts(&o);
    if (opts) o = *opts;
    check_alm_opts(o, who);
    BLWS_REQUIRE(!alm_opts_ablation(o), BLWS_EUNSUPPORTED,
                 who + ": svt_start / k_blocks ablations run in robust PCA only");
    if (prec == BLWS_FP64)
        return std::unique_ptr<Job>(new McJob<double>(m, n, nnz, row_ptr, col_idx,
                                                      (const double*)values, o, r_cap, (double*)U,
                                                      ldu, S, (double*)V, ldv));
    if (prec == BLWS_FP32)
        return std::unique_ptr<Job>(new McJob<float>(m, n, nnz, row_ptr, col_idx,
                                                     (const float*)values, o, r_cap, (float*)U,
                                                     ldu, S, (float*)V, ldv));
    throw BlwsError{BLWS_EUNSUPPORTED, who + ": precision not supported"};
}

inline std::unique_ptr<Job> make_mc_svt_job(int prec, int m, int n, int nnz, const int* row_ptr,
                                            const int* col_idx, const void* values,
                                            const blws_svt_mc_opts* opts, int r_cap, void* U,
                                            int ldu, double* S, void* V, int ldv,
                                            const std::string& who)
{
    BLWS_REQUIRE(m >= 2 && n >= 2 && nnz >= 0, BLWS_EINVAL, who + ": need m, n >= 2");
    BLWS_REQUIRE(row_ptr && U && S && V && (nnz == 0 || (col_idx && values)), BLWS_EINVAL,
                 who + ": null pointer argument");
    BLWS_REQUIRE(r_cap >= 1 && ldu >= r_cap && ldv >= r_cap, BLWS_EINVAL,
                 who + ": need r_cap >= 1 and ldu, ldv >= r_cap");
    blws_svt_mc_opts o;
    blws_default_svt_mc_opts(&o);
    if (opts) o = *opts;
    BLWS_REQUIRE(std::isfinite(o.tau) && std::isfinite(o.delta) && o.tol > 0.0 &&
                     o.max_iter >= 1 && o.rank_step >= 1 && o.b_round >= 1 && o.b_max >= 1 &&
                     o.pow_steps >= 0 && o.norm_steps >= 1,
                 BLWS_EINVAL, who + ": bad options");
    BLWS_REQUIRE(o.b_max <= 512, BLWS_EUNSUPPORTED, who + ": b_max above 512");
    if (prec == BLWS_FP64)
        return std::unique_ptr<Job>(new McSvtJob<double>(m, n, nnz, row_ptr, col_idx,
                                                         (const double*)values, o, r_cap,
                                                         (double*)U, ldu, S, (double*)V, ldv));
    if (prec == BLWS_FP32)
        return std::unique_ptr<Job>(new McSvtJob<float>(m, n, nnz, row_ptr, col_idx,
                                                        (const float*)values, o, r_cap, (float*)U,
                                                        ldu, S, (float*)V, ldv));
    throw BlwsError{BLWS_EUNSUPPORTED, who + ": precision not supported"};
}

// One BLWS SVT call (asynchronous): cold block unless warm, the step, and the
// optional reconstruction of A.
template <typename T>
void svt_call_t(Context& cx, hipStream_t s, int m, int n, const T* W, int ldw, double eps, int b,
                T* U, int ldu, T* V, int ldv, int warm, double* S, int* rank_dev, T* A, int lda,
                const blws_svt_opts& o, bool x3 = false)
{
    StepWs<T> w;
    unsigned short *Wh = nullptr, *Wl = nullptr;
    const size_t wcopy = x3 ? (size_t)m * ldw : 0;  // BF16 x 3: the two halves of W
    {
        Carver dry(nullptr);
        w.carve(dry, m, n, b);
        dry.take<unsigned short>(wcopy);
        dry.take<unsigned short>(wcopy);
        cx.ensure(dry.off + 256);
    }
    Carver c(cx.ws);
    w.carve(c, m, n, b);
    if (x3) {
        Wh = c.take<unsigned short>(wcopy);
        Wl = c.take<unsigned short>(wcopy);
        if constexpr (std::is_same<T, float>::value) split_bf16x2(m, n, W, ldw, Wh, Wl, s);
    }
    zero_bytes(w.nflag, 4 * sizeof(int), s);
    const Op<T> op{W, ldw, nullptr, Wh, Wl};
    if (!warm) cold_block<T>(cx, w, s, m, n, op, b, o.pow_steps, o.seed, 1, U, ldu, V, ldv);
    svt_step<T>(cx, w, s, m, n, op, eps, b, U, ldu, V, ldv, S, rank_dev, o.seed);
    if (A) svt_reconstruct<T>(&cx.timer, m, n, b, U, ldu, V, ldv, S, eps, A, lda, s);
}

}  // namespace
}  // namespace blws
