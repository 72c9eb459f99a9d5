// Internal: the BLWS step and its building blocks on the host side (workspace
// carving, orthonormalisation, the projected SVD, the operator products, the
// step itself, cold and grown blocks, the block-width rule). Shared by the
// solvers (jobs.h), the C ABI (engine.hip) and the request server
// (server.hip).
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <exception>
#include <functional>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "blws_common.h"

namespace blws {

// ---------------------------------------------------------------------------
// Timing: HIP events per launch, grouped by kernel family.
// ---------------------------------------------------------------------------
struct Timer {
    bool on = false;
    std::mutex mu;  // launches are recorded from two host threads
    struct Family {
        std::vector<hipEvent_t> start, stop;
        double flops = 0.0, bytes = 0.0;
        long long launches = 0;
    };
    std::map<std::string, Family> fam;
    std::set<std::string> only;    // families to record (empty: all)
    std::vector<hipEvent_t> pool;  // events of earlier recordings, reused
    bool wants(const char* family) const { return only.empty() || only.count(family) != 0; }
    hipEvent_t take()
    {
        if (pool.empty()) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    void clear()
    {
        for (auto& kv : fam) {
            pool.insert(pool.end(), kv.second.start.begin(), kv.second.start.end());
            pool.insert(pool.end(), kv.second.stop.begin(), kv.second.stop.end());
        }
        fam.clear();
    }
    void release()
    {
        clear();
        for (auto e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

namespace {

constexpr double CHOL_ETA = 1e-13;  // scaled pivot below which a column is dependent

// Bound on ||G - I||_2 (taken as n max|G_ij - I_ij|) below which the Cholesky
// inverse is replaced by (3 I - G) / 2, whose orthonormality error
// 3 ||G - I||^2 / 4 then stays below the storage precision's rounding: 1e-8 in
// FP64, 2.5e-4 in FP32 (4.7e-8; columns stored in FP32 are orthonormal to
// about 1e-7 at best, so an FP64-sized test would never pass there).
template <typename T>
constexpr double chol_ni_tol()
{
    return std::is_same<T, double>::value ? 1e-8 : 2.5e-4;
}

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

struct Context;

// A host thread that queues one task at a time (the second stream's half of
// a step), so that the launches of both halves are issued concurrently.
// Second host thread of a context: it queues the second stream's half of a
// step. A posted task is picked up by polling while tasks keep coming (for
// up to IDLE_SPIN after the last one; the tasks of a solve come an ALM
// iteration apart) and through the condition variable after that, so that
// the hand-over costs no thread wake-up in the middle of a solve. wait()
// polls likewise for up to WAIT_SPIN.
struct AuxWorker {
    static constexpr std::chrono::microseconds IDLE_SPIN{5000}, WAIT_SPIN{5000};
    std::thread th;
    std::mutex m;
    std::condition_variable cv;
    std::function<void()> task;
    std::atomic<int> state{0};  // 0 idle, 1 posted, 2 running
    bool stop = false;
    std::exception_ptr err;

    void start(int device)
    {
        th = std::thread([this, device] {
            (void)hipSetDevice(device);
            for (;;) {
                const auto t0 = std::chrono::steady_clock::now();
                while (state.load(std::memory_order_acquire) != 1 &&
                       std::chrono::steady_clock::now() - t0 < IDLE_SPIN)
                    std::this_thread::yield();
                std::function<void()> t;
                {
                    std::unique_lock<std::mutex> lk(m);
                    cv.wait(lk, [&] { return state.load(std::memory_order_acquire) == 1 || stop; });
                    if (state.load(std::memory_order_acquire) != 1) return;
                    t = std::move(task);
                    state.store(2, std::memory_order_release);
                }
                std::exception_ptr e;
                try {
                    t();
                } catch (...) {
                    e = std::current_exception();
                }
                {
                    std::lock_guard<std::mutex> g(m);
                    err = e;
                    state.store(0, std::memory_order_release);
                }
                cv.notify_all();
            }
        });
    }
    void run(std::function<void()> f)
    {
        {
            std::lock_guard<std::mutex> g(m);
            task = std::move(f);
            err = nullptr;
            state.store(1, std::memory_order_release);
        }
        cv.notify_all();
    }
    // wait for the task; rethrow what it threw
    void wait()
    {
        const auto t0 = std::chrono::steady_clock::now();
        while (state.load(std::memory_order_acquire) != 0 &&
               std::chrono::steady_clock::now() - t0 < WAIT_SPIN)
            std::this_thread::yield();
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return state.load(std::memory_order_acquire) == 0; });
        if (err) {
            std::exception_ptr e = err;
            err = nullptr;
            std::rethrow_exception(e);
        }
    }
    void shutdown()
    {
        {
            std::lock_guard<std::mutex> g(m);
            stop = true;
        }
        cv.notify_all();
        if (th.joinable()) th.join();
    }
};

// Rendezvous for the W-products of several solves stepping at the same time
// (the request server): a solve hands over its products and returns once a
// grouped launch holding them has been queued after the work already on the
// given streams, with those streams made to wait for it.
struct ProductGroup {
    virtual ~ProductGroup() {}
    virtual void submit(const WProduct* prods, const hipStream_t* streams, int n) = 0;
};

struct Context {
    ProductGroup* group = nullptr;  // set by the request server while a solve steps
    // all of a step's work on the caller's stream, queued by the calling thread
    // (no second stream, events or helper thread are created or used)
    bool single_stream = false;
    // device address of the library's static scratch on this context's device
    // (blws_svt_noalloc), looked up when the context is created
    void* static_scratch = nullptr;
    int device = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* host_pinned = nullptr;  // small readback area
    std::string last_error;
    Timer timer;
    uint64_t fix_calls = 0;      // stream ids for breakdown replacement draws
    uint64_t fix_calls_aux = 0;  // the same for the work on the second stream
    // second stream for independent halves of a step (default priority),
    // forked from and joined back into the caller's stream by events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::unique_ptr<AuxWorker> worker;  // issues the second stream's launches
    // a blocking solve may queue the next iteration's products before the
    // host has read the current one's result (see RpcaJob); ev_rb marks the
    // end of the readback it then waits for
    bool speculate = false;
    hipEvent_t ev_rb = nullptr;

    void ensure_aux()
    {
        if (aux) return;
        HIP_TRY(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
        worker.reset(new AuxWorker());
        worker->start(device);
    }
    void release_aux()
    {
        if (worker) {
            worker->shutdown();
            worker.reset();
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (ev_rb) (void)hipEventDestroy(ev_rb);
        if (aux) (void)hipStreamDestroy(aux);
        aux = nullptr;
        ev_fork = ev_join = ev_rb = nullptr;
    }
    // cx.aux waits for the work queued so far on s
    void fork(hipStream_t s)
    {
        ensure_aux();
        HIP_TRY(hipEventRecord(ev_fork, s));
        HIP_TRY(hipStreamWaitEvent(aux, ev_fork, 0));
    }
    // s waits for the work queued so far on cx.aux
    void join(hipStream_t s)
    {
        HIP_TRY(hipEventRecord(ev_join, aux));
        HIP_TRY(hipStreamWaitEvent(s, ev_join, 0));
    }

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
    double *Cp, *Gr, *Ri, *Bm, *UB, *VB, *Sall, *svd, *chol, *partial, *D1, *D2, *xv;
    int *flags, *nflag;
    size_t partial_elems;
    // the same orthonormalisation scratch and split-K partials again, for work
    // on the second stream (the breakdown counter nflag is shared: atomic)
    T *T1b, *T2b;
    double *Cpb, *Grb, *Rib, *cholb, *partialb, *xvb;
    int* flagsb;

    // second_set = false leaves out the scratch of the second stream (the
    // single-stream form of the step never uses it)
    void carve(Carver& c, int m, int n, int b, bool second_set = true)
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
        svd = c.take<double>(small_svd_gk_scratch_elems(b2));
        D1 = c.take<double>((size_t)b2 * b);
        D2 = c.take<double>((size_t)b2 * b);
        chol = c.take<double>(chol_scratch_elems(b) + 1);
        xv = c.take<double>((size_t)mx);
        flags = c.take<int>((size_t)2 * b);
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
        if (!second_set) {
            T1b = T2b = nullptr;
            Cpb = Grb = Rib = cholb = partialb = xvb = nullptr;
            flagsb = nullptr;
            return;
        }
        T1b = c.take<T>((size_t)mx * b);
        T2b = c.take<T>((size_t)mx * b);
        Cpb = c.take<double>((size_t)b * b);
        Grb = c.take<double>((size_t)b * b);
        Rib = c.take<double>((size_t)b * b);
        cholb = c.take<double>(chol_scratch_elems(b) + 1);
        xvb = c.take<double>((size_t)mx);
        flagsb = c.take<int>((size_t)2 * b);
        partialb = c.take<double>(pe + 1);
    }

    // this scratch with the second set in place of the first (for the
    // second stream)
    StepWs aux_view() const
    {
        StepWs v = *this;
        v.T1 = T1b;
        v.T2 = T2b;
        v.Cp = Cpb;
        v.Gr = Grb;
        v.Ri = Rib;
        v.chol = cholb;
        v.flags = flagsb;
        v.xv = xvb;
        v.partial = partialb;
        return v;
    }
};

// Scratch of one orthonormalisation: T1, T2 (rows x 128), Cp (b x 128, b the
// widest block projected against), Gr, Ri (128 x 128), the Cholesky scratch,
// the breakdown flags of the two passes (2 x 128; nflag[0] counts them), the
// split-K partials and one column of rows doubles for the fallback pass.
template <typename T>
struct OrthWs {
    T *T1, *T2;
    double *Cp, *Gr, *Ri, *chol, *partial;
    size_t partial_elems;
    int *flags, *nflag;
    double* xv;
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
// A column either pass finds dependent comes out of the passes as zero and is
// re-formed from the vectors by the fallback pass (orth_fallback): classical
// Gram-Schmidt with reorthogonalisation of the column as the first pass saw
// it (kept in T1), or of counter-based draws where that column lies in the
// span to rounding.
template <typename T>
void orth_chunk(Context& cx, const OrthWs<T>& w, hipStream_t s, int rows, int nx,
                const T* const* X, const int* ldx, const int* bx, const T* In, int ldin, int c,
                T* Out, int ldout, uint64_t seed)
{
    Timer* tm = &cx.timer;
    project_out<T>(cx, w, s, rows, nx, X, ldx, bx, In, ldin, w.T1, c);
    // pass 1: T2 = T1 R^{-1} (a dependent column has a zero column in R^{-1})
    gemm<T, T, double>(tm, "gemm_ts", true, c, c, rows, 1.0, w.T1, c, w.T1, c, 0.0,
                       (const double*)nullptr, 0, w.Gr, c, w.partial, w.partial_elems, s);
    chol_inv(tm, c, w.Gr, c, w.Ri, w.flags, w.nflag, CHOL_ETA, chol_ni_tol<T>(), w.chol, s);
    gemm_apply_flagged<T>(tm, rows, c, w.T1, c, w.Ri, c, w.T2, c, (const int*)nullptr, 0, 0, s);
    if (nx > 0) project_out<T>(cx, w, s, rows, nx, X, ldx, bx, w.T2, c, w.T2, c);
    // pass 2 (its flags after the first pass's; its count goes to a spare slot)
    gemm<T, T, double>(tm, "gemm_ts", true, c, c, rows, 1.0, w.T2, c, w.T2, c, 0.0,
                       (const double*)nullptr, 0, w.Gr, c, w.partial, w.partial_elems, s);
    chol_inv(tm, c, w.Gr, c, w.Ri, w.flags + c, w.nflag + 3, CHOL_ETA, chol_ni_tol<T>(), w.chol,
             s);
    gemm<T, double, T>(tm, "gemm_ts", false, rows, c, c, 1.0, w.T2, c, w.Ri, c, 0.0,
                       (const T*)nullptr, 0, Out, ldout, w.partial, w.partial_elems, s);
    // stream ids of the replacement draws: one sequence per stream
    const uint64_t sid = s == cx.aux ? (1ULL << 21) + (++cx.fix_calls_aux)
                                     : (1ULL << 20) + (++cx.fix_calls);
    orth_fallback<T>(tm, rows, c, w.flags, w.flags + c, w.T1, c, Out, ldout,
                     nx > 0 ? X[0] : (const T*)nullptr, nx > 0 ? ldx[0] : 0, nx > 0 ? bx[0] : 0,
                     nx > 1 ? X[1] : (const T*)nullptr, nx > 1 ? ldx[1] : 0, nx > 1 ? bx[1] : 0,
                     w.xv, w.nflag, seed, sid, s);
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
                      sw.flags, sw.nflag, sw.xv};
    orth_against<T>(cx, w, s, rows, b0, X, ldx, In, ldin, c, Out, ldout, seed);
}

// SVD of the small projected matrix: the top nv values and vectors, by the
// Golub-Kahan path (2 <= N <= 1024), whose leading vectors are then polished
// to orthonormal by Cholesky-QR (inverse iteration leaves the vectors of close
// values only nearly orthogonal).
// nflag[1] is set if the cooperative bidiagonalisation timed out.
void small_svd_dispatch(Context& cx, hipStream_t s, int N, int nv, const double* B, int ldb,
                        double* UB, double* S, double* VB, double* svd_scratch,
                        const OrthWs<double>& w, uint64_t seed)
{
    TimedLaunch tl(&cx.timer, "small_svd", s, 0.0, 0.0);
    if (small_svd_gk_supported(N)) {
        if (cx.single_stream) {
            small_svd_gk(&cx.timer, N, nv, B, ldb, UB, S, VB, svd_scratch, w.nflag + 1, s);
        } else {
            cx.ensure_aux();  // the reflector blocks' T factors go on the second stream
            small_svd_gk(&cx.timer, N, nv, B, ldb, UB, S, VB, svd_scratch, w.nflag + 1, s,
                         cx.aux, cx.ev_fork, cx.ev_join);
        }
        if (cholqr2_small_supported(N, nv)) {
            const uint64_t sid0 = (1ULL << 20) + (++cx.fix_calls);
            const uint64_t sid1 = (1ULL << 20) + (++cx.fix_calls);
            cholqr2_small(&cx.timer, N, nv, UB, VB, N, w.nflag, CHOL_ETA, seed, sid0, sid1, w.Gr,
                          w.Ri, s);
        } else {
            orth_against<double>(cx, w, s, N, 0, nullptr, 0, UB, N, nv, UB, N, seed);
            orth_against<double>(cx, w, s, N, 0, nullptr, 0, VB, N, nv, VB, N, seed);
        }
    } else {
        BLWS_REQUIRE(N == 1, BLWS_EUNSUPPORTED, "small SVD: size above 1024");
        small_svd_1x1(B, UB, S, VB, s);
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
    // with Wh, the low half BF16(W - Wh) (ld ldw): split-precision BF16 x 3 products
    const unsigned short* Wl = nullptr;
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
                    (float*)w.partial, 2 * w.partial_elems, s, bf ? op.Wl : nullptr);
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

// The dense W-product op_apply would launch, as a grouped-launch problem
// (same kernel, same split-K scratch, hence the same result).
template <typename T>
WProduct dense_wproduct(const StepWs<T>& w, const Op<T>& op, int m, int n, bool trans,
                        const T* X, int ldx, int c, T* out, int ldo)
{
    WProduct pr{};
    const bool bf = std::is_same<T, float>::value && op.Wh != nullptr;
    pr.prec = std::is_same<T, double>::value ? 0 : (bf ? 2 : 1);
    pr.trans = trans;
    pr.M = trans ? n : m;
    pr.N = c;
    pr.K = trans ? m : n;
    pr.A = bf ? (const void*)op.Wh : (const void*)op.W;
    pr.lda = op.ldw;
    pr.B = X;
    pr.ldb = ldx;
    pr.C = out;
    pr.ldc = ldo;
    pr.partial = w.partial;
    pr.partial_elems = std::is_same<T, double>::value ? w.partial_elems : 2 * w.partial_elems;
    return pr;
}

// The first half of a BLWS step on two streams: [U, F] and [V, G] with
// F = orth(W V against U), G = orth(W^T U against V), the right half (V, Q, G)
// on the context's second stream with its own scratch, queued by the
// context's second host thread; the caller's stream waits for both.
template <typename T>
void svt_step_pair1_two_streams(Context& cx, StepWs<T>& w, hipStream_t s, int m, int n,
                                const Op<T>& W, int b, const T* U, int ldu, const T* V, int ldv,
                                uint64_t seed)
{
    const int b2 = 2 * b;
    StepWs<T> wb = w.aux_view();
    cx.fork(s);
    // U and V into the left halves of [U, F] and [V, G], on this stream after
    // the fork: the second stream's chain is the longer one and needs neither
    // (it reads U and V and writes only the right half of [V, G])
    copy2d<T, T>(m, b, U, ldu, w.UF, b2, s);
    copy2d<T, T>(n, b, V, ldv, w.VG, b2, s);
    // products with the start block: P = W V, Q = W^T U (the low-rank
    // coefficients of the matrix-completion operator have one buffer: there
    // Q waits for P)
    const bool grouped = cx.group && W.W && !W.Wl;  // BF16 x 3 products are not grouped
    if (grouped) {
        // the request server groups these with other solves' products
        const WProduct pr[2] = {dense_wproduct<T>(w, W, m, n, false, V, ldv, b, w.PH, b2),
                                dense_wproduct<T>(wb, W, m, n, true, U, ldu, b, w.Qb, b)};
        const hipStream_t st[2] = {s, cx.aux};
        cx.group->submit(pr, st, 2);
    } else {
        op_apply<T>(cx, w, s, W, m, n, false, V, ldv, b, w.PH, b2);
        if (!W.W) cx.fork(s);
    }
    // new block: F = orth(P - U U^T P) on this thread and stream, Q = W^T U
    // and G = orth(Q - V V^T Q) queued by the context's second host thread on
    // the second stream, so that both streams are fed at once
    {
        struct Join {  // the task refers to this frame: wait for it on every path
            AuxWorker* wk;
            bool waited = false;
            ~Join()
            {
                if (!waited) try {
                        wk->wait();
                    } catch (...) {
                    }
            }
        } jn{cx.worker.get()};
        cx.worker->run([&] {
            if (!grouped) op_apply<T>(cx, wb, cx.aux, W, m, n, true, U, ldu, b, w.Qb, b);
            orth_against<T>(cx, wb, cx.aux, n, b, V, ldv, w.Qb, b, b, w.VG + b, b2, seed);
        });
        orth_against<T>(cx, w, s, m, b, U, ldu, w.PH, b2, b, w.UF + b, b2, seed);
        jn.waited = true;
        cx.worker->wait();
    }
    cx.join(s);
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
//
// In two parts: the products (the new blocks and B, written to the step's
// scratch only; U and V are read) and the rest (SVD of B, Ritz vectors into
// U and V, S, the count above eps).
template <typename T>
void svt_step_products(Context& cx, StepWs<T>& w, hipStream_t s, int m, int n, const Op<T>& W,
                       int b, const T* U, int ldu, const T* V, int ldv, uint64_t seed)
{
    Timer* tm = &cx.timer;
    const int b2 = 2 * b;
    if (cx.single_stream) {
        // everything in order on s: the right half's work reuses the left
        // half's scratch once that is done with it
        copy2d<T, T>(m, b, U, ldu, w.UF, b2, s);
        copy2d<T, T>(n, b, V, ldv, w.VG, b2, s);
        op_apply<T>(cx, w, s, W, m, n, false, V, ldv, b, w.PH, b2);
        orth_against<T>(cx, w, s, m, b, U, ldu, w.PH, b2, b, w.UF + b, b2, seed);
        op_apply<T>(cx, w, s, W, m, n, true, U, ldu, b, w.Qb, b);
        orth_against<T>(cx, w, s, n, b, V, ldv, w.Qb, b, b, w.VG + b, b2, seed);
    } else {
        svt_step_pair1_two_streams<T>(cx, w, s, m, n, W, b, U, ldu, V, ldv, seed);
    }
    // the last product of the pass: H = W G
    if (cx.group && W.W && !W.Wl && !cx.single_stream) {
        const WProduct pr = dense_wproduct<T>(w, W, m, n, false, w.VG + b, b2, b, w.PH + b, b2);
        cx.group->submit(&pr, &s, 1);
    } else {
        op_apply<T>(cx, w, s, W, m, n, false, w.VG + b, b2, b, w.PH + b, b2);
    }
    // B = [U, F]^T [P, H] in FP64
    gemm<T, T, double>(tm, "gemm_ts", true, b2, b2, m, 1.0, w.UF, b2, w.PH, b2, 0.0,
                       (const double*)nullptr, 0, w.Bm, b2, w.partial, w.partial_elems, s);
}

template <typename T>
void svt_step_finish(Context& cx, StepWs<T>& w, hipStream_t s, int m, int n, double eps, int b,
                     T* U, int ldu, T* V, int ldv, double* S, int* rank_dev, uint64_t seed)
{
    Timer* tm = &cx.timer;
    const int b2 = 2 * b;
    {
        const OrthWs<double> ow{w.D1, w.D2, w.Cp, w.Gr, w.Ri, w.chol, w.partial,
                                w.partial_elems, w.flags, w.nflag, w.xv};
        small_svd_dispatch(cx, s, b2, b, w.Bm, b2, w.UB, w.Sall, w.VB, w.svd, ow, seed);
    }
    // Ritz vectors [U, F] U_B(:, 1:b), [V, G] V_B(:, 1:b), on the two streams
    if (cx.single_stream) {
        gemm<T, double, T>(tm, "gemm_ts", false, m, b, b2, 1.0, w.UF, b2, w.UB, b2, 0.0,
                           (const T*)nullptr, 0, U, ldu, w.partial, w.partial_elems, s);
        gemm<T, double, T>(tm, "gemm_ts", false, n, b, b2, 1.0, w.VG, b2, w.VB, b2, 0.0,
                           (const T*)nullptr, 0, V, ldv, w.partial, w.partial_elems, s);
    } else {
        const StepWs<T> wb = w.aux_view();
        cx.fork(s);
        gemm<T, double, T>(tm, "gemm_ts", false, m, b, b2, 1.0, w.UF, b2, w.UB, b2, 0.0,
                           (const T*)nullptr, 0, U, ldu, w.partial, w.partial_elems, s);
        gemm<T, double, T>(tm, "gemm_ts", false, n, b, b2, 1.0, w.VG, b2, w.VB, b2, 0.0,
                           (const T*)nullptr, 0, V, ldv, wb.partial, wb.partial_elems, cx.aux);
        cx.join(s);
    }
    copy2d<double, double>(1, b, w.Sall, b2, S, b, s);
    if (rank_dev) count_above(b, S, eps, rank_dev, s);
}

template <typename T>
void svt_step(Context& cx, StepWs<T>& w, hipStream_t s, int m, int n, const Op<T>& W,
              double eps, int b, T* U, int ldu, T* V, int ldv, double* S, int* rank_dev,
              uint64_t seed)
{
    svt_step_products<T>(cx, w, s, m, n, W, b, U, ldu, V, ldv, seed);
    svt_step_finish<T>(cx, w, s, m, n, eps, b, U, ldu, V, ldv, S, rank_dev, seed);
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

// Block width for a predicted rank sv (Sec. 4.2: the Ritz output follows the
// predicted rank): rounded up to b_round, at most floor(p / 2) and b_max.
int block_width(int sv, const blws_alm_opts& o, int p)
{
    int b = ((sv + o.b_round - 1) / o.b_round) * o.b_round;
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

}  // namespace
}  // namespace blws
