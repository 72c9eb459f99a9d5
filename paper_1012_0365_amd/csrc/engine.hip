// Host side of libblws: kernel timing and the C ABI declared in
// include/blws.h (contexts, the BLWS SVT call, the solvers, diagnostics).
#include "jobs.h"

namespace blws {

TimedLaunch::TimedLaunch(Timer* timer, const char* family, hipStream_t s, double flops,
                         double bytes)
    : t(timer && timer->on ? timer : nullptr), slot(-1), stream(s), fam(family)
{
    if (!t) return;
    std::lock_guard<std::mutex> g(t->mu);
    if (!t->wants(family)) {
        t = nullptr;
        return;
    }
    Timer::Family& f = t->fam[family];
    hipEvent_t a = t->take(), b = t->take();
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
    std::lock_guard<std::mutex> g(t->mu);
    (void)hipEventRecord(t->fam[fam].stop[slot], stream);
}

namespace {

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

// Scratch of blws_svt_noalloc: a file-scope device array, so that the call
// needs no allocation. Each device the library runs on holds its own copy for
// the life of the process. Host code never passes `scratch` itself to a
// kernel (on the host it names a stand-in, not device memory): it uses the
// device address looked up per device by noalloc_scratch_address().
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

// The device address of `scratch` on the current device (called once per
// context, with its device current).
void* noalloc_scratch_address()
{
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    BLWS_REQUIRE(ptr != nullptr, BLWS_EDEVICE, "static scratch has no device address");
    return ptr;
}

}  // namespace

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
    try {
        c->cx.static_scratch = noalloc_scratch_address();
    } catch (const BlwsError& e) {
        g_noctx_error = e.msg;
        (void)hipHostFree(c->cx.host_pinned);
        delete c;
        return e.status;
    }
    *out = c;
    return BLWS_OK;
}

int blws_destroy(blws_ctx ctx)
{
    if (!ctx) return BLWS_EINVAL;
    (void)hipSetDevice(ctx->cx.device);
    (void)hipDeviceSynchronize();
    ctx->cx.timer.release();
    ctx->cx.release_aux();
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
    o->b_max = 512;
    o->ladder_tol = 1e-3;
    o->svt_start = BLWS_START_SPLIT;
    o->k_blocks = 2;
    o->ladder3_tol = 0.0;
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
    BLWS_REQUIRE(2 * b <= 1024, BLWS_EUNSUPPORTED, "blws_svt: b above 512");
    blws_svt_opts o;
    blws_default_svt_opts(&o);
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)stream;
    if (prec == BLWS_FP64)
        blws::svt_call_t<double>(cx, s, m, n, (const double*)W, ldw, eps, b, (double*)U, ldu,
                                 (double*)V, ldv, warm, S, rank_dev, (double*)A, lda, o);
    else if (prec == BLWS_FP32 || prec == BLWS_BF16X3)
        blws::svt_call_t<float>(cx, s, m, n, (const float*)W, ldw, eps, b, (float*)U, ldu,
                                (float*)V, ldv, warm, S, rank_dev, (float*)A, lda, o,
                                prec == BLWS_BF16X3);
    else
        throw BlwsError{BLWS_EUNSUPPORTED, "blws_svt: precision not supported"};
    return BLWS_OK;
    ABI_END
}

int blws_svt_lanczos(blws_ctx ctx, void* stream, int m, int n, const double* W, int ldw,
                     double eps, int b, int start, int k, double* U, int ldu, double* V,
                     int ldv, double* S, int* rank_dev, double* A, int lda)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(m >= 2 && n >= 2 && b >= 1 && k >= 1 && 2 * b <= (m < n ? m : n), BLWS_EINVAL,
                 "blws_svt_lanczos: need m, n >= 2, k >= 1 and 1 <= b <= min(m, n) / 2");
    BLWS_REQUIRE(start >= BLWS_START_SPLIT && start <= BLWS_START_RIGHT, BLWS_EINVAL,
                 "blws_svt_lanczos: unknown start block");
    BLWS_REQUIRE(W && U && V && S, BLWS_EINVAL, "blws_svt_lanczos: null W, U, V or S");
    BLWS_REQUIRE(ldw >= n && ldu >= b && ldv >= b && (!A || lda >= n), BLWS_EINVAL,
                 "blws_svt_lanczos: leading dimension too small");
    BLWS_REQUIRE(std::isfinite(eps) && eps >= 0.0, BLWS_EINVAL,
                 "blws_svt_lanczos: eps must be >= 0");
    const long long K = (long long)k * blws::lz_cols(start, b);
    BLWS_REQUIRE(K <= m + n, BLWS_EINVAL, "blws_svt_lanczos: k blocks exceed m + n columns");
    BLWS_REQUIRE(K <= 1024, BLWS_EUNSUPPORTED, "blws_svt_lanczos: k c above 1024");
    hipStream_t s = (hipStream_t)stream;
    cx.ensure(blws::lanczos_ws_bytes(m, n, b, start, k));
    Carver c(cx.ws);
    blws::LanczosWs w;
    w.carve(c, m, n, b, start, k);
    blws::zero_bytes(w.nflag, 4 * sizeof(int), s);
    const blws::Op<double> op{W, ldw, nullptr, nullptr};
    blws_svt_opts so;
    blws_default_svt_opts(&so);
    blws::lanczos_step(cx, w, s, m, n, op, eps, b, start, k, U, ldu, V, ldv, S, rank_dev, so.seed);
    if (A) blws::svt_reconstruct<double>(&cx.timer, m, n, b, U, ldu, V, ldv, S, eps, A, lda, s);
    return BLWS_OK;
    ABI_END
}

int blws_svt_noalloc(blws_ctx ctx, void* stream, int prec, int m, int n, const void* W, int ldw,
                     double eps, int b, void* U, int ldu, void* V, int ldv, int warm, double* S,
                     int* rank_dev, void* A, int lda, const blws_svt_opts* opts)
{
    ABI_BEGIN(ctx)
    const int p = m < n ? m : n;
    BLWS_REQUIRE(m >= 2 && n >= 2 && b >= 1 && 2 * b <= p, BLWS_EINVAL,
                 "blws_svt_noalloc: need m, n >= 2 and 1 <= b <= min(m, n) / 2");
    BLWS_REQUIRE(W && U && V && S, BLWS_EINVAL, "blws_svt_noalloc: null W, U, V or S");
    BLWS_REQUIRE(ldw >= n && ldu >= b && ldv >= b && (!A || lda >= n), BLWS_EINVAL,
                 "blws_svt_noalloc: leading dimension too small");
    BLWS_REQUIRE(std::isfinite(eps) && eps >= 0.0, BLWS_EINVAL,
                 "blws_svt_noalloc: eps must be >= 0");
    BLWS_REQUIRE(2 * b <= 1024, BLWS_EUNSUPPORTED, "blws_svt_noalloc: b above 512");
    BLWS_REQUIRE(prec == BLWS_FP64 || prec == BLWS_FP32, BLWS_EUNSUPPORTED,
                 "blws_svt_noalloc: precision not supported");
    BLWS_REQUIRE(cx.static_scratch, BLWS_EDEVICE, "blws_svt_noalloc: no static scratch");
    blws_svt_opts o;
    blws_default_svt_opts(&o);
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)stream;
    auto run = [&](auto tag) {
        using T = decltype(tag);
        blws::StepWs<T> w;
        Carver dry(nullptr);
        w.carve(dry, m, n, b, false);
        if (dry.off + 256 > NOALLOC_SCRATCH_BYTES)
            throw BlwsError{BLWS_EINVAL, "blws_svt_noalloc: this size needs " +
                                             std::to_string((dry.off + 256) >> 20) +
                                             " MiB of scratch, above the static 64 MiB"};
        Carver c(cx.static_scratch);
        w.carve(c, m, n, b, false);
        // single stream, no timing events, no allocation; restored on every path
        struct Mode {
            Context& cx;
            bool on;
            Mode(Context& c) : cx(c), on(c.timer.on) { cx.single_stream = true; cx.timer.on = false; }
            ~Mode() { cx.single_stream = false; cx.timer.on = on; }
        } mode(cx);
        blws::zero_bytes(w.nflag, 4 * sizeof(int), s);
        const blws::Op<T> op{(const T*)W, ldw, nullptr, nullptr};
        if (!warm)
            blws::cold_block<T>(cx, w, s, m, n, op, b, o.pow_steps, o.seed, 1, (T*)U, ldu, (T*)V,
                                ldv);
        blws::svt_step<T>(cx, w, s, m, n, op, eps, b, (T*)U, ldu, (T*)V, ldv, S, rank_dev,
                          o.seed);
        if (A)
            blws::svt_reconstruct<T>(&cx.timer, m, n, b, (T*)U, ldu, (T*)V, ldv, S, eps, (T*)A,
                                     lda, s);
    };
    if (prec == BLWS_FP64)
        run(double{});
    else
        run(float{});
    return BLWS_OK;
    ABI_END
}

int blws_rpca_solve(blws_ctx ctx, void* stream, int prec, int m, int n, const void* D, int ldd,
                    double lambda, const blws_alm_opts* opts, void* A, int lda, void* E, int lde,
                    blws_solve_info* info)
{
    ABI_BEGIN(ctx)
    auto job = blws::make_rpca_job(prec, m, n, D, ldd, lambda, opts, A, lda, E, lde,
                                   "blws_rpca_solve");
    blws::run_blocking(*job, cx, (hipStream_t)stream);
    if (info) *info = job->info;
    return job->status;
    ABI_END
}

void blws_default_mc_opts(blws_alm_opts* o)
{
    if (!o) return;
    blws_default_alm_opts(o);
    o->tol = 1e-6;
    o->rho = 1.05;
    o->mu0_scale = 1.0;
    o->b_max = 256;
}

int blws_mc_solve(blws_ctx ctx, void* stream, int prec, int m, int n, int nnz,
                  const int* row_ptr, const int* col_idx, const void* values,
                  const blws_alm_opts* opts, int r_cap, void* U, int ldu, double* S, void* V,
                  int ldv, blws_solve_info* info)
{
    ABI_BEGIN(ctx)
    auto job = blws::make_mc_job(prec, m, n, nnz, row_ptr, col_idx, values, opts, r_cap, U, ldu,
                                 S, V, ldv, "blws_mc_solve");
    blws::run_blocking(*job, cx, (hipStream_t)stream);
    if (info) *info = job->info;
    return job->status;
    ABI_END
}

void blws_default_svt_mc_opts(blws_svt_mc_opts* o)
{
    if (!o) return;
    o->tau = 0.0;
    o->delta = 0.0;
    o->tol = 1e-4;
    o->max_iter = 500;
    o->rank_step = 5;
    o->b_round = 16;
    o->b_max = 512;
    o->pow_steps = 2;
    o->seed = 20101202ULL;
    o->norm_steps = 8;
    o->norm_rtol = 1e-13;
}

int blws_mc_svt_solve(blws_ctx ctx, void* stream, int prec, int m, int n, int nnz,
                      const int* row_ptr, const int* col_idx, const void* values,
                      const blws_svt_mc_opts* opts, int r_cap, void* U, int ldu, double* S,
                      void* V, int ldv, blws_solve_info* info)
{
    ABI_BEGIN(ctx)
    auto job = blws::make_mc_svt_job(prec, m, n, nnz, row_ptr, col_idx, values, opts, r_cap, U,
                                     ldu, S, V, ldv, "blws_mc_svt_solve");
    blws::run_blocking(*job, cx, (hipStream_t)stream);
    if (info) *info = job->info;
    return job->status;
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

int blws_gemm_bf16x3(blws_ctx ctx, void* stream, int trans_a, int M, int N, int K,
                     const void* A_hi, const void* A_lo, int lda, const float* B, int ldb,
                     float* C, int ldc)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(M >= 0 && N >= 0 && K >= 1 && A_hi && A_lo && B && C, BLWS_EINVAL,
                 "blws_gemm_bf16x3: bad arguments");
    BLWS_REQUIRE(ldb >= N && ldc >= N && lda >= (trans_a ? M : K), BLWS_EINVAL,
                 "blws_gemm_bf16x3: leading dimension too small");
    const size_t pe = blws::gemm_lp_partial_elems(M, N, K);
    cx.ensure((pe + 1) * sizeof(float) + 256);
    blws::gemm_lp(&cx.timer, "gemm_diag", true, trans_a != 0, M, N, K, A_hi, lda, B, ldb, C, ldc,
                  (float*)cx.ws, pe + 1, (hipStream_t)stream, (const unsigned short*)A_lo);
    return BLWS_OK;
    ABI_END
}

int blws_small_svd_f64(blws_ctx ctx, void* stream, int N, const double* B, int ldb, double* UB,
                       double* S, double* VB)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(N >= 1 && N <= 1024 && B && UB && S && VB && ldb >= N, BLWS_EINVAL,
                 "blws_small_svd_f64: bad arguments");
    double* svd = nullptr;
    auto layout = [&](Carver& c, blws::OrthWs<double>& w) {
        svd = c.take<double>(blws::small_svd_gk_scratch_elems(N));
        w.T1 = c.take<double>((size_t)N * N);
        w.T2 = c.take<double>((size_t)N * N);
        w.Cp = c.take<double>((size_t)N * N);
        w.Gr = c.take<double>((size_t)N * N);
        w.Ri = c.take<double>((size_t)N * N);
        w.chol = c.take<double>(blws::chol_scratch_elems(N) + 1);
        w.flags = c.take<int>((size_t)2 * N);
        w.nflag = c.take<int>(4);
        w.xv = c.take<double>((size_t)N);
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
    blws::zero_bytes(w.nflag, 4 * sizeof(int), s);
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

int blws_timing_only(blws_ctx ctx, const char* families)
{
    ABI_BEGIN(ctx)
    HIP_TRY(hipDeviceSynchronize());
    cx.timer.only.clear();
    if (families) {
        std::string cur;
        for (const char* c = families;; ++c) {
            if (*c == ',' || *c == '\0') {
                if (!cur.empty()) cx.timer.only.insert(cur);
                cur.clear();
                if (*c == '\0') break;
            } else {
                cur += *c;
            }
        }
    }
    return BLWS_OK;
    ABI_END
}

int blws_timing_list(blws_ctx ctx, char* buf, size_t len)
{
    ABI_BEGIN(ctx)
    BLWS_REQUIRE(buf && len > 0, BLWS_EINVAL, "blws_timing_list: null buffer");
    std::string names;
    for (auto& kv : cx.timer.fam) {
        if (!names.empty()) names += ",";
        names += kv.first;
    }
    BLWS_REQUIRE(names.size() < len, BLWS_EINVAL, "blws_timing_list: buffer too small");
    std::memcpy(buf, names.c_str(), names.size() + 1);
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
