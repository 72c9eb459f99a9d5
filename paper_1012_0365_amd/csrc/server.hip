// Request server: RPCA and matrix-completion solves of any sizes, submitted at
// any time, run with continuous batching on one GPU.
//
// A scheduler thread owns max_slots slots; each slot has its own HIP stream,
// workspace and pinned readback area, and holds one solve (a Job) at a time.
// Requests wait in a FIFO queue and are admitted, in order, as soon as a slot
// is free and their workspace fits the memory budget next to the solves in
// flight. The scheduler then works in rounds: the solves whose last readback
// has landed (event queries, no blocking; a ready solve waits up to the
// grouping window for others) run their host logic together, one thread per
// slot, each queueing its next tick on its own stream, so the GPU work of
// different requests overlaps on the device. The dense W-products of the
// BLWS steps of a round go to one collector and out as grouped launches.
// Each solve keeps D, E, Y (or the samples and multipliers) and its warm
// block resident in its slot until it finishes. The per-request arithmetic is
// the same as in the blocking solvers (a grouped launch computes each problem
// exactly as its own launch would), so a result does not depend on the mix it
// ran in.
#include <algorithm>
#include <functional>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "jobs.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Slot {
    blws::Context cx;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::unique_ptr<blws::Job> job;
    long long ticket = -1;
    size_t bytes = 0;
    bool busy = false;
    bool started = false;
    Clock::time_point t_submit;
};

struct Pending {
    long long ticket;
    std::unique_ptr<blws::Job> job;
    size_t bytes;
    Clock::time_point t_submit;
};

struct Result {
    bool done = false;
    int status = BLWS_OK;
    blws_solve_info info{};
    std::string error;
};

// One thread per slot; run() hands them a round's tasks and waits for all.
struct Pool {
    int device = 0;
    std::vector<std::thread> th;
    std::mutex m;
    std::condition_variable cv_task, cv_done;
    std::deque<std::function<void()>> q;
    int pending = 0;
    bool stop = false;

    void start(int n, int dev)
    {
        device = dev;
        for (int i = 0; i < n; ++i) th.emplace_back([this] { loop(); });
    }
    void loop()
    {
        (void)hipSetDevice(device);
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(m);
                cv_task.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty()) return;  // stop
                f = std::move(q.front());
                q.pop_front();
            }
            f();  // does not throw
            std::lock_guard<std::mutex> g(m);
            if (--pending == 0) cv_done.notify_all();
        }
    }
    void run(std::vector<std::function<void()>>& tasks)
    {
        {
            std::lock_guard<std::mutex> g(m);
            pending += (int)tasks.size();
            for (auto& t : tasks) q.push_back(std::move(t));
        }
        cv_task.notify_all();
        std::unique_lock<std::mutex> lk(m);
        cv_done.wait(lk, [&] { return pending == 0; });
    }
    void shutdown()
    {
        {
            std::lock_guard<std::mutex> g(m);
            stop = true;
        }
        cv_task.notify_all();
        for (auto& t : th)
            if (t.joinable()) t.join();
        th.clear();
    }
};

// The W-products of one round's solves. A solve hands over its products
// (submit, from its slot thread) and waits; once every solve of the round has
// either handed over products or finished its work for the round (leave),
// the last one to arrive queues them: the grouped stream waits for the work
// already on every stream handed over, runs one grouped launch per precision
// (products that only the special skinny kernels take go alone), and every
// stream handed over then waits for it.
struct Collector : blws::ProductGroup {
    std::mutex m;
    std::condition_variable cv;
    int inside = 0;
    struct Req {
        const blws::WProduct* p;
        const hipStream_t* st;
        int n;
        bool issued;
    };
    std::vector<Req*> pending;
    hipStream_t bs = nullptr;
    hipEvent_t ev_batch = nullptr;
    std::vector<hipEvent_t> ev_in;
    bool failed = false;
    std::string error;
    long long launches = 0, products = 0;
    int max_group = 0;

    void create(int max_streams)
    {
        HIP_TRY(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ev_batch, hipEventDisableTiming));
        ev_in.resize(max_streams, nullptr);
        for (auto& e : ev_in) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    void destroy()
    {
        for (auto& e : ev_in)
            if (e) (void)hipEventDestroy(e);
        ev_in.clear();
        if (ev_batch) (void)hipEventDestroy(ev_batch);
        if (bs) {
            (void)hipStreamSynchronize(bs);
            (void)hipStreamDestroy(bs);
        }
        ev_batch = nullptr;
        bs = nullptr;
    }
    void begin(int n)
    {
        std::lock_guard<std::mutex> g(m);
        inside = n;
        failed = false;
        error.clear();
    }
    void leave()
    {
        std::lock_guard<std::mutex> g(m);
        --inside;
        if (!pending.empty() && (int)pending.size() == inside) launch_locked();
    }
    void submit(const blws::WProduct* p, const hipStream_t* st, int n) override
    {
        Req r{p, st, n, false};
        std::unique_lock<std::mutex> lk(m);
        pending.push_back(&r);
        if ((int)pending.size() == inside) launch_locked();
        cv.wait(lk, [&] { return r.issued; });
        if (failed) throw blws::BlwsError{BLWS_EDEVICE, "server: grouped launch: " + error};
    }
    void launch_locked()
    {
        try {
            issue();
        } catch (const blws::BlwsError& e) {
            failed = true;
            error = e.msg;
        } catch (const std::exception& e) {
            failed = true;
            error = e.what();
        }
        for (Req* r : pending) r->issued = true;
        pending.clear();
        cv.notify_all();
    }
    void launch_single(const blws::WProduct& w)
    {
        if (w.prec == 0)
            blws::gemm<double, double, double>(
                nullptr, "gemm_w", w.trans, w.M, w.N, w.K, 1.0, (const double*)w.A, w.lda,
                (const double*)w.B, w.ldb, 0.0, (const double*)nullptr, 0, (double*)w.C, w.ldc,
                (double*)w.partial, w.partial_elems, bs);
        else
            blws::gemm_lp(nullptr, "gemm_w", w.prec == 2, w.trans, w.M, w.N, w.K, w.A, w.lda,
                          (const float*)w.B, w.ldb, (float*)w.C, w.ldc, (float*)w.partial,
                          w.partial_elems, bs);
    }
    void issue()
    {
        size_t k = 0;
        for (Req* r : pending)
            for (int i = 0; i < r->n; ++i) {
                BLWS_REQUIRE(k < ev_in.size(), BLWS_EDEVICE, "too many streams in one round");
                HIP_TRY(hipEventRecord(ev_in[k], r->st[i]));
                HIP_TRY(hipStreamWaitEvent(bs, ev_in[k], 0));
                ++k;
            }
        std::vector<blws::WProduct> g[3];
        for (Req* r : pending)
            for (int i = 0; i < r->n; ++i) {
                const blws::WProduct& w = r->p[i];
                const bool ok = w.prec == 0 ? blws::wproduct_groupable(w)
                                            : blws::wproduct_lp_groupable(w);
                if (ok)
                    g[w.prec].push_back(w);
                else
                    launch_single(w);
            }
        for (int prec = 0; prec < 3; ++prec)
            for (size_t c0 = 0; c0 < g[prec].size(); c0 += blws::GEMM_GROUP_MAX) {
                const int cnt = (int)std::min<size_t>(blws::GEMM_GROUP_MAX, g[prec].size() - c0);
                if (prec == 0)
                    blws::gemm_f64_grouped(g[prec].data() + c0, cnt, bs);
                else
                    blws::gemm_lp_grouped(g[prec].data() + c0, cnt, bs);
                ++launches;
                products += cnt;
                max_group = std::max(max_group, cnt);
            }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(ev_batch, bs));
        for (Req* r : pending)
            for (int i = 0; i < r->n; ++i) HIP_TRY(hipStreamWaitEvent(r->st[i], ev_batch, 0));
    }
};

}  // namespace

struct blws_server_s {
    int device = 0;
    int max_slots = 4;
    size_t budget = 0;
    bool group = true;
    int window_us = 200;
    Pool pool;
    Collector col;
    std::vector<std::unique_ptr<Slot>> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::unordered_map<long long, Result> results;
    long long next_ticket = 1;
    bool stop = false;

    // statistics (under mu)
    long long submitted = 0, completed = 0, failed = 0;
    int active = 0, max_active = 0;
    size_t in_use = 0, peak = 0;
    std::string last_error;

    std::thread worker;
    std::string worker_error;

    void finish(Slot& sl, int status, const std::string& err)
    {
        if (status < 0) (void)hipStreamSynchronize(sl.stream);  // the slot is reused next
        std::lock_guard<std::mutex> g(mu);
        Result& r = results[sl.ticket];
        r.done = true;
        r.status = status;
        if (sl.job) r.info = sl.job->info;
        if (status < 0) std::memset(&r.info, 0, sizeof(r.info));
        r.info.status = status < 0 ? status : r.info.status;
        r.info.seconds = std::chrono::duration<double>(Clock::now() - sl.t_submit).count();
        r.error = err;
        if (status < 0) ++failed;
        else ++completed;
        in_use -= sl.bytes;
        --active;
        sl.job.reset();
        sl.busy = false;
        sl.started = false;
        sl.ticket = -1;
        sl.bytes = 0;
        cv_done.notify_all();
    }

    // Admit queued requests in order while a slot is free and the workspace
    // fits the budget (a request larger than the budget runs alone).
    std::vector<Slot*> admit()
    {
        std::vector<Slot*> out;
        std::lock_guard<std::mutex> g(mu);
        while (!queue.empty()) {
            Slot* free_slot = nullptr;
            for (auto& sp : slots)
                if (!sp->busy) {
                    free_slot = sp.get();
                    break;
                }
            if (!free_slot) break;
            Pending& pr = queue.front();
            if (in_use > 0 && in_use + pr.bytes > budget) break;
            free_slot->job = std::move(pr.job);
            free_slot->ticket = pr.ticket;
            free_slot->bytes = pr.bytes;
            free_slot->t_submit = pr.t_submit;
            free_slot->busy = true;
            free_slot->started = false;
            in_use += pr.bytes;
            if (in_use > peak) peak = in_use;
            ++active;
            if (active > max_active) max_active = active;
            queue.pop_front();
            out.push_back(free_slot);
        }
        return out;
    }

    // the busy slots whose last tick has finished: finished solves are
    // reported, the others appended to `ready` (once)
    void poll_ready(std::vector<std::pair<Slot*, bool>>& ready, bool& progressed)
    {
        for (auto& sp : slots) {
            Slot& sl = *sp;
            if (!sl.busy || !sl.started) continue;
            bool listed = false;
            for (auto& r : ready) listed = listed || r.first == &sl;
            if (listed) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            progressed = true;
            if (q != hipSuccess) {
                finish(sl, BLWS_EDEVICE, std::string("server: ") + hipGetErrorString(q));
                continue;
            }
            if (sl.job->done) {
                finish(sl, sl.job->status, "");
                continue;
            }
            ready.push_back({&sl, false});
        }
    }

    bool others_pending(const std::vector<std::pair<Slot*, bool>>& ready)
    {
        for (auto& sp : slots) {
            if (!sp->busy || !sp->started) continue;
            bool listed = false;
            for (auto& r : ready) listed = listed || r.first == sp.get();
            if (!listed) return true;
        }
        return false;
    }

    // one round: every listed solve starts or advances on its slot thread;
    // their W-products meet in the collector
    void run_round(std::vector<std::pair<Slot*, bool>>& ready)
    {
        std::vector<int> st(ready.size(), BLWS_OK);
        std::vector<std::string> err(ready.size());
        if (group) col.begin((int)ready.size());
        std::vector<std::function<void()>> tasks;
        for (size_t i = 0; i < ready.size(); ++i) {
            tasks.push_back([this, &ready, &st, &err, i] {
                Slot* sl = ready[i].first;
                try {
                    if (ready[i].second) {
                        sl->cx.fix_calls = 0;
                        sl->cx.fix_calls_aux = 0;
                        sl->cx.ensure(sl->bytes);
                        sl->job->start(sl->cx, sl->stream);
                    } else {
                        sl->job->advance(sl->cx, sl->stream);
                    }
                    HIP_TRY(hipEventRecord(sl->ev, sl->stream));
                } catch (const blws::BlwsError& e) {
                    st[i] = e.status;
                    err[i] = e.msg;
                } catch (const std::exception& e) {
                    st[i] = BLWS_EDEVICE;
                    err[i] = e.what();
                }
                if (group) col.leave();
            });
        }
        pool.run(tasks);
        for (size_t i = 0; i < ready.size(); ++i) {
            Slot* sl = ready[i].first;
            if (st[i] < 0)
                finish(*sl, st[i], err[i]);
            else if (ready[i].second)
                sl->started = true;
        }
    }

    void run()
    {
        if (hipSetDevice(device) != hipSuccess) {
            worker_error = "server: hipSetDevice failed";
            return;
        }
        for (;;) {
            bool progressed = false;
            std::vector<std::pair<Slot*, bool>> ready;
            for (Slot* sl : admit()) {
                progressed = true;
                ready.push_back({sl, true});
            }
            poll_ready(ready, progressed);
            if (!ready.empty() && group && window_us > 0) {
                // give the other solves in flight a short window to be ready too
                const auto t0 = Clock::now();
                while (others_pending(ready) &&
                       Clock::now() - t0 < std::chrono::microseconds(window_us)) {
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                    poll_ready(ready, progressed);
                }
            }
            if (!ready.empty()) run_round(ready);
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && active == 0) break;
            if (!progressed) {
                if (active == 0)
                    cv_work.wait(lk, [&] { return stop || !queue.empty(); });
                else
                    cv_work.wait_for(lk, std::chrono::microseconds(20));
            }
        }
    }
};

static thread_local std::string g_server_error;

static int server_fail(blws_server srv, const blws::BlwsError& e)
{
    if (srv) {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->last_error = e.msg;
    } else {
        g_server_error = e.msg;
    }
    return e.status;
}

static long long enqueue(blws_server srv, std::unique_ptr<blws::Job> job)
{
    const size_t bytes = job->workspace_bytes();
    std::lock_guard<std::mutex> g(srv->mu);
    const long long t = srv->next_ticket++;
    srv->results[t] = Result{};
    srv->queue.push_back(Pending{t, std::move(job), bytes, Clock::now()});
    ++srv->submitted;
    srv->cv_work.notify_one();
    return t;
}

extern "C" {

void blws_default_server_opts(blws_server_opts* o)
{
    if (!o) return;
    o->max_slots = 4;
    o->mem_budget = 0;
    o->group_products = 1;
    o->group_window_us = 200;
}

int blws_server_create(blws_server* out, int device, const blws_server_opts* opts)
{
    if (!out) return BLWS_EINVAL;
    *out = nullptr;
    blws_server_opts o;
    blws_default_server_opts(&o);
    if (opts) o = *opts;
    if (o.max_slots < 1 || o.max_slots > 16) {
        g_server_error = "blws_server_create: max_slots must be in 1..16";
        return BLWS_EINVAL;
    }
    if (o.group_window_us < 0 || o.group_window_us > 10000) {
        g_server_error = "blws_server_create: group_window_us must be in 0..10000";
        return BLWS_EINVAL;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        g_server_error = "blws_server_create: no such HIP device";
        return BLWS_EDEVICE;
    }
    std::unique_ptr<blws_server_s> sv(new (std::nothrow) blws_server_s());
    if (!sv) return BLWS_ENOMEM;
    sv->device = device;
    sv->max_slots = o.max_slots;
    sv->group = o.group_products != 0;
    sv->window_us = o.group_window_us;
    try {
        HIP_TRY(hipSetDevice(device));
        sv->col.create(2 * o.max_slots);
        size_t free_b = 0, total_b = 0;
        HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        sv->budget = o.mem_budget ? o.mem_budget : (size_t)(0.8 * (double)free_b);
        for (int i = 0; i < o.max_slots; ++i) {
            std::unique_ptr<Slot> sl(new Slot());
            sl->cx.device = device;
            HIP_TRY(hipHostMalloc(&sl->cx.host_pinned, 4096, hipHostMallocDefault));
            HIP_TRY(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming));
            if (sv->group) sl->cx.group = &sv->col;
            sv->slots.push_back(std::move(sl));
        }
    } catch (const blws::BlwsError& e) {
        for (auto& sl : sv->slots) {
            if (sl->ev) (void)hipEventDestroy(sl->ev);
            if (sl->stream) (void)hipStreamDestroy(sl->stream);
            if (sl->cx.host_pinned) (void)hipHostFree(sl->cx.host_pinned);
        }
        sv->col.destroy();
        g_server_error = e.msg;
        return e.status;
    }
    blws_server_s* raw = sv.get();
    raw->pool.start(o.max_slots, device);
    raw->worker = std::thread([raw] { raw->run(); });
    *out = sv.release();
    return BLWS_OK;
}

int blws_server_destroy(blws_server srv)
{
    if (!srv) return BLWS_EINVAL;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    srv->pool.shutdown();
    (void)hipSetDevice(srv->device);
    srv->col.destroy();
    for (auto& sl : srv->slots) {
        (void)hipStreamSynchronize(sl->stream);
        (void)hipEventDestroy(sl->ev);
        (void)hipStreamDestroy(sl->stream);
        sl->cx.timer.release();
        sl->cx.release_aux();
        if (sl->cx.ws) (void)hipFree(sl->cx.ws);
        if (sl->cx.host_pinned) (void)hipHostFree(sl->cx.host_pinned);
    }
    delete srv;
    return BLWS_OK;
}

int blws_server_submit_rpca(blws_server srv, int prec, int m, int n, const void* D, int ldd,
                            double lambda, const blws_alm_opts* opts, void* A, int lda, void* E,
                            int lde, long long* ticket)
{
    if (!srv || !ticket) return BLWS_EINVAL;
    try {
        auto job = blws::make_rpca_job(prec, m, n, D, ldd, lambda, opts, A, lda, E, lde,
                                       "blws_server_submit_rpca");
        *ticket = enqueue(srv, std::move(job));
        return BLWS_OK;
    } catch (const blws::BlwsError& e) {
        return server_fail(srv, e);
    } catch (const std::exception& e) {
        return server_fail(srv, blws::BlwsError{BLWS_ENOMEM, e.what()});
    }
}

int blws_server_submit_mc(blws_server srv, int prec, int m, int n, int nnz, const int* row_ptr,
                          const int* col_idx, const void* values, const blws_alm_opts* opts,
                          int r_cap, void* U, int ldu, double* S, void* V, int ldv,
                          long long* ticket)
{
    if (!srv || !ticket) return BLWS_EINVAL;
    try {
        auto job = blws::make_mc_job(prec, m, n, nnz, row_ptr, col_idx, values, opts, r_cap, U,
                                     ldu, S, V, ldv, "blws_server_submit_mc");
        *ticket = enqueue(srv, std::move(job));
        return BLWS_OK;
    } catch (const blws::BlwsError& e) {
        return server_fail(srv, e);
    } catch (const std::exception& e) {
        return server_fail(srv, blws::BlwsError{BLWS_ENOMEM, e.what()});
    }
}

static int take_result(blws_server srv, std::unordered_map<long long, Result>::iterator it,
                       blws_solve_info* info)
{
    const int st = it->second.status;
    if (info) *info = it->second.info;
    if (st < 0) srv->last_error = it->second.error;
    srv->results.erase(it);
    return st;
}

int blws_server_poll(blws_server srv, long long ticket, int* done, blws_solve_info* info)
{
    if (!srv || !done) return BLWS_EINVAL;
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = srv->results.find(ticket);
    if (it == srv->results.end()) {
        srv->last_error = "blws_server_poll: unknown ticket";
        return BLWS_EINVAL;
    }
    *done = it->second.done ? 1 : 0;
    if (!it->second.done) return BLWS_OK;
    return take_result(srv, it, info);
}

int blws_server_wait(blws_server srv, long long ticket, blws_solve_info* info)
{
    if (!srv) return BLWS_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->results.find(ticket);
    if (it == srv->results.end()) {
        srv->last_error = "blws_server_wait: unknown ticket";
        return BLWS_EINVAL;
    }
    srv->cv_done.wait(lk, [&] { return srv->results[ticket].done; });
    return take_result(srv, srv->results.find(ticket), info);
}

int blws_server_get_stats(blws_server srv, blws_server_stats* st)
{
    if (!srv || !st) return BLWS_EINVAL;
    std::lock_guard<std::mutex> g(srv->mu);
    st->submitted = srv->submitted;
    st->completed = srv->completed;
    st->failed = srv->failed;
    st->active = srv->active;
    st->queued = (int)srv->queue.size();
    st->max_active = srv->max_active;
    st->mem_in_use = srv->in_use;
    st->mem_peak = srv->peak;
    st->mem_budget = srv->budget;
    std::lock_guard<std::mutex> gc(srv->col.m);
    st->grouped_launches = srv->col.launches;
    st->grouped_products = srv->col.products;
    st->max_group = srv->col.max_group;
    return BLWS_OK;
}

const char* blws_server_last_error(blws_server srv)
{
    if (!srv) return g_server_error.c_str();
    return srv->last_error.c_str();
}

}  // extern "C"
