// Serving: continuous batching of LP solve requests (see include/dualip.h).
//
// Threads per server, each with its own HIP stream (default priority):
//   loaders    (kLoaders of them) take queued requests first-come first-served
//              when a slot is free and the request's device footprint fits the
//              HBM budget, build and upload its problem and initialize its
//              iteration state -- while the device keeps iterating the
//              admitted ones (building a layout is host work of about 15 ms
//              per million nonzeros, so one loader would cap admissions);
//   scheduler  runs kTicksPerSync ticks of kTick iterations (gap test on the
//              last of each) over all active requests with the batched fused
//              launches, then reads their states back, retires the
//              finished ones (lambda copied to host) and adds the ready ones at
//              the next tick boundary;
//   reaper     releases the device memory of retired requests (freeing can
//              wait on the whole device, so the scheduler does not do it) and
//              returns their bytes to the budget.
// A request's iterates do not depend on what it shares a tick with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"

using namespace dl;
using dlh::hip_fail;
using dlh::set_error;

namespace {

constexpr int kTick = 10;     // iterations per tick; the gap is tested on the last
// ticks enqueued between two state read-backs: the device idles while the
// host reads states and enqueues the next launches, so fewer read-backs keep
// it busier; a request that stops in the first tick skips the second (its
// launches return at once) and leaves one tick later
constexpr int kTicksPerSync = 2;
constexpr int kLoaders = 4;   // concurrent problem builds

struct Request {
    uint64_t ticket = 0;
    // deep copies of the caller's arrays
    std::vector<int64_t> ptr, block_off;
    std::vector<int32_t> idx;
    std::vector<double> val, c, b, upper, v;
    std::vector<uint8_t> block_proj;
    dl_problem_desc desc;
    dl_problem_opts popts;
    dl_solve_opts sopts;
    size_t est_bytes = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int state = 0;   // 0 queued, 1 loading, 2 ready, 3 running, 4 finished
    dl_solve_result res;
    std::vector<double> lam_host;
    dl_problem* prob = nullptr;
    double* lam_dev = nullptr;
    SolveParams prm;
};

template <typename T>
static void copy_in(std::vector<T>& dst, const T* src, int64_t n)
{
    if (src && n > 0) dst.assign(src, src + n);
    else dst.clear();
}

}  // namespace

struct dl_server {
    size_t budget = 0;
    int max_slots = 1;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Request*> queue;
    std::vector<Request*> ready;
    std::map<uint64_t, Request*> all;
    size_t used = 0;
    int slots_used = 0;
    uint64_t next_ticket = 1;
    std::vector<std::thread> loaders;
    std::thread scheduler;
    // retired problems waiting to be freed, each with its lambda buffer, its
    // budget bytes and whether its stream is known to be idle
    struct Retired {
        dl_problem* prob;
        double* lam_dev;
        size_t bytes;
        bool idle;
    };
    std::deque<Retired> reap;
    bool sched_done = false;
    std::thread reaper;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// An upper bound of the device bytes dl_problem_create will hold for the
// request, by the same rules it allocates with: the edge stream (a, c, dst,
// perm; box bounds whenever any block is a box; 1/v^2 with primal scaling),
// at most one work item per block, up to two chunks per compute unit (the
// autotuner's largest choice) of partial sums for at most 16384 LDS rows, the
// row vectors, the request's lambda buffer and its share of the batched
// argument tables.  Once the problem exists the admission charge is lowered
// to its actual footprint.
static size_t estimate_bytes(const dl_problem_desc* d, const dl_problem_opts* o)
{
    const size_t es = o->storage == DL_F64 ? 8 : (o->storage == DL_F32 ? 4 : 2);
    const size_t n = (size_t)d->n, m = (size_t)d->m, nb = (size_t)d->num_blocks;
    bool has_box = false;
    for (size_t i = 0; i < nb && !has_box; ++i) has_box = d->block_proj[i] != DL_PROJ_SIMPLEX;
    size_t bytes = n * (2 * es + 4 + 8) + (has_box ? 4 * n : 0) + (o->primal_scale ? 4 * n : 0);
    bytes += nb * sizeof(Item);
    const size_t nch = std::min<size_t>(2 * 256, std::max<size_t>(1, (n + 32767) / 32768));
    bytes += nch * (sizeof(Chunk) + 3 * 8) + 3 * nch * std::min<size_t>(m, 16384) * 4;
    bytes += m * (8 * 14 + 4) + ((m + 63) / 64) * kRedStride * 8;
    bytes += m * 8 + 4096 + (1 << 20);
    return bytes;
}

// the bytes the request actually holds once built
static size_t actual_bytes(const dl_problem* p, const dl_problem_desc* d)
{
    return p->device_bytes + (size_t)d->m * 8 + 4096;
}

static void loader_main(dl_server* S)
{
    (void)hipSetDevice(S->device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] {
                if (S->stop) return true;
                if (S->queue.empty()) return false;
                Request* h = S->queue.front();
                return S->slots_used < S->max_slots && S->used + h->est_bytes <= S->budget;
            });
            if (S->stop) break;
            r = S->queue.front();
            S->queue.pop_front();
            S->slots_used += 1;
            S->used += r->est_bytes;
            r->state = 1;
        }
        dl_status st = dl_problem_create(&r->desc, &r->popts, s, &r->prob);
        hipError_t e = hipSuccess;
        if (st == DL_OK) {
            r->prm = dlh::make_params(&r->sopts, r->prob);
            e = hipMalloc((void**)&r->lam_dev, (size_t)r->desc.m * sizeof(double));
            if (e == hipSuccess)
                e = launch_solve_init(r->prob->st, r->prm, nullptr, r->prob->orig, r->prob->D, r->prob->J,
                                      r->prob->lam, r->prob->y, r->prob->yp, r->prob->G, r->prob->Gp,
                                      r->prob->lam_eval, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = DL_ERR_DEVICE;
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (st != DL_OK) {
            if (r->prob) dl_problem_destroy(r->prob);
            r->prob = nullptr;
            if (r->lam_dev) (void)hipFree(r->lam_dev);
            r->lam_dev = nullptr;
            std::memset(&r->res, 0, sizeof r->res);
            r->res.status = st;
            r->t_start = r->t_done = S->now();
            r->state = 4;
            S->slots_used -= 1;
            S->used -= r->est_bytes;
        } else {
            // charge the actual footprint from now on (never above the estimate)
            const size_t act = std::min(actual_bytes(r->prob, &r->desc), r->est_bytes);
            S->used -= r->est_bytes - act;
            r->est_bytes = act;
            r->state = 2;
            S->ready.push_back(r);
        }
        S->cv.notify_all();
    }
    if (s) (void)hipStreamDestroy(s);
}

static void scheduler_main(dl_server* S)
{
    (void)hipSetDevice(S->device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    std::vector<Request*> active;
    dlh::BatchRunner br;
    std::vector<SolveState> states;
    bool changed = false;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->ready.empty() || !active.empty(); });
            if (S->stop && active.empty() && S->ready.empty()) break;
            for (Request* r : S->ready) {
                r->state = 3;
                r->t_start = S->now();
                active.push_back(r);
                changed = true;
            }
            S->ready.clear();
        }
        if (active.empty()) continue;
        if (changed) {
            std::vector<dl_problem*> ps;
            std::vector<SolveParams> prm;
            for (Request* r : active) {
                ps.push_back(r->prob);
                prm.push_back(r->prm);
            }
            if (br.build(ps, prm, s) != DL_OK) {
                // cannot iterate: fail every active request
                std::lock_guard<std::mutex> lk(S->mu);
                for (Request* r : active) {
                    std::memset(&r->res, 0, sizeof r->res);
                    r->res.status = DL_ERR_DEVICE;
                    r->state = 4;
                    r->t_done = S->now();
                    dl_problem_destroy(r->prob);
                    r->prob = nullptr;
                    (void)hipFree(r->lam_dev);
                    r->lam_dev = nullptr;
                    S->slots_used -= 1;
                    S->used -= r->est_bytes;
                }
                active.clear();
                S->cv.notify_all();
                continue;
            }
            changed = false;
        }
        hipError_t e = hipSuccess;
        for (int q = 0; q < kTick * kTicksPerSync && e == hipSuccess; ++q)
            e = br.enqueue_iteration(q % kTick == kTick - 1 ? 1 : 0, s);
        if (e == hipSuccess) e = br.states(s, states);
        std::vector<Request*> keep, fin;
        for (size_t k = 0; k < active.size(); ++k) {
            if (e != hipSuccess || states[k].done) fin.push_back(active[k]);
            else keep.push_back(active[k]);
        }
        for (Request* r : fin) {
            dl_solve_result& res = r->res;
            std::memset(&res, 0, sizeof res);
            bool idle = false;   // this stream waited for all of the problem's work
            const size_t k = std::find(active.begin(), active.end(), r) - active.begin();
            if (e == hipSuccess) {
                const SolveState& f = states[k];
                hipError_t e2 = launch_solve_final(r->prob->st, r->prob->y, r->prob->yp, r->prob->orig,
                                                   r->prob->D, r->prob->J, r->lam_dev, s);
                r->lam_host.resize((size_t)r->desc.m);
                if (e2 == hipSuccess)
                    e2 = hipMemcpyAsync(r->lam_host.data(), r->lam_dev, r->lam_host.size() * sizeof(double),
                                        hipMemcpyDeviceToHost, s);
                if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
                idle = e2 == hipSuccess;
                res.converged = f.converged;
                res.stage = f.stage_eval;
                res.iters = f.k;
                res.gamma = f.gamma_eval;
                res.g = f.g;
                res.P = f.P;
                res.rel_gap = f.rel_gap;
                res.max_infeas = f.max_infeas;
                res.status = e2 != hipSuccess ? DL_ERR_DEVICE
                             : (f.status == 5 ? DL_ERR_NUMERIC : (f.converged ? DL_OK : DL_ERR_NOT_CONVERGED));
            } else {
                res.status = DL_ERR_DEVICE;
            }
            // its work ran on this stream, which the copy above waited for;
            // the reaper frees it and returns its bytes to the budget
            std::lock_guard<std::mutex> lk(S->mu);
            S->reap.push_back({r->prob, r->lam_dev, r->est_bytes, idle});
            r->prob = nullptr;
            r->lam_dev = nullptr;
            r->t_done = S->now();
            res.seconds = r->t_done - r->t_start;
            r->state = 4;
            S->slots_used -= 1;
            S->cv.notify_all();
        }
        if (!fin.empty()) {
            active.swap(keep);
            changed = true;
        }
    }
    br.release();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->sched_done = true;
        S->cv.notify_all();
    }
    if (s) (void)hipStreamDestroy(s);
}

static void reaper_main(dl_server* S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        dl_server::Retired x;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return !S->reap.empty() || S->sched_done; });
            if (S->reap.empty()) break;   // the scheduler has exited and nothing is left
            x = S->reap.front();
            S->reap.pop_front();
        }
        if (x.prob) {
            if (x.idle) dlh::destroy_idle(x.prob);
            else dl_problem_destroy(x.prob);
        }
        if (x.lam_dev) (void)hipFree(x.lam_dev);
        std::lock_guard<std::mutex> lk(S->mu);
        S->used -= x.bytes;
        S->cv.notify_all();
    }
}

extern "C" dl_status dl_server_create(size_t hbm_budget_bytes, int32_t max_slots, dl_server** out)
{
    if (!out || hbm_budget_bytes == 0 || max_slots < 1) { set_error("invalid server arguments"); return DL_ERR_INVALID_ARG; }
    dl_server* S = new dl_server();
    S->budget = hbm_budget_bytes;
    S->max_slots = max_slots;
    if (hipGetDevice(&S->device) != hipSuccess) { delete S; set_error("no HIP device"); return DL_ERR_DEVICE; }
    S->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < kLoaders; ++i) S->loaders.emplace_back(loader_main, S);
    S->scheduler = std::thread(scheduler_main, S);
    S->reaper = std::thread(reaper_main, S);
    *out = S;
    return DL_OK;
}

extern "C" dl_status dl_server_submit(dl_server* S, const dl_problem_desc* d, const dl_problem_opts* po,
                                      const dl_solve_opts* so, uint64_t* ticket)
{
    if (!S || !d || !so || !ticket) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    dl_problem_opts popts;
    dl_problem_opts_init(&popts);
    if (po) popts = *po;
    int col_entries = 1;
    dl_status st = dlh::validate_desc(d, &popts, &col_entries);
    if (st != DL_OK) return st;
    if (col_entries > 1) { set_error("served requests take one entry per column"); return DL_ERR_UNSUPPORTED; }
    st = dlh::check_solve_opts(so);
    if (st != DL_OK) return st;
    for (int64_t k = 0; k < d->nnz; ++k)
        if (d->val[k] < 0.0) { set_error("serving needs a >= 0"); return DL_ERR_UNSUPPORTED; }
    for (int64_t j = 0; j < d->m; ++j)
        if (d->b[j] < 0.0) { set_error("serving needs b >= 0"); return DL_ERR_UNSUPPORTED; }
    Request* r = new Request();
    const int64_t nptr = d->ptr ? (d->layout == DL_CSC ? d->n + 1 : d->m + 1) : 0;
    copy_in(r->ptr, d->ptr, nptr);
    copy_in(r->idx, d->idx, d->nnz);
    copy_in(r->val, d->val, d->nnz);
    copy_in(r->c, d->c, d->n);
    copy_in(r->b, d->b, d->m);
    copy_in(r->block_off, d->block_off, d->num_blocks + 1);
    copy_in(r->block_proj, d->block_proj, d->num_blocks);
    copy_in(r->upper, d->upper, d->n);
    r->desc = *d;
    r->desc.ptr = r->ptr.empty() ? nullptr : r->ptr.data();
    r->desc.idx = r->idx.data();
    r->desc.val = r->val.data();
    r->desc.c = r->c.data();
    r->desc.b = r->b.data();
    r->desc.block_off = r->block_off.data();
    r->desc.block_proj = r->block_proj.data();
    r->desc.upper = r->upper.empty() ? nullptr : r->upper.data();
    r->popts = popts;
    if (popts.primal_scale == 2) {
        copy_in(r->v, popts.v, d->n);
        r->popts.v = r->v.data();
    }
    r->sopts = *so;
    r->sopts.trace_host = nullptr;
    r->sopts.warm_start = 0;
    r->sopts.check_every = kTick;
    r->est_bytes = estimate_bytes(d, &popts);
    if (r->est_bytes > S->budget) {
        delete r;
        set_error("request needs about %zu bytes, more than the whole budget", estimate_bytes(d, &popts));
        return DL_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    r->t_submit = S->now();
    S->all[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
    S->cv.notify_all();
    return DL_OK;
}

extern "C" dl_status dl_server_poll(dl_server* S, uint64_t ticket, int32_t* done, dl_solve_result* out,
                                    double* lambda_host)
{
    if (!S || !done) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) { set_error("unknown ticket %llu", (unsigned long long)ticket); return DL_ERR_NOT_FOUND; }
    Request* r = it->second;
    *done = r->state == 4 ? 1 : 0;
    if (!*done) return DL_OK;
    if (out) *out = r->res;
    if (lambda_host && !r->lam_host.empty()) std::memcpy(lambda_host, r->lam_host.data(), r->lam_host.size() * 8);
    S->all.erase(it);
    delete r;
    return DL_OK;
}

extern "C" dl_status dl_server_times(dl_server* S, uint64_t ticket, double* ts, double* tb, double* td)
{
    if (!S) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) { set_error("unknown ticket"); return DL_ERR_NOT_FOUND; }
    if (ts) *ts = it->second->t_submit;
    if (tb) *tb = it->second->t_start;
    if (td) *td = it->second->t_done;
    return DL_OK;
}

extern "C" dl_status dl_server_destroy(dl_server* S)
{
    if (!S) return DL_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        // queued requests are dropped; running ones finish their solve
        for (Request* r : S->queue) {
            S->all.erase(r->ticket);
            delete r;
        }
        S->queue.clear();
        S->cv.notify_all();
    }
    for (auto& t : S->loaders) t.join();
    S->scheduler.join();
    S->reaper.join();   // exits once the scheduler is done and every retired problem is freed
    for (auto& kv : S->all) {
        if (kv.second->prob) dl_problem_destroy(kv.second->prob);
        if (kv.second->lam_dev) (void)hipFree(kv.second->lam_dev);
        delete kv.second;
    }
    delete S;
    return DL_OK;
}
