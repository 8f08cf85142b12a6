// dl_solve: accelerated dual ascent on one problem (see include/dualip.h).
//
// Each iteration is three kernels on the caller's stream: the fused gradient
// pass, the per-destination reduction and the one-workgroup ascent step.
// Every scalar the stopping test depends on stays on the device in FP64; the
// host only reads the stop flag.  Iterations are captured as a hipGraph of
// `seg` iterations (the gap check falls on the last one) and replayed; after
// a replay the state is copied to pinned memory and the host checks it one
// replay later, so the GPU never waits for the host.  Once the device sets
// the stop flag every later kernel returns at once.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "problem.hpp"

using namespace dl;
using dlh::hip_fail;
using dlh::set_error;

namespace {

struct Cleanup {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    double* trace = nullptr;
    std::vector<hipEvent_t> events;
    ~Cleanup()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (trace) (void)hipFree(trace);
        for (auto e : events) (void)hipEventDestroy(e);
    }
};

}  // namespace

#define TRY(call, what)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

extern "C" dl_status dl_solve(dl_problem* p, const dl_solve_opts* o, double* lam_inout, dl_solve_result* out,
                              void* hip_stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!p || !lam_inout || !out) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    dl_status st = dlh::check_solve_opts(o);
    if (st != DL_OK) return st;
    if (!p->solve_ok) {
        set_error("dl_solve needs a >= 0 and b >= 0 (the gap restoration scales x down)");
        return DL_ERR_UNSUPPORTED;
    }
    std::memset(out, 0, sizeof *out);
    hipStream_t s = (hipStream_t)hip_stream;
    const SolveParams prm = dlh::make_params(o, p);
    Cleanup cl;
    if (o->trace_host && o->max_iters > 0)
        TRY(hipMalloc(&cl.trace, (size_t)o->max_iters * DL_TRACE_W * sizeof(double)), "trace buffer");
    TRY(launch_solve_init(p->st, prm, o->warm_start ? lam_inout : nullptr, p->orig, p->D, p->J, p->lam, p->y,
                          p->yp, p->G, p->Gp, p->lam_eval, s),
        "init kernel");

    const int64_t N = o->max_iters;
    int64_t seg = o->graph_iters > 0 ? o->graph_iters : (o->check_every > 0 ? o->check_every : 16);
    if (o->check_every > 0 && seg % o->check_every != 0) seg = o->check_every;
    int64_t k = 0;
    double kernel_ms = 0.0, check_ms = 0.0;   // ordinary and gap-check gradient launches
    int64_t launches = 0, check_launches = 0;
    SolveState* hst = p->st_host;

    if (o->time_kernels) {
        // eager launches, HIP events around every fused gradient launch
        const int64_t W = 256;
        cl.events.resize((size_t)(2 * W + 2), nullptr);
        for (auto& e : cl.events) TRY(hipEventCreate(&e), "event");
        while (k < N) {
            const int64_t nb = std::min<int64_t>(W, N - k);
            std::vector<char> chk((size_t)nb);
            for (int64_t q = 0; q < nb; ++q, ++k) {
                chk[(size_t)q] = dlh::is_check_iter(o, k) ? 1 : 0;
                TRY(dlh::enqueue_iteration(p, prm, chk[(size_t)q], cl.trace, s, cl.events[2 * q],
                                           cl.events[2 * q + 1]),
                    "iteration");
            }
            TRY(hipMemcpyAsync(hst, p->st, sizeof(SolveState), hipMemcpyDeviceToHost, s), "copy state");
            TRY(hipStreamSynchronize(s), "synchronize");
            for (int64_t q = 0; q < nb; ++q) {
                float ms = 0.0f;
                TRY(hipEventElapsedTime(&ms, cl.events[2 * q], cl.events[2 * q + 1]), "elapsed");
                if (chk[(size_t)q]) {
                    check_ms += ms;
                    ++check_launches;
                } else {
                    kernel_ms += ms;
                    ++launches;
                }
            }
            if (hst->done) break;
        }
    } else {
        bool stop = false;
        const int64_t nfull = N / seg;
        if (nfull > 0) {
            // a graph of `seg` iterations: the problem's cached one when the
            // last solve captured it with the same parameters, else a new
            // capture (kept for the next solve unless it records a trace)
            // (the iteration cap is read from the device state, so solves of
            // different lengths share a graph)
            auto& gc = p->gc;
            SolveParams key = prm;
            key.max_iters = 0;
            const bool same = gc.exec && !cl.trace && gc.seg == seg && gc.check_every == o->check_every &&
                              std::memcmp(&gc.prm, &key, sizeof key) == 0;
            hipGraphExec_t exec = same ? gc.exec : nullptr;
            if (!exec) {
                TRY(hipStreamCreateWithFlags(&cl.cap, hipStreamNonBlocking), "capture stream");
                TRY(hipStreamBeginCapture(cl.cap, hipStreamCaptureModeThreadLocal), "begin capture");
                for (int64_t q = 0; q < seg; ++q) {
                    const int check = o->check_every > 0 && (q + 1) % o->check_every == 0;
                    hipError_t e = dlh::enqueue_iteration(p, prm, check, cl.trace, cl.cap, nullptr, nullptr);
                    if (e != hipSuccess) {
                        hipGraph_t gtmp = nullptr;
                        (void)hipStreamEndCapture(cl.cap, &gtmp);
                        if (gtmp) (void)hipGraphDestroy(gtmp);
                        return hip_fail(e, "capture iteration");
                    }
                }
                TRY(hipStreamEndCapture(cl.cap, &cl.graph), "end capture");
                TRY(hipGraphInstantiate(&cl.exec, cl.graph, nullptr, nullptr, 0), "instantiate graph");
                exec = cl.exec;
                if (!cl.trace) {
                    // hand the new graph to the problem (the old one is idle:
                    // solves on one problem do not overlap)
                    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
                    if (gc.graph) (void)hipGraphDestroy(gc.graph);
                    gc.exec = cl.exec;
                    gc.graph = cl.graph;
                    cl.exec = nullptr;
                    cl.graph = nullptr;
                    gc.seg = seg;
                    gc.check_every = o->check_every;
                    gc.prm = key;
                }
            }
            for (auto& e : gc.ev)
                if (!e) TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
            for (int64_t gi = 0; gi < nfull && !stop; ++gi) {
                TRY(hipGraphLaunch(exec, s), "graph launch");
                k += seg;
                const int slot = (int)(gi & 1);
                TRY(hipMemcpyAsync(hst + slot, p->st, sizeof(SolveState), hipMemcpyDeviceToHost, s), "copy state");
                TRY(hipEventRecord(gc.ev[slot], s), "record");
                if (gi >= 1) {
                    TRY(hipEventSynchronize(gc.ev[1 - slot]), "poll");
                    if (hst[1 - slot].done) stop = true;
                }
            }
        }
        // the remainder of max_iters that fills no whole graph (none once the
        // device has stopped: those launches would only return at once)
        for (; k < N && !stop; ++k)
            TRY(dlh::enqueue_iteration(p, prm, dlh::is_check_iter(o, k) ? 1 : 0, cl.trace, s, nullptr, nullptr),
                "iteration");
    }
    TRY(launch_solve_final(p->st, p->y, p->yp, p->orig, p->D, p->J, lam_inout, s), "final kernel");
    TRY(hipMemcpyAsync(hst, p->st, sizeof(SolveState), hipMemcpyDeviceToHost, s), "copy state");
    TRY(hipStreamSynchronize(s), "synchronize");
    const SolveState fs = *hst;
    if (o->trace_host && fs.k > 0)
        TRY(hipMemcpy(o->trace_host, cl.trace, (size_t)fs.k * DL_TRACE_W * sizeof(double), hipMemcpyDeviceToHost),
            "copy trace");
    out->converged = fs.converged;
    out->stage = fs.stage_eval;
    out->iters = fs.k;
    out->gamma = fs.gamma_eval;
    out->g = fs.g;
    out->P = fs.P;
    out->rel_gap = fs.rel_gap;
    out->max_infeas = fs.max_infeas;
    out->grad_kernel_ms = launches > 0 ? kernel_ms / (double)launches : 0.0;
    out->grad_launches = launches;
    out->check_kernel_ms = check_launches > 0 ? check_ms / (double)check_launches : 0.0;
    out->check_launches = check_launches;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (fs.status == 5) {
        set_error("non-finite dual objective at iteration %lld", (long long)fs.k);
        out->status = DL_ERR_NUMERIC;
    } else if (fs.converged) {
        out->status = DL_OK;
    } else {
        set_error("gap target not reached in %lld iterations", (long long)fs.k);
        out->status = DL_ERR_NOT_CONVERGED;
    }
    return out->status;
}
