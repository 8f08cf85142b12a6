// dl_batch_solve and the batched iteration driver (see batch.hpp).
#include "batch.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <tuple>

using namespace dl;
using dlh::hip_fail;
using dlh::set_error;

namespace dlh {

void BatchRunner::release()
{
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(gtab_);
    f(rtab_[0]);
    f(rtab_[1]);
    f(atab_[0]);
    f(atab_[1]);
    f(ctab_);
    f(rbt_);
    f(ndone_dev_);
    f(st_dev_);
    if (ndone_host_) (void)hipHostFree(ndone_host_);
    if (st_host_) (void)hipHostFree(st_host_);
    gtab_ = nullptr;
    rtab_[0] = rtab_[1] = nullptr;
    atab_[0] = atab_[1] = nullptr;
    ctab_ = rbt_ = nullptr;
    ndone_dev_ = ndone_host_ = nullptr;
    st_dev_ = nullptr;
    st_host_ = nullptr;
    st_cap_ = 0;
    for (size_t& c : cap_) c = 0;
    probs_.clear();
    groups_.clear();
}

// copies v into *dst, growing the allocation (by half again) only when it is
// too small: the server rebuilds its tables at every admission and
// retirement, and allocation calls cost more than the copies
template <typename T>
static hipError_t upload(T** dst, size_t* cap, const std::vector<T>& v, hipStream_t s)
{
    const size_t need = std::max<size_t>(1, v.size());
    if (*cap < need) {
        if (*dst) (void)hipFree(*dst);
        *dst = nullptr;
        *cap = 0;
        const size_t want = need + need / 2;
        hipError_t e = hipMalloc((void**)dst, want * sizeof(T));
        if (e != hipSuccess) {
            *dst = nullptr;
            return e;
        }
        *cap = want;
    }
    if (!v.empty()) return hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return hipSuccess;
}

dl_status BatchRunner::build(const std::vector<dl_problem*>& probs, const std::vector<SolveParams>& prm,
                             hipStream_t s)
{
    // the stream has no work of the previous tables in flight (callers build
    // between synchronized ticks), so their allocations are reused
    probs_ = probs;
    groups_.clear();
    const int n = (int)probs.size();
    std::vector<GradArgs> g(n);
    std::vector<ReduceArgs> r0(n), r1(n);
    std::vector<AgdArgs> a0(n), a1(n);
    for (int k = 0; k < n; ++k) {
        dl_problem* p = probs[k];
        g[k] = grad_args(p, p->lam_eval, &p->st->gamma, 0.0, &p->st->done, nullptr);
        r0[k] = reduce_args(p, 0, 0, p->lam_eval, &p->st->gamma, 0.0, &p->st->done, nullptr);
        r1[k] = reduce_args(p, 1, 0, p->lam_eval, &p->st->gamma, 0.0, &p->st->done, nullptr);
        a0[k] = agd_args(p, prm[k], 0, nullptr);
        a1[k] = agd_args(p, prm[k], 1, nullptr);
    }
    // groups by kernel variant (storage, weights, rows beyond LDS: the layout
    // of each problem matches its variant); the largest problems go first
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> by;
    for (int k = 0; k < n; ++k)
        by[{probs[k]->storage, probs[k]->has_w, probs[k]->K < probs[k]->J ? 1 : 0, probs[k]->has_cut,
            probs[k]->det}].push_back(k);
    std::vector<int2> ct, rb;
    for (auto& kv : by) {
        auto idx = kv.second;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return probs[a]->n > probs[b]->n; });
        Group G;
        G.storage = std::get<0>(kv.first);
        G.has_w = std::get<1>(kv.first);
        G.tail = std::get<2>(kv.first);
        G.cut = std::get<3>(kv.first);
        G.det = std::get<4>(kv.first);
        G.lds = 0;
        G.c0 = (int)ct.size();
        // round-robin over problems so long chunks of big problems start early
        int maxc = 0;
        for (int k : idx) {
            maxc = std::max(maxc, probs[k]->nchunks);
            const bool tl = probs[k]->K < probs[k]->J;
            G.lds = std::max({G.lds, grad_lds_bytes(probs[k]->K, probs[k]->Kc, false, tl, probs[k]->det != 0),
                              grad_lds_bytes(probs[k]->K, probs[k]->Kc, true, tl, probs[k]->det != 0)});
        }
        for (int c = 0; c < maxc; ++c)
            for (int k : idx)
                if (c < probs[k]->nchunks) ct.push_back(make_int2(k, c));
        G.nblocks = (int)ct.size() - G.c0;
        groups_.push_back(G);
    }
    for (int k = 0; k < n; ++k)
        for (int b = 0; b < probs[k]->nblk2; ++b) rb.push_back(make_int2(k, b));
    nrb_ = (int)rb.size();
    hipError_t e;
    if ((e = upload(&gtab_, &cap_[0], g, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = upload(&rtab_[0], &cap_[1], r0, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = upload(&rtab_[1], &cap_[2], r1, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = upload(&atab_[0], &cap_[3], a0, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = upload(&atab_[1], &cap_[4], a1, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = upload(&ctab_, &cap_[5], ct, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = upload(&rbt_, &cap_[6], rb, s)) != hipSuccess) return hip_fail(e, "batch tables");
    if (!ndone_dev_ && (e = hipMalloc((void**)&ndone_dev_, sizeof(int))) != hipSuccess) {
        ndone_dev_ = nullptr;
        return hip_fail(e, "batch flag");
    }
    if (!ndone_host_ && (e = hipHostMalloc((void**)&ndone_host_, sizeof(int), hipHostMallocDefault)) != hipSuccess) {
        ndone_host_ = nullptr;
        return hip_fail(e, "batch flag");
    }
    if (st_cap_ < (size_t)std::max(1, n)) {
        if (st_dev_) (void)hipFree(st_dev_);
        if (st_host_) (void)hipHostFree(st_host_);
        st_dev_ = nullptr;
        st_host_ = nullptr;
        st_cap_ = 0;
        const size_t want = (size_t)std::max(1, n) + (size_t)n / 2;
        if ((e = hipMalloc((void**)&st_dev_, want * sizeof(SolveState))) != hipSuccess) {
            st_dev_ = nullptr;
            return hip_fail(e, "batch states");
        }
        if ((e = hipHostMalloc((void**)&st_host_, want * sizeof(SolveState), hipHostMallocDefault)) != hipSuccess) {
            st_host_ = nullptr;
            return hip_fail(e, "batch states");
        }
        st_cap_ = want;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "batch tables");
    return DL_OK;
}

hipError_t BatchRunner::enqueue_iteration(int check, hipStream_t s) const
{
    hipError_t e;
    for (const Group& G : groups_)
        if ((e = launch_grad_batch(gtab_, ctab_ + G.c0, G.nblocks, G.lds, G.storage, check != 0, G.has_w != 0,
                                   G.tail != 0, G.cut != 0, G.det != 0, s)) != hipSuccess)
            return e;
    if ((e = launch_reduce_batch(rtab_[check ? 1 : 0], rbt_, nrb_, s)) != hipSuccess) return e;
    return launch_agd_batch(atab_[check ? 1 : 0], (int)probs_.size(), s);
}

hipError_t BatchRunner::count_done(hipStream_t s, int* ndone)
{
    hipError_t e = launch_count_done(atab_[0], (int)probs_.size(), ndone_dev_, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ndone_host_, ndone_dev_, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) *ndone = *ndone_host_;
    return e;
}

hipError_t BatchRunner::states(hipStream_t s, std::vector<SolveState>& out)
{
    out.resize(probs_.size());
    hipError_t e = launch_gather_states(atab_[0], (int)probs_.size(), st_dev_, s);
    if (e == hipSuccess && !out.empty())
        e = hipMemcpyAsync(st_host_, st_dev_, out.size() * sizeof(SolveState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && !out.empty()) std::memcpy(out.data(), st_host_, out.size() * sizeof(SolveState));
    return e;
}

}  // namespace dlh

namespace {
struct GraphHolder {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    ~GraphHolder()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};
}  // namespace

#define TRY(call, what)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

extern "C" dl_status dl_batch_solve(dl_problem* const* probs, int32_t count, const dl_solve_opts* o,
                                    double* const* lambdas, dl_solve_result* out, void* hip_stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!probs || count < 1 || !lambdas || !out) { set_error("invalid batch arguments"); return DL_ERR_INVALID_ARG; }
    dl_status st = dlh::check_solve_opts(o);
    if (st != DL_OK) return st;
    std::vector<dl_problem*> ps(probs, probs + count);
    for (int k = 0; k < count; ++k) {
        if (!ps[k] || !lambdas[k]) { set_error("NULL problem or lambda at %d", k); return DL_ERR_INVALID_ARG; }
        if (!ps[k]->solve_ok) { set_error("problem %d has a < 0 or b < 0", k); return DL_ERR_UNSUPPORTED; }
        if (ps[k]->nf > 1) { set_error("problem %d has columns with several entries: batched solves take one entry per column", k); return DL_ERR_UNSUPPORTED; }
        for (int q = 0; q < k; ++q)
            if (ps[q] == ps[k]) { set_error("problem %d appears twice in the batch", k); return DL_ERR_INVALID_ARG; }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<SolveParams> prms((size_t)count);
    for (int k = 0; k < count; ++k) prms[(size_t)k] = dlh::make_params(o, ps[k]);
    for (int k = 0; k < count; ++k) {
        dl_problem* p = ps[k];
        const SolveParams& prm = prms[(size_t)k];
        TRY(launch_solve_init(p->st, prm, o->warm_start ? lambdas[k] : nullptr, p->orig, p->D, p->J, p->lam, p->y,
                              p->yp, p->G, p->Gp, p->lam_eval, s),
            "init kernel");
    }
    // br_all: the tables of every problem (done count, final states);
    // iterations run on the tables of the problems still running, rebuilt
    // (and the graph captured again) whenever a quarter of them have
    // stopped, so that stopped problems no longer occupy the launches
    dlh::BatchRunner br_all, br_act;
    st = br_all.build(ps, prms, s);
    if (st != DL_OK) return st;
    dlh::BatchRunner* br = &br_all;
    int nact = count;
    const int64_t N = o->max_iters;
    int64_t seg = o->graph_iters > 0 ? o->graph_iters : (o->check_every > 0 ? o->check_every : 16);
    if (o->check_every > 0 && seg % o->check_every != 0) seg = o->check_every;
    int64_t k = 0;
    bool all_done = false;
    const int64_t nfull = N / seg;
    int64_t gi = 0;
    while (gi < nfull && !all_done) {
        GraphHolder gh;
        TRY(hipStreamCreateWithFlags(&gh.cap, hipStreamNonBlocking), "capture stream");
        TRY(hipStreamBeginCapture(gh.cap, hipStreamCaptureModeThreadLocal), "begin capture");
        for (int64_t q = 0; q < seg; ++q) {
            const int check = o->check_every > 0 && (q + 1) % o->check_every == 0;
            hipError_t e = br->enqueue_iteration(check, gh.cap);
            if (e != hipSuccess) {
                hipGraph_t gtmp = nullptr;
                (void)hipStreamEndCapture(gh.cap, &gtmp);
                if (gtmp) (void)hipGraphDestroy(gtmp);
                return hip_fail(e, "capture batch iteration");
            }
        }
        TRY(hipStreamEndCapture(gh.cap, &gh.graph), "end capture");
        TRY(hipGraphInstantiate(&gh.exec, gh.graph, nullptr, nullptr, 0), "instantiate graph");
        bool rebuild = false;
        for (; gi < nfull && !rebuild; ++gi) {
            TRY(hipGraphLaunch(gh.exec, s), "graph launch");
            k += seg;
            // poll every few replays (the check itself waits for the stream)
            if ((gi & 3) == 3 || gi == nfull - 1) {
                int nd = 0;
                TRY(br_all.count_done(s, &nd), "poll");
                if (nd == count) {
                    all_done = true;
                    ++gi;
                    break;
                }
                rebuild = 4 * (count - nd) <= 3 * nact;
            }
        }
        if (rebuild) {
            std::vector<SolveState> fs;
            TRY(br_all.states(s, fs), "read states");
            std::vector<dl_problem*> act;
            std::vector<SolveParams> aprm;
            for (int q = 0; q < count; ++q)
                if (!fs[q].done) {
                    act.push_back(ps[q]);
                    aprm.push_back(prms[(size_t)q]);
                }
            st = br_act.build(act, aprm, s);
            if (st != DL_OK) return st;
            br = &br_act;
            nact = (int)act.size();
        }
    }
    // the remainder of max_iters that fills no whole graph (none once every
    // problem has stopped)
    for (; k < N && !all_done; ++k)
        TRY(br->enqueue_iteration(dlh::is_check_iter(o, k) ? 1 : 0, s), "batch iteration");
    for (int q = 0; q < count; ++q) {
        dl_problem* p = ps[q];
        TRY(launch_solve_final(p->st, p->y, p->yp, p->orig, p->D, p->J, lambdas[q], s), "final kernel");
    }
    std::vector<SolveState> fs;
    TRY(br_all.states(s, fs), "read states");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    dl_status worst = DL_OK;
    for (int q = 0; q < count; ++q) {
        dl_solve_result& r = out[q];
        std::memset(&r, 0, sizeof r);
        r.converged = fs[q].converged;
        r.stage = fs[q].stage_eval;
        r.iters = fs[q].k;
        r.gamma = fs[q].gamma_eval;
        r.g = fs[q].g;
        r.P = fs[q].P;
        r.rel_gap = fs[q].rel_gap;
        r.max_infeas = fs[q].max_infeas;
        r.seconds = secs;
        r.status = fs[q].status == 5 ? DL_ERR_NUMERIC : (fs[q].converged ? DL_OK : DL_ERR_NOT_CONVERGED);
        if (r.status != DL_OK && worst == DL_OK) worst = r.status;
    }
    if (worst != DL_OK) set_error("some problems did not converge");
    return worst;
}
