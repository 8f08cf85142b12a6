// Allocation-free dual evaluation: dl_dual_grad_noalloc.
//
// The same kernels as dl_dual_grad (lambda permutation, fused gradient,
// per-destination reduction, evaluation scalars), but every intermediate
// buffer of the evaluation -- the permuted lambda, the chunk partial sums, the
// FP64 accumulators of rows beyond LDS, the objective and block partials and
// the six scalars -- is carved from one file-scope device array instead of
// the buffers dl_problem_create allocated.  The call makes no allocation of
// any kind, so callers that cannot allocate (code under stream capture,
// serving loops that forbid it) can use it.
//
// The array lives once per device for the life of the process.  Host code
// never passes its name to a kernel: the name is a host-side stand-in, not a
// device address.  The device address is taken with hipGetSymbolAddress once
// per device (with that device current) and cached.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dualip.h"
#include "common.hpp"
#include "kernels.hpp"
#include "problem.hpp"

namespace {

constexpr size_t kScratchBytes = DL_NOALLOC_SCRATCH_BYTES;   // per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// the device address of `scratch` on `dev` (the current device)
hipError_t scratch_ptr(int dev, unsigned char** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!q) return hipErrorInvalidSymbol;
        g_ptr[dev] = q;
    }
    *out = (unsigned char*)g_ptr[dev];
    return hipSuccess;
}

__global__ void zero_f64_kernel(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// byte needs of one evaluation of p: permuted lambda, row accumulators,
// objective and block partials, scalars, chunk partial sums (3 planes when
// the scalars are requested, else 1)
static size_t noalloc_bytes(const dl_problem* p, int check, size_t* off)
{
    const size_t J = (size_t)p->J;
    const size_t K = (size_t)(p->K > 0 ? p->K : 1);
    size_t o = 0;
    off[0] = o; o = align256(o + J * sizeof(double));                                      // lambda
    off[1] = o; o = align256(o + 3 * J * sizeof(double));                                  // tail
    off[2] = o; o = align256(o + 3 * (size_t)p->nchunks * sizeof(double));                 // obj_part
    off[3] = o; o = align256(o + (size_t)p->nblk2 * dl::kRedStride * sizeof(double));      // blockpart
    off[4] = o; o = align256(o + 8 * sizeof(double));                                      // scalars
    off[5] = o; o = align256(o + (size_t)(check ? 3 : 1) * p->nchunks * K * (p->det ? 8 : 4));  // partials
    off[6] = o; o = align256(o + (p->nf > 1 ? J : 0) * sizeof(double));                   // row ratios
    off[7] = o; o = align256(o + (p->nf > 1 ? (size_t)p->nchunks : 0) * sizeof(double));   // restoration
    return o;
}

extern "C" dl_status dl_dual_grad_noalloc(dl_problem* p, const double* lambda_dev, double gamma,
                                          double* grad_dev, double* x_dev, dl_eval* eval_host,
                                          void* hip_stream)
{
    using dlh::set_error;
    if (!p || !lambda_dev || !grad_dev) { set_error("NULL argument"); return DL_ERR_INVALID_ARG; }
    if (!(gamma > 0.0) || !(gamma < INFINITY)) { set_error("gamma must be positive and finite"); return DL_ERR_INVALID_ARG; }
    if (p->device < 0 || p->device >= kMaxDevices) { set_error("device %d out of range", p->device); return DL_ERR_UNSUPPORTED; }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return dlh::hip_fail(e, "hipGetDevice");
    if (cur != p->device) {
        set_error("the current device (%d) is not the problem's device (%d)", cur, p->device);
        return DL_ERR_INVALID_ARG;
    }
    const int check = eval_host ? 1 : 0;
    size_t off[8];
    const size_t need = noalloc_bytes(p, check, off);
    if (need > kScratchBytes) {
        set_error("the evaluation needs %zu bytes of scratch; the static scratch holds %zu", need, kScratchBytes);
        return DL_ERR_UNSUPPORTED;
    }
    unsigned char* base = nullptr;
    if ((e = scratch_ptr(p->device, &base)) != hipSuccess) return dlh::hip_fail(e, "scratch symbol address");

    hipStream_t s = (hipStream_t)hip_stream;
    double* lam = (double*)(base + off[0]);
    double* tail = (double*)(base + off[1]);
    double* obj_part = (double*)(base + off[2]);
    double* blockpart = (double*)(base + off[3]);
    double* out6 = (double*)(base + off[4]);
    float* part = (float*)(base + off[5]);
    double* srow = (double*)(base + off[6]);
    double* corr = (double*)(base + off[7]);

    // the accumulators of rows beyond LDS must start at zero (the reduction
    // clears them after reading, but an earlier call may have stopped early)
    const int64_t nt = 3 * (int64_t)p->J;
    hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, tail, nt);
    if ((e = hipGetLastError()) != hipSuccess) return dlh::hip_fail(e, "clear scratch");
    if ((e = dl::launch_permute_in(lambda_dev, p->orig, p->J, lam, s)) != hipSuccess)
        return dlh::hip_fail(e, "permute lambda");
    dl::GradArgs g = dlh::grad_args(p, lam, nullptr, gamma, nullptr, x_dev);
    g.part = part;
    g.tail = tail;
    g.obj_part = obj_part;
    g.srow = srow;
    g.corr_part = corr;
    if ((e = dl::launch_grad(g, p->storage, check != 0, p->has_w != 0, p->has_cut != 0, s)) != hipSuccess)
        return dlh::hip_fail(e, "gradient kernel");
    dl::ReduceArgs r = dlh::reduce_args(p, check, 1, lam, nullptr, gamma, nullptr, grad_dev);
    r.part = part;
    r.tail = tail;
    r.blockpart = blockpart;
    if (r.srow) r.srow = srow;
    if ((e = dl::launch_reduce(r, p->nblk2, s)) != hipSuccess) return dlh::hip_fail(e, "reduce kernel");
    if (eval_host) {
        if (p->nf > 1) {
            // the gap's restoration over each edge's rows
            dl::GradArgs gr = g;
            gr.restore = 1;
            gr.X = nullptr;
            if ((e = dl::launch_grad(gr, p->storage, false, p->has_w != 0, p->has_cut != 0, s)) != hipSuccess)
                return dlh::hip_fail(e, "restoration pass");
        }
        if ((e = dl::launch_eval_finish(obj_part, p->nchunks, blockpart, p->nblk2, 1, gamma, out6, s,
                                        p->nf > 1 ? corr : nullptr)) != hipSuccess)
            return dlh::hip_fail(e, "evaluation kernel");
        double h[6];
        if ((e = hipMemcpyAsync(h, out6, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return dlh::hip_fail(e, "copy scalars");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return dlh::hip_fail(e, "synchronize");
        eval_host->g = h[0];
        eval_host->cx = h[1];
        eval_host->reg = h[2];
        eval_host->P = h[3];
        eval_host->rel_gap = h[4];
        eval_host->max_infeas = h[5];
    }
    return DL_OK;
}
