// HIP kernels of libdualip for CDNA4 (gfx950) other than the fused gradient
// (grad_impl.hpp, instantiated per storage type): the per-destination
// combination of the chunk partial sums, the FP64 scalar reductions, the
// accelerated ascent step (Appendix B) with its stop test and gamma stages
// (Section 5), and small helpers.  Their work is O(m); the O(nnz) pass is the
// gradient kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "kernels.hpp"
#include "lanes.hpp"

namespace dl {

template <typename VT, bool CUT, bool DET>
hipError_t launch_grad_vt(const GradArgs& a, bool check, bool has_w, hipStream_t s);
template <typename VT, bool CUT, bool DET>
hipError_t set_grad_attributes_vt(size_t lds);
template <typename VT, bool CUT, bool DET>
hipError_t launch_grad_batch_vt(const GradArgs* tab, const int2* ct, int nblocks, size_t lds, bool check,
                                bool has_w, bool tail, hipStream_t s);

// kernel variants: plain, with capped-simplex blocks (cut), deterministic
// (det: integer sums; also handles capped blocks)
template <typename VT>
static hipError_t launch_grad_batch_s(const GradArgs* tab, const int2* ct, int nblocks, size_t lds, bool check,
                                      bool has_w, bool tail, bool cut, bool det, hipStream_t s)
{
    if (det) return launch_grad_batch_vt<VT, true, true>(tab, ct, nblocks, lds, check, has_w, tail, s);
    if (cut) return launch_grad_batch_vt<VT, true, false>(tab, ct, nblocks, lds, check, has_w, tail, s);
    return launch_grad_batch_vt<VT, false, false>(tab, ct, nblocks, lds, check, has_w, tail, s);
}

hipError_t launch_grad_batch(const GradArgs* tab, const int2* ct, int nblocks, size_t lds, int storage,
                             bool check, bool has_w, bool tail, bool cut, bool det, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    switch (storage) {
    case 0: return launch_grad_batch_s<double>(tab, ct, nblocks, lds, check, has_w, tail, cut, det, s);
    case 1: return launch_grad_batch_s<float>(tab, ct, nblocks, lds, check, has_w, tail, cut, det, s);
    default: return launch_grad_batch_s<uint16_t>(tab, ct, nblocks, lds, check, has_w, tail, cut, det, s);
    }
}

size_t grad_lds_bytes(int K, int Kc, bool check, bool tail, bool det)
{
    const size_t base = 4 * kWaves * sizeof(double);
    const size_t es = det ? 8 : 4;
    // ordinary passes: lam and the a x sum per row, 8 bytes (FP64 without
    // rows beyond K, or a 64-bit integer in deterministic mode) or f32
    if (!check) return base + (size_t)K * (sizeof(double) + ((det || !tail) ? 8 : 4));
    if (tail) return base + (size_t)K * es + (size_t)Kc * 2 * es;
    return base + (size_t)K * (sizeof(double) + es) + (size_t)Kc * 2 * es;
}

template <typename VT>
static hipError_t launch_grad_s(const GradArgs& a, bool check, bool has_w, bool cut, hipStream_t s)
{
    if (a.det) return launch_grad_vt<VT, true, true>(a, check, has_w, s);
    if (cut) return launch_grad_vt<VT, true, false>(a, check, has_w, s);
    return launch_grad_vt<VT, false, false>(a, check, has_w, s);
}

template <typename VT>
hipError_t launch_grad_mf_vt(const GradArgs& a, bool has_w, hipStream_t s);
template <typename VT>
hipError_t set_grad_mf_attributes_vt(size_t lds);

hipError_t launch_grad_mf(const GradArgs& a, int storage, bool has_w, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
    switch (storage) {
    case 0: return launch_grad_mf_vt<double>(a, has_w, s);
    case 1: return launch_grad_mf_vt<float>(a, has_w, s);
    default: return launch_grad_mf_vt<uint16_t>(a, has_w, s);
    }
}

hipError_t launch_grad(const GradArgs& a, int storage, bool check, bool has_w, bool cut, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
    // columns with several entries: the multi-entry kernel (it keeps the
    // c x sum on every pass; the gap's restoration is a pass of its own)
    if (a.nf > 1) return launch_grad_mf(a, storage, has_w, s);
    switch (storage) {
    case 0: return launch_grad_s<double>(a, check, has_w, cut, s);
    case 1: return launch_grad_s<float>(a, check, has_w, cut, s);
    default: return launch_grad_s<uint16_t>(a, check, has_w, cut, s);
    }
}

template <typename VT>
static hipError_t set_grad_attributes_s(size_t lds)
{
    hipError_t e = hipSuccess, r;
    if ((r = set_grad_attributes_vt<VT, false, false>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_attributes_vt<VT, true, false>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_attributes_vt<VT, true, true>(lds)) != hipSuccess) e = r;
    return e;
}

hipError_t set_grad_attributes(size_t lds)
{
    hipError_t e = hipSuccess, r;
    if ((r = set_grad_attributes_s<double>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_attributes_s<float>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_attributes_s<uint16_t>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_mf_attributes_vt<double>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_mf_attributes_vt<float>(lds)) != hipSuccess) e = r;
    if ((r = set_grad_mf_attributes_vt<uint16_t>(lds)) != hipSuccess) e = r;
    return e;
}

// ---------------------------------------------------------------------------
// per-destination combination of the chunk partials (fixed order)
// ---------------------------------------------------------------------------
// a workgroup takes 64 rows; each row's chunk partials are split into
// kRedSlices slices read by separate waves (all loads of a slice in flight
// together), then combined in slice order
constexpr int kRedSlices = 16;
constexpr int kRedThreads = 64 * kRedSlices;

// the per-row inputs of the finishing wave, read before the partial sums so
// that both sets of loads are in flight together
struct RowIn {
    double b, lam, D, Gp, y, yp;
    int32_t orig;
};

__device__ __forceinline__ RowIn row_inputs(const ReduceArgs& r, const int j)
{
    RowIn in{};
    if (j < r.J) {
        in.b = r.b[j];
        in.lam = r.lam[j];
        if (r.mode == 1) {
            in.orig = r.orig[j];
        } else {
            in.D = r.D[j];
            in.Gp = r.Gp[j];
            in.y = r.y[j];
            in.yp = r.yp[j];
        }
    }
    return in;
}

// wave 0: per-row gradient and the block's scalar sums
__device__ __forceinline__ void reduce_finish(const ReduceArgs& r, const int blk, const int l, const int j,
                                              const double (*sh)[kRedSlices][64], const RowIn& in)
{
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < r.J) {
        const double gamma = r.gamma_ptr ? *r.gamma_ptr : r.gamma_val;
        double ax = 0.0, cj = 0.0, qj = 0.0;
        // a global accumulator (an integer in deterministic mode), cleared
        // for the next pass
        auto take = [&](int64_t idx, int plane) {
            const double v = r.det ? (double)((const long long*)r.tail)[idx] * r.iqs[plane] : r.tail[idx];
            r.tail[idx] = 0.0;
            return v;
        };
        if (j < r.K) {
            for (int i = 0; i < kRedSlices; ++i) ax += sh[0][i][l];
        } else {
            ax = take(j, 0);
        }
        if (j < r.Kc) {
            if (r.check) {
                for (int i = 0; i < kRedSlices; ++i) {
                    cj += sh[1][i][l];
                    qj += sh[2][i][l];
                }
            }
        } else {
            cj = take(r.J + j, 1);
            qj = take(2 * (int64_t)r.J + j, 2);
        }
        const double bj = in.b;
        const double res = ax - bj;
        S[0] = in.lam * bj;
        if (r.mode == 1) {
            r.grad_out[in.orig] = res;
        } else {
            const double Gj = in.D * res;
            r.G[j] = Gj;
            S[1] = Gj * Gj;
            const double dg = Gj - in.Gp;
            S[2] = dg * dg;
            const double dy = in.y - in.yp;
            S[3] = dy * dy;
        }
        if (r.check) {
            const double sj = ax > bj ? bj / ax : 1.0;
            if (r.srow) r.srow[j] = sj;
            S[4] = (sj - 1.0) * cj + 0.5 * gamma * (sj * sj - 1.0) * qj;
            S[5] = res > 0.0 ? res : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) S[i] = wave_sum(S[i]);
    S[5] = wave_max(S[5]);
    if (l == 0) {
        double* out = r.blockpart + (int64_t)blk * kRedStride;
#pragma unroll
        for (int i = 0; i < 6; ++i) out[i] = S[i];
    }
}

// all threads of the workgroup return from it (the row part runs on wave 0)
__device__ __forceinline__ void reduce_rows(const ReduceArgs& r, const int blk)
{
    __shared__ double sh[3][kRedSlices][64];
    const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int j = blk * 64 + l;
    const int planes = r.check ? 3 : 1;
    const int64_t plane = (int64_t)r.nchunks * r.K;
    RowIn in{};
    if (q == 0) in = row_inputs(r, j);
    for (int p = 0; p < planes; ++p) {
        double acc = 0.0;
        if (r.det && j < (p == 0 ? r.K : r.Kc)) {
            // integer partials: exact sums, converted once per slice
            const int c0 = (int)(((int64_t)r.nchunks * q) / kRedSlices);
            const int c1 = (int)(((int64_t)r.nchunks * (q + 1)) / kRedSlices);
            const long long* col = (const long long*)r.part + p * plane + j;
            long long ia = 0;
            for (int c = c0; c < c1; ++c) ia += col[(int64_t)c * r.K];
            acc = (double)ia * r.iqs[p];
        } else if (j < (p == 0 ? r.K : r.Kc)) {
            const int c0 = (int)(((int64_t)r.nchunks * q) / kRedSlices);
            const int c1 = (int)(((int64_t)r.nchunks * (q + 1)) / kRedSlices);
            const float* col = r.part + p * plane + j;
            int c = c0;
            for (; c + 16 <= c1; c += 16) {
                float v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = col[(int64_t)(c + u) * r.K];
#pragma unroll
                for (int u = 0; u < 16; ++u) acc += (double)v[u];
            }
            for (; c + 4 <= c1; c += 4) {
                float v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = col[(int64_t)(c + u) * r.K];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += (double)v[u];
            }
            for (; c < c1; ++c) acc += (double)col[(int64_t)c * r.K];
        }
        sh[p][q][l] = acc;
    }
    __syncthreads();
    if (q == 0) reduce_finish(r, blk, l, j, sh, in);
}

__device__ __forceinline__ void reduce_body(const ReduceArgs& r, const int blk)
{
    if (r.done && *r.done) return;
    reduce_rows(r, blk);
}

__global__ __launch_bounds__(kRedThreads) void reduce_kernel(ReduceArgs r) { reduce_body(r, blockIdx.x); }

// batched form: block b reduces row block rt[b].y of problem rt[b].x
__global__ __launch_bounds__(kRedThreads) void reduce_kernel_batch(const ReduceArgs* __restrict__ tab,
                                                           const int2* __restrict__ rt)
{
    // the arguments stay in memory (a copy would be indexed by the plane and
    // go to scratch)
    const int2 e = rt[blockIdx.x];
    reduce_body(tab[e.x], e.y);
}

hipError_t launch_reduce(const ReduceArgs& a, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(nblk), dim3(kRedThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const ReduceArgs* tab, const int2* rt, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel_batch, dim3(nblocks), dim3(kRedThreads), 0, s, tab, rt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deterministic block reduction of the scalars (all threads of one WG)
// ---------------------------------------------------------------------------
// the scalar kernels run one workgroup of kScalarThreads threads
constexpr int kScalarThreads = 1024;
constexpr int kSW = kScalarThreads / 64;

__device__ __forceinline__ void reduce_scalars(const double* obj_part, int nchunks, const double* bp,
                                               int nblk, double* out /*[9] shared*/,
                                               double* red /*[9*kSW] shared*/, const double* corr)
{
    // out: 0 sum t x, 1 sum v^2 x^2, 2 sum c x, 3..7 block sums 0..4 (7: the
    // gap's restoration correction, plus the per-chunk corrections of a
    // restoration pass when corr is given), 8 max of block value 5
    double v[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nchunks; i += blockDim.x) {
        v[0] += obj_part[3 * i];
        v[1] += obj_part[3 * i + 1];
        v[2] += obj_part[3 * i + 2];
        if (corr) v[7] += corr[i];
    }
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 5; ++k) v[3 + k] += bp[(int64_t)i * kRedStride + k];
        v[8] = fmax(v[8], bp[(int64_t)i * kRedStride + 5]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = wave_sum(v[k]);
    v[8] = wave_max(v[8]);
    const int w = threadIdx.x >> 6;
    const int nw = (int)(blockDim.x >> 6);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 9; ++k) red[k * kSW + w] = v[k];
    __syncthreads();
    // thread k combines scalar k over the waves, in wave order
    if (threadIdx.x < 9) {
        const int k = threadIdx.x;
        double a = 0.0;
        for (int i = 0; i < nw; ++i) a = k == 8 ? fmax(a, red[k * kSW + i]) : a + red[k * kSW + i];
        out[k] = a;
    }
    __syncthreads();
}

// evaluation scalars: g, c'x, gamma/2 |D_v x|^2, P, rel_gap, max_infeas
__global__ __launch_bounds__(kScalarThreads) void eval_finish_kernel(const double* obj_part, int nchunks,
                                                                     const double* bp, int nblk, int check,
                                                                     double gamma, double* out6,
                                                                     const double* corr)
{
    __shared__ double red[9 * kSW];
    __shared__ double v[9];
    reduce_scalars(obj_part, nchunks, bp, nblk, v, red, check ? corr : nullptr);
    if (threadIdx.x == 0) {
        const double reg = 0.5 * gamma * v[1];
        const double g = -v[0] + reg - v[3];
        out6[0] = g;
        out6[1] = check ? v[2] : NAN;
        out6[2] = reg;
        double P = NAN, rel = NAN;
        if (check) {
            P = v[2] + reg + v[7];
            rel = (P - g) / fmax(1.0, fabs(g));
        }
        out6[3] = P;
        out6[4] = rel;
        out6[5] = check ? v[8] : NAN;
    }
}

hipError_t launch_eval_finish(const double* obj_part, int nchunks, const double* blockpart, int nblk,
                              int check, double gamma, double* out6, hipStream_t s, const double* corr_part)
{
    hipLaunchKernelGGL(eval_finish_kernel, dim3(1), dim3(kScalarThreads), 0, s, obj_part, nchunks, blockpart,
                       nblk, check, gamma, out6, corr_part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// accelerated ascent step (one workgroup): scalars, step size, stop test,
// gamma stage, projected step and momentum on lam'
// ---------------------------------------------------------------------------
// scalar half of the step (all threads of one workgroup): the reduced
// scalars, the step size, the stop test and the stage logic; sc receives
// eta, beta, advance, stop (shared memory).  TEST_DONE: the caller has not
// tested st->done; it is read with the state (a stopped solve's partial sums
// are read and ignored) and a stopped solve gets stop = 1 and no update.
template <bool TEST_DONE>
__device__ __forceinline__ void agd_scalars(const AgdArgs& a, double* sc)
{
    SolveState* st = a.st;
    __shared__ double red[9 * kSW];
    __shared__ double v[9];
    // thread 0 reads the state before the reductions, so its loads overlap them
    double cur_gamma = 0.0, cur_eta = 0.0, cur_eta_cap = 0.0, cur_tm = 0.0;
    int64_t cur_k = 0, cur_ks = 0, cur_kmax = 0;
    int32_t cur_stage = 0, cur_done = 0;
    if (threadIdx.x == 0) {
        if (TEST_DONE) cur_done = st->done;
        cur_kmax = st->kmax;
        cur_gamma = st->gamma;
        cur_eta = st->eta;
        cur_eta_cap = st->eta_cap;
        cur_tm = st->tm;
        cur_k = st->k;
        cur_ks = st->ks;
        cur_stage = st->stage;
    }
    reduce_scalars(a.obj_part, a.nchunks, a.blockpart, a.nblk, v, red, a.check ? a.corr_part : nullptr);
    const SolveParams& P = a.prm;
    if (TEST_DONE && threadIdx.x == 0 && cur_done) {
        sc[0] = 0.0;
        sc[1] = 0.0;
        sc[2] = 0.0;
        sc[3] = 1.0;
    } else if (threadIdx.x == 0) {
        const int64_t k = cur_k;
        const int64_t ks = cur_ks;
        const double gamma = cur_gamma;
        const double reg = 0.5 * gamma * v[1];
        const double g = -v[0] + reg - v[3];
        const double obj = v[2] + reg;
        double eta = cur_eta;
        if (P.adaptive) {
            if (ks > 0 && v[6] > 0.0) {
                const double Lh = sqrt(v[5]) / sqrt(v[6]);
                eta = (Lh > 0.0 && 1.0 / Lh < cur_eta_cap) ? 1.0 / Lh : cur_eta_cap;
            }
        } else {
            eta = cur_eta_cap;
        }
        double rel = NAN;
        st->g = g;
        st->obj = obj;
        st->gamma_eval = gamma;
        st->stage_eval = cur_stage;
        st->gnorm = sqrt(v[4]);
        if (a.check) {
            const double Pv = obj + v[7];
            rel = (Pv - g) / fmax(1.0, fabs(g));
            st->P = Pv;
            st->rel_gap = rel;
            st->max_infeas = v[8];
        }
        if (a.trace) {
            double* row = a.trace + k * 6;
            row[0] = g;
            row[1] = rel;
            row[2] = eta;
            row[3] = gamma;
            row[4] = (double)cur_stage;
            row[5] = sqrt(v[4]);
        }
        double stop = 0.0, advance = 0.0, beta = 0.0;
        if (!isfinite(g)) {
            st->status = 5;
            st->done = 1;
            stop = 1.0;
        } else {
            const int last = cur_stage == P.n_stages - 1;
            if (a.check && last && rel <= P.tol) {
                st->converged = 1;
                st->done = 1;
                st->k = k + 1;
                stop = 1.0;
            } else {
                const double tm = cur_tm;
                const double tn = P.momentum ? 0.5 * (1.0 + sqrt(1.0 + 4.0 * tm * tm)) : 1.0;
                beta = P.momentum ? (tm - 1.0) / tn : 0.0;
                if (!last) {
                    if (P.stage_iters > 0 && ks + 1 >= P.stage_iters) advance = 1.0;
                    if (a.check && P.stage_tol > 0.0 && rel <= P.stage_tol) advance = 1.0;
                }
                st->eta = eta;
                if (advance != 0.0) {
                    const double gnew = P.gamma0 * pow(P.gamma_final / P.gamma0,
                                                       (double)(cur_stage + 1) / (double)(P.n_stages - 1));
                    st->eta = eta * gnew / gamma;
                    st->eta_cap = P.max_step * gnew / P.gamma0;
                    st->gamma = gnew;
                    st->stage = cur_stage + 1;
                    st->tm = 1.0;
                    st->ks = 0;
                } else {
                    st->tm = tn;
                    st->ks = ks + 1;
                }
                st->k = k + 1;
                if (k + 1 >= cur_kmax) st->done = 1;
            }
        }
        sc[0] = eta;
        sc[1] = beta;
        sc[2] = advance;
        sc[3] = stop;
    }
    __syncthreads();
}

// row half of the step: projected ascent step and momentum on rows
// j0, j0 + stride, ... (four rows per thread in flight at once)
__device__ __forceinline__ void agd_row(const AgdArgs& a, const int j, const double yj, const double Gj,
                                        const double lj, const double Dj, const double eta, const double beta,
                                        const bool adv)
{
    double ln = yj + eta * Gj;
    ln = ln > 0.0 ? ln : 0.0;
    double yn;
    if (adv) {
        yn = ln;
    } else {
        const double z = ln + beta * (ln - lj);
        yn = z > 0.0 ? z : 0.0;
    }
    a.yp[j] = yj;
    a.Gp[j] = Gj;
    a.lam[j] = ln;
    a.y[j] = yn;
    a.lam_eval[j] = Dj * yn;
}

__device__ __forceinline__ void agd_rows(const AgdArgs& a, const double eta, const double beta, const bool adv,
                                         const int j0, const int stride)
{
    int j = j0;
    for (; j + 3 * stride < a.J; j += 4 * stride) {
        double yv[4], gv[4], lv[4], dv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = j + u * stride;
            yv[u] = a.y[i];
            gv[u] = a.G[i];
            lv[u] = a.lam[i];
            dv[u] = a.D[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) agd_row(a, j + u * stride, yv[u], gv[u], lv[u], dv[u], eta, beta, adv);
    }
    for (; j < a.J; j += stride) agd_row(a, j, a.y[j], a.G[j], a.lam[j], a.D[j], eta, beta, adv);
}

// single problem: the scalar kernel (one workgroup) leaves the step in the
// solve state, the row kernel applies it with one thread per row
__global__ __launch_bounds__(kScalarThreads) void agd_scalar_kernel(AgdArgs a)
{
    SolveState* st = a.st;
    __shared__ double sc[4];
    agd_scalars<true>(a, sc);
    if (threadIdx.x == 0) {
        st->step_eta = sc[0];
        st->step_beta = sc[1];
        st->step_adv = sc[2] != 0.0 ? 1 : 0;
        st->step_stop = sc[3] != 0.0 ? 1 : 0;
    }
}

constexpr int kRowThreads = 256;

__global__ __launch_bounds__(kRowThreads) void agd_row_kernel(AgdArgs a)
{
    const SolveState* st = a.st;
    // the thread's first row is read together with the step (reading it is
    // harmless when no step is taken); further rows, if the grid is smaller
    // than J, go through the loop
    const int j = blockIdx.x * kRowThreads + threadIdx.x;
    const int stride = gridDim.x * kRowThreads;
    double yv = 0.0, gv = 0.0, lv = 0.0, dv = 0.0;
    if (j < a.J) {
        yv = a.y[j];
        gv = a.G[j];
        lv = a.lam[j];
        dv = a.D[j];
    }
    const int32_t stop = st->step_stop;
    const double eta = st->step_eta, beta = st->step_beta;
    const bool adv = st->step_adv != 0;
    if (stop) return;
    if (j < a.J) agd_row(a, j, yv, gv, lv, dv, eta, beta, adv);
    if (j + stride < a.J) agd_rows(a, eta, beta, adv, j + stride, stride);
}

// small problems: both halves in one workgroup (one launch less per iteration)
constexpr int kAgdFusedRows = 4096;

__global__ __launch_bounds__(kScalarThreads) void agd_fused_kernel(AgdArgs a)
{
    if (a.st->done) return;
    __shared__ double sc[4];
    agd_scalars<false>(a, sc);
    if (sc[3] != 0.0) return;
    agd_rows(a, sc[0], sc[1], sc[2] != 0.0, threadIdx.x, blockDim.x);
}

hipError_t launch_agd(const AgdArgs& a, hipStream_t s)
{
    if (a.J <= kAgdFusedRows) {
        hipLaunchKernelGGL(agd_fused_kernel, dim3(1), dim3(kScalarThreads), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(agd_scalar_kernel, dim3(1), dim3(kScalarThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb = a.J > 0 ? (a.J + kRowThreads - 1) / kRowThreads : 1;
    hipLaunchKernelGGL(agd_row_kernel, dim3(nb), dim3(kRowThreads), 0, s, a);
    return hipGetLastError();
}

// batched form: workgroup b steps problem b (both halves in one workgroup)
__global__ __launch_bounds__(kScalarThreads) void agd_kernel_batch(const AgdArgs* __restrict__ tab)
{
    const AgdArgs a = tab[blockIdx.x];
    if (a.st->done) return;
    __shared__ double sc[4];
    agd_scalars<false>(a, sc);
    if (sc[3] != 0.0) return;
    agd_rows(a, sc[0], sc[1], sc[2] != 0.0, threadIdx.x, blockDim.x);
}

hipError_t launch_agd_batch(const AgdArgs* tab, int count, hipStream_t s)
{
    hipLaunchKernelGGL(agd_kernel_batch, dim3(count), dim3(kScalarThreads), 0, s, tab);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void permute_in_kernel(const double* src, const int32_t* orig, int J, double* dst)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < J) dst[j] = src[orig[j]];
}

hipError_t launch_permute_in(const double* src, const int32_t* orig, int J, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(permute_in_kernel, dim3((J + 255) / 256), dim3(256), 0, s, src, orig, J, dst);
    return hipGetLastError();
}

__global__ void solve_init_kernel(SolveState* st, SolveParams prm, const double* lam_in,
                                  const int32_t* orig, const double* D, int J, double* lam, double* y,
                                  double* yp, double* G, double* Gp, double* lam_eval)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < J) {
        double v = 0.0;
        if (lam_in) {
            v = lam_in[orig[j]] / D[j];
            v = v > 0.0 ? v : 0.0;
        }
        lam[j] = v;
        y[j] = v;
        yp[j] = v;
        G[j] = 0.0;
        Gp[j] = 0.0;
        lam_eval[j] = D[j] * v;
    }
    if (j == 0) {
        st->gamma = prm.gamma0;
        st->eta = prm.init_step;
        st->eta_cap = prm.max_step;
        st->tm = 1.0;
        st->g = NAN;
        st->P = NAN;
        st->rel_gap = NAN;
        st->max_infeas = NAN;
        st->gnorm = NAN;
        st->obj = NAN;
        st->gamma_eval = prm.gamma0;
        st->stage_eval = 0;
        st->k = 0;
        st->ks = 0;
        st->kmax = prm.max_iters;
        st->stage = 0;
        st->done = prm.max_iters <= 0 ? 1 : 0;
        st->converged = 0;
        st->status = 0;
    }
}

hipError_t launch_solve_init(SolveState* st, SolveParams prm, const double* lam_in, const int32_t* orig,
                             const double* D, int J, double* lam, double* y, double* yp, double* G,
                             double* Gp, double* lam_eval, hipStream_t s)
{
    hipLaunchKernelGGL(solve_init_kernel, dim3((J + 255) / 256), dim3(256), 0, s, st, prm, lam_in, orig,
                       D, J, lam, y, yp, G, Gp, lam_eval);
    return hipGetLastError();
}

// lam_out (original rows, caller units) = D * (y if converged or no step was
// taken, else y_prev): the last point whose g and gap were evaluated
__global__ void solve_final_kernel(const SolveState* st, const double* y, const double* yp,
                                   const int32_t* orig, const double* D, int J, double* lam_out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < J) {
        const bool use_y = st->converged || st->k == 0;
        lam_out[orig[j]] = D[j] * (use_y ? y[j] : yp[j]);
    }
}

hipError_t launch_solve_final(const SolveState* st, const double* y, const double* yp,
                              const int32_t* orig, const double* D, int J, double* lam_out, hipStream_t s)
{
    hipLaunchKernelGGL(solve_final_kernel, dim3((J + 255) / 256), dim3(256), 0, s, st, y, yp, orig, D, J,
                       lam_out);
    return hipGetLastError();
}

// number of finished problems of a batch (one workgroup)
__global__ __launch_bounds__(256) void count_done_kernel(const AgdArgs* __restrict__ tab, int count, int* out)
{
    __shared__ int part[256];
    int n = 0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) n += tab[i].st->done ? 1 : 0;
    part[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
        *out = t;
    }
}

hipError_t launch_count_done(const AgdArgs* tab, int count, int* out, hipStream_t s)
{
    hipLaunchKernelGGL(count_done_kernel, dim3(1), dim3(256), 0, s, tab, count, out);
    return hipGetLastError();
}

// copies every problem's state into one contiguous array
__global__ void gather_states_kernel(const AgdArgs* __restrict__ tab, int count, SolveState* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = *tab[i].st;
}

hipError_t launch_gather_states(const AgdArgs* tab, int count, SolveState* out, hipStream_t s)
{
    hipLaunchKernelGGL(gather_states_kernel, dim3((count + 63) / 64), dim3(64), 0, s, tab, count, out);
    return hipGetLastError();
}

}  // namespace dl
