// Fused dual-gradient kernel for LPs whose columns have several entries:
// several matching families (Definition 1, Section 3.2: an edge (i, j) enters
// row k J + j of every family k) and dense rows such as the global count
// constraint sum_e x_e <= cap (Section 4).  Included once per storage type by
// grad_mf_{f32,bf16,f64}.hip.
//
// Each edge carries nf <= kMfPlanes entries (a_f, r_f), held in planes (plane
// 0 in the single-family arrays a and dst, the others in A2/dst2); columns
// with fewer entries are padded with a = 0.  One pass per evaluation:
//   t_e = -(c_e + sum_f a_f lam_{r_f}),  x = blockwise projection of t
//   (simplex, box or capped simplex, the thresholds of the one-family
//   kernel), and a_f x_e added to row r_f for every f.
// Rows are relabelled by degree, so a dense row (present in every column) is
// row 0 and lives in LDS; its plane's terms are summed per lane and added
// once per wave.  Work items are the one-family layout's, with at most
// kMfLaneCap edges on one lane and kMfRmax rows per lane (the planes
// multiply the registers per edge), segments on 2..64 lanes with register
// classes of 4 or kMfRmax rows; longer blocks take one workgroup that
// re-reads the block from L2 on every pass of its threshold.
//
// Restore mode (g.restore = 1, on gap-check iterations after the reduction
// has written s_j = min(1, b_j / (A x)_j) per row): x is recomputed and each
// edge is scaled by the smallest s over its rows, the feasible restoration of
// the duality gap; the pass adds (s_e - 1) c_e x_e + gamma/2 (s_e^2 - 1)
// v_e^2 x_e^2 per chunk to corr_part and touches no row sums.
#pragma once
#include "grad_impl.hpp"

namespace dl {

// adds a x to row j: FP64 LDS sums for the first K rows (every variant of
// this kernel: an active column adds to several rows, and the LDS's f32
// atomic add is the slow one), FP64 global accumulators beyond
template <bool TAIL>
__device__ __forceinline__ void mf_add(const Lds& s, const GradArgs& g, int j, double v)
{
    if (!TAIL || j < g.K) __hip_atomic_fetch_add(s.hgd + j, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else gl_add(&g.tail[j], v);
}

// plane f (0 <= f < kMfPlanes) of the coefficients and rows
template <typename VT>
__device__ __forceinline__ const VT* mf_a(const GradArgs& g, int f)
{
    return (const VT*)(f == 0 ? g.A : g.A2[f - 1]);
}
__device__ __forceinline__ const int32_t* mf_r(const GradArgs& g, int f)
{
    return f == 0 ? g.dst : g.dst2[f - 1];
}

// simplex / capped / box threshold of blocks on S lanes (S = 1: one lane per
// block) from the t of the lane's rows
template <int S, bool HASW, int PJ, int P>
__device__ __forceinline__ double mf_tau(const double (&t)[P], const float (&u)[PJ != 0 ? P : 1],
                                        const float (&w)[HASW ? P : 1], double gamma, double inv_g)
{
    if constexpr (PJ == 2) return cut_threshold<S, HASW, P>(t, u, w, gamma, inv_g);
    else if constexpr (PJ == 0) return seg_threshold<S, HASW, P>(t, w, gamma, inv_g);
    else return 0.0;
}

// one LANE group: loads, t, threshold, then row sums (or the restoration)
template <int S, int P, int PJ, typename VT, bool HASW, bool TAIL>
__device__ __forceinline__ void mf_lane_group(const GradArgs& g, const Item& it, const Lds& s, double gamma,
                                              Obj& ob, double& corr, double& dacc)
{
    constexpr bool BOX = PJ != 0;
    const SegGeo q = seg_geo<S>(it);
    const double inv_g = 1.0 / gamma;
    const int nf = g.nf;
    typename Val<VT>::reg cv[P];
    float u[BOX ? P : 1];
    float w[HASW ? P : 1];
    VT a[kMfPlanes][P];
    int r[kMfPlanes][P];
    const VT* __restrict__ C = (const VT*)g.C + q.ib;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const uint32_t off = seg_off<S>(q, k);
        cv[k] = Val<VT>::cvt(ldo(C, off));
        if (BOX) u[k] = ldo(g.U + q.ib, off);
        if (HASW) w[k] = ldo(g.IV + q.ib, off);
#pragma unroll
        for (int f = 0; f < kMfPlanes; ++f) {
            if (f < nf) {
                a[f][k] = ldo(mf_a<VT>(g, f) + q.ib, off);
                r[f][k] = ldo(mf_r(g, f) + q.ib, off);
            } else {
                a[f][k] = VT(0);
                r[f][k] = 0;
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    double t[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double tk = (double)cv[k];
#pragma unroll
        for (int f = 0; f < kMfPlanes; ++f)
            if (f < nf) tk += (double)Val<VT>::cvt(a[f][k]) * get_lam<false, TAIL>(s, g, r[f][k]);
        t[k] = seg_valid<S>(q, k) ? -tk : -INFINITY;
    }
    const double tau = mf_tau<S, HASW, PJ, P>(t, u, w, gamma, inv_g);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double wk = HASW ? (double)w[HASW ? k : 0] * inv_g : inv_g;
        const double x = xval<BOX>(t[k], wk, tau, BOX ? u[BOX ? k : 0] : 0.0f);
        if (x != 0.0) {
            const double q2 = HASW ? x * x / (double)w[HASW ? k : 0] : x * x;
            const double cx = (double)cv[k] * x;
            if (!g.restore) {
                ob.ot += t[k] * x;
                ob.oq += q2;
                ob.oc += cx;
#pragma unroll
                for (int f = 0; f < kMfPlanes; ++f) {
                    const double af = (double)Val<VT>::cvt(a[f][k]);
                    if (f == g.dense_f) dacc += af * x;
                    else if (f < nf && af != 0.0) mf_add<TAIL>(s, g, r[f][k], af * x);
                }
            } else {
                double se = 1.0;
#pragma unroll
                for (int f = 0; f < kMfPlanes; ++f)
                    if (f < nf && (double)Val<VT>::cvt(a[f][k]) != 0.0) se = fmin(se, g.srow[r[f][k]]);
                corr += (se - 1.0) * cx + 0.5 * gamma * (se * se - 1.0) * q2;
            }
        }
    }
    if (g.X && !g.restore) {
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (seg_valid<S>(q, k)) {
                const double wk = HASW ? (double)w[HASW ? k : 0] * inv_g : inv_g;
                g.X[g.perm[q.ib + seg_off<S>(q, k)]] = xval<BOX>(t[k], wk, tau, BOX ? u[BOX ? k : 0] : 0.0f);
            }
    }
}

// t of one edge from memory (WG blocks)
template <typename VT, bool HASW, bool TAIL>
__device__ __forceinline__ double mf_edge_t(const GradArgs& g, const Lds& s, int64_t idx, double& w,
                                            double inv_g)
{
    double tk = (double)Val<VT>::ld((const VT*)g.C, idx);
    for (int f = 0; f < g.nf; ++f)
        tk += (double)Val<VT>::ld(mf_a<VT>(g, f), idx) * get_lam<false, TAIL>(s, g, mf_r(g, f)[idx]);
    w = HASW ? (double)g.IV[idx] * inv_g : inv_g;
    return -tk;
}

// one block on a whole workgroup, t recomputed on every pass (the block
// stays in L2 between passes)
template <int PJ, typename VT, bool HASW, bool TAIL>
__device__ __forceinline__ void mf_wg_block(const GradArgs& g, const Item& it, const Lds& s, double gamma,
                                            Obj& ob, double& corr, double& dacc)
{
    constexpr bool BOX = PJ != 0;
    const int d = uni(it.d);
    const int64_t base = uni64(it.base);
    const double inv_g = 1.0 / gamma;
    double tau = 0.0;
    if constexpr (PJ == 0) {
        // simplex: tau_0 = max(0, max_e (t_e - 1/w_e)) when the unconstrained
        // sum exceeds 1, then the fixed point over S = {t > tau}
        double s0 = 0.0, mx = -INFINITY;
        for (int e = threadIdx.x; e < d; e += kWG) {
            double w;
            const double t = mf_edge_t<VT, HASW, TAIL>(g, s, base + e, w, inv_g);
            const double z = w * t;
            s0 += z > 0.0 ? z : 0.0;
            mx = fmax(mx, t - 1.0 / w);
        }
        wg_sum_max(s0, mx, s.red);
        if (s0 > 1.0) {
            tau = mx > 0.0 ? mx : 0.0;
            double sw = 0.0, swt = 0.0;
            int n = 0;
            for (int e = threadIdx.x; e < d; e += kWG) {
                double w;
                const double t = mf_edge_t<VT, HASW, TAIL>(g, s, base + e, w, inv_g);
                if (t > tau) {
                    sw += w;
                    swt += w * t;
                    ++n;
                }
            }
            wg_sum3(sw, swt, n, s.red);
#pragma unroll 1
            for (int rep = 0; rep < 2 * d + 4; ++rep) {
                const double tn = (swt - 1.0) / sw;
                double sw2 = 0.0, swt2 = 0.0;
                int n2 = 0;
                for (int e = threadIdx.x; e < d; e += kWG) {
                    double w;
                    const double t = mf_edge_t<VT, HASW, TAIL>(g, s, base + e, w, inv_g);
                    if (t > tn) {
                        sw2 += w;
                        swt2 += w * t;
                        ++n2;
                    }
                }
                wg_sum3(sw2, swt2, n2, s.red);
                tau = tn;
                if (n2 >= n || n2 == 0) break;
                sw = sw2;
                swt = swt2;
                n = n2;
            }
        }
    } else if constexpr (PJ == 2) {
        auto et = [&](int64_t idx, double& w) { return mf_edge_t<VT, HASW, TAIL>(g, s, idx, w, inv_g); };
        tau = wg_cut_threshold_fn<HASW>(g, et, base, d, gamma, s.red);
    }
    for (int e = threadIdx.x; e < d; e += kWG) {
        const int64_t idx = base + e;
        double w;
        const double t = mf_edge_t<VT, HASW, TAIL>(g, s, idx, w, inv_g);
        const double x = xval<BOX>(t, w, tau, BOX ? g.U[idx] : 0.0f);
        if (x != 0.0) {
            const double q2 = HASW ? x * x / (double)g.IV[idx] : x * x;
            const double cx = (double)Val<VT>::ld((const VT*)g.C, idx) * x;
            if (!g.restore) {
                ob.ot += t * x;
                ob.oq += q2;
                ob.oc += cx;
                for (int f = 0; f < g.nf; ++f) {
                    const double af = (double)Val<VT>::ld(mf_a<VT>(g, f), idx);
                    if (f == g.dense_f) dacc += af * x;
                    else if (af != 0.0) mf_add<TAIL>(s, g, mf_r(g, f)[idx], af * x);
                }
            } else {
                double se = 1.0;
                for (int f = 0; f < g.nf; ++f)
                    if ((double)Val<VT>::ld(mf_a<VT>(g, f), idx) != 0.0) se = fmin(se, g.srow[mf_r(g, f)[idx]]);
                corr += (se - 1.0) * cx + 0.5 * gamma * (se * se - 1.0) * q2;
            }
        }
        if (g.X && !g.restore) g.X[g.perm[idx]] = x;
    }
    __syncthreads();
}

// lanes per block S = 2^lg (the host picks the S that pads the degree least)
// and a register class of 4 or kMfRmax rows per lane
template <int S, int PJ, typename VT, bool HASW, bool TAIL>
__device__ __forceinline__ void mf_seg(const GradArgs& g, const Item& it, const Lds& s, double gamma, Obj& ob,
                                       double& corr, double& dacc)
{
    if ((it.d + S - 1) / S <= 4) mf_lane_group<S, 4, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
    else mf_lane_group<S, kMfRmax, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
}
template <int PJ, typename VT, bool HASW, bool TAIL>
__device__ __forceinline__ void mf_lane_dispatch(const GradArgs& g, const Item& it, const Lds& s, double gamma,
                                                 Obj& ob, double& corr, double& dacc)
{
    switch (it.lg) {
    case 0:
        if (it.d <= 4) mf_lane_group<1, 4, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
        else mf_lane_group<1, kMfLaneCap, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
        break;
    case 1: mf_seg<2, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc); break;
    case 2: mf_seg<4, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc); break;
    case 3: mf_seg<8, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc); break;
    case 4: mf_seg<16, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc); break;
    case 5: mf_seg<32, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc); break;
    default: mf_seg<64, PJ, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc); break;
    }
}

template <typename VT, bool HASW, bool TAIL>
__global__ __launch_bounds__(kWG) void grad_mf_kernel(GradArgs g)
{
    if (g.done && *g.done) return;
    const int chunk = blockIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    Lds s;
    s.lam_rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)g.lam, (short)0, g.J * 8, 0x00020000);
    s.red = (double*)smem;
    unsigned char* p = smem + 4 * kWaves * sizeof(double);
    const int K = g.K;
    s.lam = (double*)p;
    p += (size_t)K * sizeof(double);
    // the a x sums of the first K rows, FP64
    s.hg = nullptr;
    s.hgd = (double*)p;
    s.hc = s.hq = nullptr;
    const double gamma = g.gamma_ptr ? *g.gamma_ptr : g.gamma_val;
    for (int j = threadIdx.x; j < K; j += kWG) {
        s.lam[j] = g.lam[j];
        s.hgd[j] = 0.0;
    }
    __syncthreads();

    const Chunk ch = g.chunks[chunk];
    Obj ob = {0.0, 0.0, 0.0};
    double corr = 0.0;
    // the dense plane's a x, summed per lane and added once per wave
    double dacc = 0.0;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // (descriptors by scalar loads: reading one never waits for the vector
    // memory operations in flight)
    for (int i = ch.a0 + wave; i < ch.a1; i += kWaves) {
        Item it = wg_item(g, i);
        it.base = uni64(it.base);
        it.d = uni(it.d);
        if (it.proj == 1) mf_lane_dispatch<1, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
        else if (it.proj == 2) mf_lane_dispatch<2, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
        else mf_lane_dispatch<0, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
    }
    for (int i = ch.b0; i < ch.b1; ++i) {
        const Item it = wg_item(g, i);
        if (it.proj == 1) mf_wg_block<1, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
        else if (it.proj == 2) mf_wg_block<2, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
        else mf_wg_block<0, VT, HASW, TAIL>(g, it, s, gamma, ob, corr, dacc);
    }
    if (g.dense_f >= 0 && !g.restore) {
        dacc = wave_sum(dacc);
        if ((threadIdx.x & 63) == 0 && dacc != 0.0) mf_add<TAIL>(s, g, g.dense_row, dacc);
    }
    __syncthreads();

    // flush: row partials (ordinary pass) and the objective or correction parts
    if (!g.restore) {
        float* row = g.part + (int64_t)chunk * K;
        for (int j = threadIdx.x; j < K; j += kWG) row[j] = (float)s.hgd[j];
    }
    ob.ot = wave_sum(ob.ot);
    ob.oq = wave_sum(ob.oq);
    ob.oc = wave_sum(ob.oc);
    corr = wave_sum(corr);
    if ((threadIdx.x & 63) == 0) {
        s.red[threadIdx.x >> 6] = ob.ot;
        s.red[kWaves + (threadIdx.x >> 6)] = ob.oq;
        s.red[2 * kWaves + (threadIdx.x >> 6)] = ob.oc;
        s.red[3 * kWaves + (threadIdx.x >> 6)] = corr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0, e = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            a += s.red[i];
            b += s.red[kWaves + i];
            c += s.red[2 * kWaves + i];
            e += s.red[3 * kWaves + i];
        }
        if (g.restore) {
            g.corr_part[chunk] = e;
        } else {
            g.obj_part[3 * chunk] = a;
            g.obj_part[3 * chunk + 1] = b;
            g.obj_part[3 * chunk + 2] = c;
        }
    }
}

template <typename VT, bool HASW, bool TAIL>
static hipError_t launch_grad_mf_t(const GradArgs& a, hipStream_t s)
{
    // lam and an FP64 a x sum per LDS row
    const size_t lds = 4 * kWaves * sizeof(double) + (size_t)a.K * 16;
    hipLaunchKernelGGL((grad_mf_kernel<VT, HASW, TAIL>), dim3(a.nchunks), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

template <typename VT>
hipError_t launch_grad_mf_vt(const GradArgs& a, bool has_w, hipStream_t s)
{
    const bool tail = a.K < a.J;
    if (has_w) return tail ? launch_grad_mf_t<VT, true, true>(a, s) : launch_grad_mf_t<VT, true, false>(a, s);
    return tail ? launch_grad_mf_t<VT, false, true>(a, s) : launch_grad_mf_t<VT, false, false>(a, s);
}

template <typename VT>
hipError_t set_grad_mf_attributes_vt(size_t lds)
{
    hipError_t e = hipSuccess, r;
#define DL_A(W, T)                                                                               \
    r = hipFuncSetAttribute((const void*)grad_mf_kernel<VT, W, T>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            (int)lds);                                                           \
    if (r != hipSuccess) e = r;
    DL_A(false, false) DL_A(false, true) DL_A(true, false) DL_A(true, true)
#undef DL_A
    return e;
}

#define DL_INSTANTIATE_GRAD_MF(VT)                                                           \
    template hipError_t launch_grad_mf_vt<VT>(const GradArgs&, bool, hipStream_t);           \
    template hipError_t set_grad_mf_attributes_vt<VT>(size_t);

}  // namespace dl
