// Device code of the fused dual-gradient kernel (included once per storage
// type by grad_f64.hip, grad_f32.hip and grad_bf16.hip).
//
// One pass over the edge stream per dual-gradient evaluation (Section 3.1,
// Danskin): gather lam for each edge's destination, t_e = -(c_e + a_e
// lam_j(e)) in FP64, project each source block onto its simple set (Eq.(4),(5)
// simplex or box), and accumulate a_e x_e into the per-destination sums of
// A x.  Nothing per-edge is written back.  The work is sparse and
// bandwidth-bound, so it runs on the vector ALUs; no MFMA.
//
// Simplex threshold.  With w_e = 1/(gamma v_e^2) the block solution is
// x_e = max(0, w_e (t_e - tau)), tau = 0 when sum_e max(0, w_e t_e) <= 1, else
// the root of sum_e max(0, w_e (t_e - tau)) = 1.  Since x_e <= 1 forces
// tau >= t_e - 1/w_e, the search starts at tau_0 = max(0, max_e (t_e - 1/w_e)),
// whose set S_0 = {t > tau_0} holds every active edge.  Then the fixed point
// tau <- (sum_S w t - 1) / sum_S w with S = {t > tau} (Michelot 1986) rises
// monotonically and stops when S no longer shrinks; the result is exact (KKT
// hold for the final set), not limited by a bisection tolerance.  Because
// tau_1 > tau_0 (the top edge alone already gives w (t - tau_0) = 1) every
// set along the way is a threshold set {t > tau}, so no membership mask is
// kept.  With uniform weights the first pass also finds the second-largest
// t; when it is at most tau_0 only the largest t is active, tau_0 is already
// the threshold and the fixed-point passes are skipped.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "kernels.hpp"
#include "lanes.hpp"

namespace dl {

// ---------------------------------------------------------------------------
// stored value types
// ---------------------------------------------------------------------------
template <typename VT>
struct Val;
template <>
struct Val<double> {
    using reg = double;
    static __device__ __forceinline__ double ld(const double* p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ double cvt(double v) { return v; }
};
template <>
struct Val<float> {
    using reg = float;
    static __device__ __forceinline__ float ld(const float* p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ float cvt(float v) { return v; }
};
template <>
struct Val<uint16_t> {   // bfloat16 bits: widen by a 16-bit shift (exact)
    using reg = float;
    static __device__ __forceinline__ float ld(const uint16_t* p, int64_t i)
    {
        return __uint_as_float(((uint32_t)p[i]) << 16);
    }
    static __device__ __forceinline__ float cvt(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }
};

// an opaque copy: keeps the compiler from carrying an FP64 widening of a
// stored value from one pass to the next (it would double its registers)
__device__ __forceinline__ float opq(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ double opq(double v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// load at a 32-bit unsigned byte offset from a wave-uniform base: lets the
// compiler use the scalar-base + 32-bit vector-offset form of global loads
template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t elem)
{
    return *(const T*)((const char*)base + elem * (uint32_t)sizeof(T));
}

// wave-uniform copies (scalar registers) of values the compiler cannot prove uniform
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

struct Lds {
    __amdgpu_buffer_rsrc_t lam_rsrc;   // global lam (rows beyond K)
    double* red;   // [4 * kWaves] workgroup reduction scratch
    double* lam;   // [K] (normal passes)
    float* hg;     // [K] sum a x
    float* hc;     // [K] sum c x   (check passes)
    float* hq;     // [K] sum v^2 x^2 (check passes)
    double* hgd;   // [K] sum a x in FP64 (ordinary passes without rows beyond K,
                   // outside deterministic mode)
};

// three sums and a count over the whole workgroup (all threads call it)
__device__ __forceinline__ void wg_sum3(double& a, double& b, int& n, double* red)
{
    a = wave_sum(a);
    b = wave_sum(b);
    n = wave_sum_i(n);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = a;
        red[kWaves + w] = b;
        red[2 * kWaves + w] = (double)n;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    double nn = 0.0;
    for (int i = 0; i < kWaves; ++i) {
        a += red[i];
        b += red[kWaves + i];
        nn += red[2 * kWaves + i];
    }
    n = (int)nn;
}
__device__ __forceinline__ void wg_sum_max(double& s, double& m, double* red)
{
    s = wave_sum(s);
    m = wave_max(m);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = s;
        red[kWaves + w] = m;
    }
    __syncthreads();
    s = 0.0;
    m = -INFINITY;
    for (int i = 0; i < kWaves; ++i) {
        s += red[i];
        m = fmax(m, red[kWaves + i]);
    }
}

// a sum and the two largest values over the whole workgroup
__device__ __forceinline__ void wg_sum_top2(double& s, double& m1, double& m2, double* red)
{
    s = wave_sum(s);
    wave_top2(m1, m2);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = s;
        red[kWaves + w] = m1;
        red[2 * kWaves + w] = m2;
    }
    __syncthreads();
    s = 0.0;
    m1 = -INFINITY;
    m2 = -INFINITY;
    for (int i = 0; i < kWaves; ++i) {
        s += red[i];
        top2_merge(m1, m2, red[kWaves + i], red[2 * kWaves + i]);
    }
}

// ---------------------------------------------------------------------------
// per-edge helpers
// ---------------------------------------------------------------------------
// lam of row j: from LDS for rows below K; rows beyond K come from a raw
// buffer load whose offset is pushed out of range (returns 0, no memory
// access) for LDS rows, so no per-edge branch or flat load is needed.  Check
// passes of problems with rows beyond K keep the LDS for the three sums and
// read lam from global memory.
template <bool CHECK, bool TAIL>
__device__ __forceinline__ double get_lam(const Lds& s, const GradArgs& g, int j)
{
    if (CHECK && TAIL) return ldo(g.lam, (uint32_t)j);
    if (!TAIL) return s.lam[j];
    const double l = s.lam[j < g.K ? j : g.K - 1];
    const uint32_t off = j >= g.K ? (uint32_t)j * 8u : 0xFFFFFFFFu;
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(s.lam_rsrc, off, 0, 0);
    const double gv = __longlong_as_double((long long)(((unsigned long long)v.y << 32) | v.x));
    return j < g.K ? l : gv;
}

__device__ __forceinline__ void lds_add(float* p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gl_add(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One term of a per-destination sum (plane 0: a x, 1: c x, 2: v^2 x^2).
// Ordinarily an f32 atomic add into LDS or an FP64 atomic add into the global
// accumulators, whose result depends on the order the waves add in.  In
// deterministic mode the term is rounded to a 64-bit fixed-point integer
// (scale qs[plane], chosen at create so that no row's sum can overflow) and
// added with an integer atomic: integer addition is associative, so every
// run gives the same bits.
// The mode is a compile-time property of the kernel variant: the
// projection-level templates carry a code PJ whose low two bits are the
// block's dl_proj and whose bit 2 selects deterministic sums.
constexpr int pj_proj(int pj) { return pj & 3; }
constexpr bool pj_det(int pj) { return (pj & 4) != 0; }
__device__ __forceinline__ unsigned long long fixq(const GradArgs& g, double v, int plane)
{
    return (unsigned long long)__double2ll_rn(v * g.qs[plane]);
}
template <bool DET>
__device__ __forceinline__ void lds_term(const GradArgs& g, float* base, int j, double v, int plane)
{
    if (DET)
        __hip_atomic_fetch_add((unsigned long long*)base + j, fixq(g, v, plane), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        lds_add(base + j, (float)v);
}
template <bool DET>
__device__ __forceinline__ void gl_term(const GradArgs& g, double* p, double v, int plane)
{
    if (DET)
        __hip_atomic_fetch_add((unsigned long long*)p, fixq(g, v, plane), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    else
        gl_add(p, v);
}

// per-destination sums: rows below K in LDS (f32, or 64-bit integers in
// deterministic mode), the rest in global accumulators (a separate, rarely
// taken path so the main loop stays lean).  Check passes keep the c x and
// v^2 x^2 sums of the first Kc rows in LDS and add the others to the global
// accumulators.
template <bool CHECK, bool TAIL, bool DET>
__device__ __forceinline__ void accum_lds(const Lds& s, const GradArgs& g, int j, double ax, double cx, double q)
{
    // ordinary passes of problems whose rows all fit in LDS at 16 bytes add
    // a x in FP64 (the LDS's f32 atomic add runs at a fraction of the rate
    // of its FP64 and integer ones: box blocks, whose active edges are most
    // of their edges, ran 1.5x slower with it)
    if constexpr (!CHECK && !DET && !TAIL) __hip_atomic_fetch_add(s.hgd + j, ax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else lds_term<DET>(g, s.hg, j, ax, 0);
    if (CHECK) {
        if (j < g.Kc) {
            lds_term<DET>(g, s.hc, j, cx, 1);
            lds_term<DET>(g, s.hq, j, q, 2);
        } else {
            gl_term<DET>(g, &g.tail[g.J + j], cx, 1);
            gl_term<DET>(g, &g.tail[2 * (int64_t)g.J + j], q, 2);
        }
    }
}
template <bool CHECK, bool DET>
__device__ __forceinline__ void accum_tail(const GradArgs& g, int j, double ax, double cx, double q)
{
    gl_term<DET>(g, &g.tail[j], ax, 0);
    if (CHECK) {
        gl_term<DET>(g, &g.tail[g.J + j], cx, 1);
        gl_term<DET>(g, &g.tail[2 * (int64_t)g.J + j], q, 2);
    }
}
template <bool CHECK, bool TAIL, bool DET>
__device__ __forceinline__ void accum(const Lds& s, const GradArgs& g, int j, double ax, double cx,
                                      double q)
{
    if (!TAIL || j < g.K) accum_lds<CHECK, TAIL, DET>(s, g, j, ax, cx, q);
    else accum_tail<CHECK, DET>(g, j, ax, cx, q);
}

// the projected value of one edge given its block threshold: clamp(w (t -
// tau), 0, u), u = inf on simplex blocks, tau = 0 on box blocks (t - 0 is t,
// so a box edge is exactly clamp(w t, 0, u))
template <bool BOX>
__device__ __forceinline__ double xval(double t, double w, double tau, float u)
{
    const double z = w * (t - tau);
    if (BOX) return z > 0.0 ? (z < (double)u ? z : (double)u) : 0.0;
    return z > 0.0 ? z : 0.0;
}

// ---------------------------------------------------------------------------
// Objective bookkeeping.  With t = -(c + A'lam) the dual objective is
//   g = c'x + gamma/2 |D_v x|^2 + lam'(A x - b) = -t'x + gamma/2 |D_v x|^2 - lam'b,
// so ordinary passes accumulate ot = sum t x and oq = sum v^2 x^2 only (c is
// not kept past pass 1); check passes also accumulate oc = sum c x for the
// primal value of the gap.
// ---------------------------------------------------------------------------
struct Obj {
    double ot, oq, oc;
};

// ---------------------------------------------------------------------------
// LANE items (block-to-wavefront binning).  A group holds nb blocks of one
// degree d.  Each block owns S = 2^lg consecutive lanes of a wave (S = 1: one
// lane per block, up to 64 blocks; S = 64: one block per wave) and each lane
// keeps up to P of its block's edges in registers.  Edge e = k S + s of block
// b (lane b S + s) is stored at base + k nb S + b S + s for the R - 1 full
// rows; the last row (rem = d - (R - 1) S edges per block) is stored
// compacted at base + (R - 1) nb S + b rem + s.  A group is exactly nb d
// positions, every row of loads is one contiguous run, and S = 1 is the
// plain lane-interleaved layout (edge k of block b at base + k nb + b).
//
// A group is handled in three steps: the loads of its stored values, the t
// phase (gather lam, t in FP64) and the projection phase (threshold, x,
// objective, per-destination sums).  With S > 1 the threshold sums are
// reduced over the block's S lanes with butterfly shuffles (every lane of
// the segment gets the same bits).  Runs of groups of one class are
// software-pipelined: the loads of the next group are issued before the
// projection phase of the current one, so a wave keeps memory busy while it
// computes.
// ---------------------------------------------------------------------------
struct SegGeo {
    int64_t ib;   // stream offset of the group
    int d, nb;    // degree, blocks in the group
    int R, rem;   // rows per lane, edges of the last row per block
};
template <int S>
__device__ __forceinline__ SegGeo seg_geo(const Item& it)
{
    SegGeo q;
    q.ib = uni64(it.base);
    q.d = uni(it.d);
    q.nb = uni(it.nb);
    if (S == 1) {
        q.R = q.d;
        q.rem = 1;
    } else {
        q.R = (q.d + S - 1) / S;
        q.rem = q.d - (q.R - 1) * S;
    }
    return q;
}
template <int S>
__device__ __forceinline__ int seg_b()
{
    return (int)(threadIdx.x & 63) / S;
}
template <int S>
__device__ __forceinline__ int seg_s()
{
    return (int)(threadIdx.x & 63) & (S - 1);
}

// offset from the group base of this lane's row k; rows beyond the block
// re-read its last edge and idle lanes read the last block's, so every load
// is unconditional and in bounds (32-bit offsets from a wave-uniform base)
template <int S>
__device__ __forceinline__ uint32_t seg_off(const SegGeo& q, int k)
{
    const int b = seg_b<S>();
    const int bc = b < q.nb ? b : q.nb - 1;
    const int kk = k < q.R ? k : q.R - 1;
    if (S == 1) return (uint32_t)(kk * q.nb + bc);
    const int s = seg_s<S>();
    const int W = q.nb * S;
    const int last = (q.R - 1) * W + bc * q.rem + (s < q.rem ? s : q.rem - 1);
    return (uint32_t)(kk < q.R - 1 ? kk * W + bc * S + s : last);
}
// whether row k of this lane is an edge of its block
template <int S>
__device__ __forceinline__ bool seg_valid(const SegGeo& q, int k)
{
    const int b = seg_b<S>();
    if (S == 1) return b < q.nb && k < q.d;
    const int s = seg_s<S>();
    return b < q.nb && (k < q.R - 1 || (k == q.R - 1 && s < q.rem));
}

// reductions over the S lanes of a segment
template <int S>
__device__ __forceinline__ double seg_sum(double v)
{
    return grp_sum<S>(v);
}
template <int S>
__device__ __forceinline__ double seg_max(double v)
{
    return grp_max<S>(v);
}
template <int S>
__device__ __forceinline__ void seg_top2(double& m1, double& m2)
{
    grp_top2<S>(m1, m2);
}
template <int S>
__device__ __forceinline__ int seg_sum_i(int v)
{
    return grp_sum_i<S>(v);
}

// stored values of rows k < P, as loaded
template <typename VT, bool BOX, bool HASW, int P>
struct LaneRaw {
    VT a[P], c[P];
    int j[P];
    float u[BOX ? P : 1];
    float w[HASW ? P : 1];
};

// values the projection phase works on
template <typename VT, bool CHECK, bool BOX, bool HASW, int P>
struct LaneVals {
    using R = typename Val<VT>::reg;
    double t[P];
    R a[P];
    R c[CHECK ? P : 1];
    int j[P];
    float u[BOX ? P : 1];
    float w[HASW ? P : 1];
};

// loads of rows [K0, K1)
template <int K0, int K1, int S, typename VT, bool BOX, bool HASW, int P>
__device__ __forceinline__ void lane_load(const GradArgs& g, const SegGeo& q, LaneRaw<VT, BOX, HASW, P>& r)
{
    const VT* __restrict__ A = (const VT*)g.A + q.ib;
    const VT* __restrict__ C = (const VT*)g.C + q.ib;
    const int32_t* __restrict__ Dst = g.dst + q.ib;
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        const uint32_t off = seg_off<S>(q, k);
        r.a[k] = ldo(A, off);
        r.c[k] = ldo(C, off);
        r.j[k] = ldo(Dst, off);
        if (BOX) r.u[k] = ldo(g.U + q.ib, off);
        if (HASW) r.w[k] = ldo(g.IV + q.ib, off);
    }
}

// t of row k from its stored values and lam: t_e = -(c_e + a_e lam_j(e)) in
// FP64; rows that are no edge of the lane's block get t = -inf (never active)
template <int S, typename VT, bool CHECK, bool BOX, bool HASW, int P>
__device__ __forceinline__ void lane_t_row(const SegGeo& q, const LaneRaw<VT, BOX, HASW, P>& r, const int k,
                                           const double lam, LaneVals<VT, CHECK, BOX, HASW, P>& v)
{
    using R = typename Val<VT>::reg;
    v.a[k] = Val<VT>::cvt(r.a[k]);
    const R c = Val<VT>::cvt(r.c[k]);
    v.j[k] = r.j[k];
    if (BOX) v.u[k] = r.u[k];
    if (HASW) v.w[k] = r.w[k];
    const double tk = -((double)c + (double)v.a[k] * lam);
    v.t[k] = seg_valid<S>(q, k) ? tk : -INFINITY;
    if (CHECK) v.c[k] = c;
}

// t phase of rows [K0, K1), lam gathered here
template <int K0, int K1, int S, typename VT, bool CHECK, bool TAIL, bool BOX, bool HASW, int P>
__device__ __forceinline__ void lane_t(const GradArgs& g, const Lds& s, const SegGeo& q,
                                       const LaneRaw<VT, BOX, HASW, P>& r,
                                       LaneVals<VT, CHECK, BOX, HASW, P>& v)
{
#pragma unroll
    for (int k = K0; k < K1; ++k) lane_t_row<S>(q, r, k, get_lam<CHECK, TAIL>(s, g, r.j[k]), v);
}

// lam gathers of rows [0, P) (global or buffer loads on passes that read lam
// from memory) and the t phase that consumes them, for the pipelined runs
template <typename VT, bool CHECK, bool TAIL, bool BOX, bool HASW, int P>
__device__ __forceinline__ void lane_gather(const GradArgs& g, const Lds& s, const LaneRaw<VT, BOX, HASW, P>& r,
                                            double (&lam)[P])
{
#pragma unroll
    for (int k = 0; k < P; ++k) lam[k] = get_lam<CHECK, TAIL>(s, g, r.j[k]);
}
template <int S, typename VT, bool CHECK, bool BOX, bool HASW, int P>
__device__ __forceinline__ void lane_t_gathered(const SegGeo& q, const LaneRaw<VT, BOX, HASW, P>& r,
                                                const double (&lam)[P], LaneVals<VT, CHECK, BOX, HASW, P>& v)
{
#pragma unroll
    for (int k = 0; k < P; ++k) lane_t_row<S>(q, r, k, lam[k], v);
}

// simplex threshold of blocks spread over S > 1 lanes: every lane holds
// partial sums over its rows, reduced over the segment.  Segments iterate in
// lock step (the loop runs while any segment of the wave is still moving,
// finished ones hold their tau) so every shuffle sees the whole wave.
template <int S, bool HASW, int P>
__device__ __forceinline__ double seg_threshold(const double (&t)[P], const float (&wv)[HASW ? P : 1],
                                                const double gamma, const double inv_g)
{
    double tau = 0.0;
    if (!HASW) {
        double sp = 0.0, mt = -INFINITY, m2 = -INFINITY;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            sp += t[k] > 0.0 ? t[k] : 0.0;
            m2 = fmax(m2, fmin(mt, t[k]));
            mt = fmax(mt, t[k]);
        }
        sp = seg_sum<S>(sp);
        seg_top2<S>(mt, m2);
        bool live = sp > gamma;
        if (!__builtin_amdgcn_ballot_w64(live)) return 0.0;
        double tv = live ? (mt - gamma > 0.0 ? mt - gamma : 0.0) : 0.0;
        // segments with one t above tau_0 are done (see the one-lane case)
        if (!__builtin_amdgcn_ballot_w64(live && m2 > tv)) return tv;
        double st = 0.0;
        int n = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const bool in = t[k] > tv;
            st += in ? t[k] : 0.0;
            n += in ? 1 : 0;
        }
        st = seg_sum<S>(st);
        n = seg_sum_i<S>(n);
        const bool moved = live;
#pragma unroll 1
        for (int rep = 0; rep < 2 * P * S + 4; ++rep) {
            if (!__builtin_amdgcn_ballot_w64(live)) break;
            const double tn = live ? (st - gamma) / (double)n : tv;
            double st2 = 0.0;
            int n2 = 0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const bool in = t[k] > tn;
                st2 += in ? t[k] : 0.0;
                n2 += in ? 1 : 0;
            }
            st2 = seg_sum<S>(st2);
            n2 = seg_sum_i<S>(n2);
            if (live) {
                tv = tn;
                if (n2 >= n || n2 == 0) {
                    live = false;
                } else {
                    st = st2;
                    n = n2;
                }
            }
        }
        tau = moved ? tv : 0.0;
    } else {
        double s0 = 0.0, mx = -INFINITY;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double w = (double)wv[HASW ? k : 0] * inv_g;
            const double iw = gamma / (double)wv[HASW ? k : 0];
            const double z = w * t[k];
            s0 += z > 0.0 ? z : 0.0;
            const double lo = t[k] - iw;
            mx = lo > mx ? lo : mx;
        }
        s0 = seg_sum<S>(s0);
        mx = seg_max<S>(mx);
        bool live = s0 > 1.0;
        if (!__builtin_amdgcn_ballot_w64(live)) return 0.0;
        double tv = live ? (mx > 0.0 ? mx : 0.0) : 0.0;
        double sw = 0.0, swt = 0.0;
        int n = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double w = (double)wv[HASW ? k : 0] * inv_g;
            const bool in = t[k] > tv;
            sw += in ? w : 0.0;
            swt += in ? w * t[k] : 0.0;
            n += in ? 1 : 0;
        }
        sw = seg_sum<S>(sw);
        swt = seg_sum<S>(swt);
        n = seg_sum_i<S>(n);
        const bool moved = live;
#pragma unroll 1
        for (int rep = 0; rep < 2 * P * S + 4; ++rep) {
            if (!__builtin_amdgcn_ballot_w64(live)) break;
            const double tn = live ? (swt - 1.0) / sw : tv;
            double sw2 = 0.0, swt2 = 0.0;
            int n2 = 0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double w = (double)opq(wv[HASW ? k : 0]) * inv_g;
                const bool in = t[k] > tn;
                sw2 += in ? w : 0.0;
                swt2 += in ? w * t[k] : 0.0;
                n2 += in ? 1 : 0;
            }
            sw2 = seg_sum<S>(sw2);
            swt2 = seg_sum<S>(swt2);
            n2 = seg_sum_i<S>(n2);
            if (live) {
                tv = tn;
                if (n2 >= n || n2 == 0) {
                    live = false;
                } else {
                    sw = sw2;
                    swt = swt2;
                    n = n2;
                }
            }
        }
        tau = moved ? tv : 0.0;
    }
    return tau;
}

// ---------------------------------------------------------------------------
// Capped simplex {0 <= x <= u, sum x <= 1} (the reading of the box-cut set):
// x_e = clamp(w_e (t_e - tau), 0, u_e) with tau = 0 when phi(0) =
// sum_e clamp(w_e t_e, 0, u_e) <= 1, else the root tau > 0 of phi(tau) = 1.
// The root is found by variable fixing on a bracket [lo, hi] that holds it
// (Kiwiel 2008, on the continuous quadratic knapsack): edges with t <= lo sit
// at 0, edges with t > lo and t - u/w >= hi at their bound u, the others are
// free.  The free edges' relaxed root tau_F = (sum_F w t + sum_U u - 1) /
// sum_F w makes the free values sum to what the fixed ones leave; clipping
// those that leave [0, u] adds dn (from below 0) and removes up (above u), so
// phi(tau_F) - 1 = dn - up and the root lies above tau_F when dn >= up (lo
// moves to tau_F: the edges pushed below 0 are fixed there) and below it
// otherwise (hi moves: the edges above u are fixed at u).  Each step fixes at
// least one edge; when no free edge leaves [0, u], tau_F is the root and the
// result satisfies the KKT conditions exactly.  (The oracle uses a different
// exact method, a breakpoint search.)
// ---------------------------------------------------------------------------
// rows that are no edge carry t = -inf: never free, never at a bound
template <bool HASW>
__device__ __forceinline__ bool cut_free(double t, float u, float wv, double gamma, double lo, double hi)
{
    const double iw = HASW ? gamma / (double)wv : gamma;   // 1/w
    return t > lo && t - (double)u * iw < hi;
}
template <bool HASW>
__device__ __forceinline__ bool cut_upper(double t, float u, float wv, double gamma, double lo, double hi)
{
    const double iw = HASW ? gamma / (double)wv : gamma;
    return t > lo && !(t - (double)u * iw < hi);
}

// blocks on S lanes (S = 1: one lane per block); the segments of a wave
// iterate in lock step, finished ones holding their tau
template <int S, bool HASW, int P>
__device__ __forceinline__ double cut_threshold(const double (&t)[P], const float (&u)[P],
                                               const float (&wv)[HASW ? P : 1], const double gamma,
                                               const double inv_g)
{
    double s0 = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double w = HASW ? (double)wv[HASW ? k : 0] * inv_g : inv_g;
        const double z = w * t[k];
        s0 += z > 0.0 ? (z < (double)u[k] ? z : (double)u[k]) : 0.0;
    }
    s0 = seg_sum<S>(s0);
    bool live = s0 > 1.0;
    if (!__builtin_amdgcn_ballot_w64(live)) return 0.0;
    double lo = 0.0, hi = INFINITY, tau = 0.0;
#pragma unroll 1
    for (int rep = 0; rep < P * S + 4; ++rep) {
        if (!__builtin_amdgcn_ballot_w64(live)) break;
        double sw = 0.0, swt = 0.0, su = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const float wk = wv[HASW ? k : 0];
            const double w = HASW ? (double)wk * inv_g : inv_g;
            const bool fr = cut_free<HASW>(t[k], u[k], wk, gamma, lo, hi);
            const bool up = cut_upper<HASW>(t[k], u[k], wk, gamma, lo, hi);
            sw += fr ? w : 0.0;
            swt += fr ? w * t[k] : 0.0;
            su += up ? (double)u[k] : 0.0;
        }
        sw = seg_sum<S>(sw);
        swt = seg_sum<S>(swt);
        su = seg_sum<S>(su);
        const double tf = sw > 0.0 ? (swt + su - 1.0) / sw : lo;
        double dn = 0.0, dup = 0.0;
        int nv = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const float wk = wv[HASW ? k : 0];
            const double w = HASW ? (double)wk * inv_g : inv_g;
            const bool fr = cut_free<HASW>(t[k], u[k], wk, gamma, lo, hi);
            const double z = w * (t[k] - tf);
            const bool below = fr && z < 0.0, above = fr && z > (double)u[k];
            dn += below ? -z : 0.0;
            dup += above ? z - (double)u[k] : 0.0;
            nv += (below || above) ? 1 : 0;
        }
        dn = seg_sum<S>(dn);
        dup = seg_sum<S>(dup);
        nv = seg_sum_i<S>(nv);
        if (live) {
            tau = tf;
            if (nv == 0 || !(sw > 0.0)) live = false;
            else if (dn >= dup) lo = fmax(lo, tf);
            else hi = fmin(hi, tf);
        }
    }
    return tau;
}

// projection phase: simplex threshold, then x, the objective and the
// per-destination sums
template <int S, typename VT, bool CHECK, bool HASW, bool TAIL, int PJ, int P>
__device__ __forceinline__ void lane_project(const GradArgs& g, const Lds& s, const SegGeo& q,
                                             double gamma, Obj& ob, const LaneVals<VT, CHECK, pj_proj(PJ) != 0, HASW, P>& v)
{
    constexpr bool BOX = pj_proj(PJ) != 0;   // per-edge bounds (box and capped blocks)
    constexpr bool DET = pj_det(PJ);
    const double inv_g = 1.0 / gamma;
    const double* t = v.t;
    double tau = 0.0;
    if constexpr (pj_proj(PJ) == 2) {
        tau = cut_threshold<S, HASW, P>(v.t, v.u, v.w, gamma, inv_g);
    } else if (S > 1) {
        if (!BOX) tau = seg_threshold<S, HASW, P>(v.t, v.w, gamma, inv_g);
    } else if (!BOX && !HASW) {
        // uniform weight w = 1/gamma: sum max(0, w t) > 1  <=>  sum max(0, t) > gamma,
        // tau_0 = max(0, max t - gamma), tau <- (sum_S t - gamma) / |S|
        // m2: second largest t.  With m2 <= tau_0 only the largest t is above
        // tau_0, so tau_0 = max t - gamma is the threshold (the iteration would
        // return it unchanged); otherwise iterate.
        double sp = 0.0, mt = -INFINITY, m2 = -INFINITY;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            sp += t[k] > 0.0 ? t[k] : 0.0;
            m2 = fmax(m2, fmin(mt, t[k]));
            mt = fmax(mt, t[k]);
        }
        if (sp > gamma) tau = mt - gamma > 0.0 ? mt - gamma : 0.0;
        if (sp > gamma && m2 > tau) {
            double st = 0.0;
            int n = 0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const bool in = t[k] > tau;
                st += in ? t[k] : 0.0;
                n += in ? 1 : 0;
            }
#pragma unroll 1
            for (int rep = 0; rep < 2 * P + 4; ++rep) {
                const double tn = (st - gamma) / (double)n;
                double st2 = 0.0;
                int n2 = 0;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const bool in = t[k] > tn;
                    st2 += in ? t[k] : 0.0;
                    n2 += in ? 1 : 0;
                }
                tau = tn;
                if (n2 >= n || n2 == 0) break;
                st = st2;
                n = n2;
            }
        }
    } else if (!BOX) {
        double s0 = 0.0, mx = -INFINITY;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double w = (double)v.w[HASW ? k : 0] * inv_g;
            const double iw = gamma / (double)v.w[HASW ? k : 0];
            const double z = w * t[k];
            s0 += z > 0.0 ? z : 0.0;
            const double lo = t[k] - iw;
            mx = lo > mx ? lo : mx;
        }
        if (s0 > 1.0) {
            tau = mx > 0.0 ? mx : 0.0;
            double sw = 0.0, swt = 0.0;
            int n = 0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double w = (double)v.w[HASW ? k : 0] * inv_g;
                const bool in = t[k] > tau;
                sw += in ? w : 0.0;
                swt += in ? w * t[k] : 0.0;
                n += in ? 1 : 0;
            }
#pragma unroll 1
            for (int rep = 0; rep < 2 * P + 4; ++rep) {
                const double tn = (swt - 1.0) / sw;
                double sw2 = 0.0, swt2 = 0.0;
                int n2 = 0;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    // recomputed each round (opaque): hoisting P FP64 weights
                    // out of the loop would cost 2P registers
                    const double w = (double)opq(v.w[HASW ? k : 0]) * inv_g;
                    const bool in = t[k] > tn;
                    sw2 += in ? w : 0.0;
                    swt2 += in ? w * t[k] : 0.0;
                    n2 += in ? 1 : 0;
                }
                tau = tn;
                if (n2 >= n || n2 == 0) break;
                sw = sw2;
                swt = swt2;
                n = n2;
            }
        }
    }

    // x, objective, per-destination sums of the LDS-resident rows (rows that
    // are no edge have t = -inf, hence x = 0, and are skipped); then rows
    // beyond K (only when some lane of the wave has one)
    bool tail = false;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
        const double x = xval<BOX>(t[k], w, tau, BOX ? v.u[k] : 0.0f);
        if (x != 0.0) {
            const double q2 = HASW ? x * x / (double)v.w[k] : x * x;
            ob.ot += t[k] * x;
            ob.oq += q2;
            const double cx = CHECK ? (double)v.c[k] * x : 0.0;
            if (CHECK) ob.oc += cx;
            if (!TAIL || v.j[k] < g.K) accum_lds<CHECK, TAIL, DET>(s, g, v.j[k], (double)opq(v.a[k]) * x, cx, q2);
            else tail = true;
        }
    }
    if (TAIL && __builtin_amdgcn_ballot_w64(tail)) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
            const double x = xval<BOX>(t[k], w, tau, BOX ? v.u[k] : 0.0f);
            if (x != 0.0 && v.j[k] >= g.K) {
                const double q2 = HASW ? x * x / (double)v.w[k] : x * x;
                accum_tail<CHECK, DET>(g, v.j[k], (double)opq(v.a[k]) * x, CHECK ? (double)opq(v.c[k]) * x : 0.0,
                                       q2);
            }
        }
    }
    if (g.X) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (seg_valid<S>(q, k)) {
                const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
                g.X[g.perm[q.ib + seg_off<S>(q, k)]] = xval<BOX>(t[k], w, tau, BOX ? v.u[k] : 0.0f);
            }
        }
    }
}

// one group of up to 32 rows with S = 1, not pipelined: the loads go out in
// tiles, each tile's loads all issued before their first use behind a
// scheduling fence (left to itself the scheduler interleaves each row's loads
// with its use, one memory round trip per row)
template <typename VT, bool CHECK, bool HASW, bool TAIL, int PJ, int P>
__device__ __forceinline__ void lane_group(const GradArgs& g, const Item& it, const Lds& s,
                                           double gamma, Obj& ob)
{
    constexpr bool BOX = pj_proj(PJ) != 0;
    static_assert(P <= 32, "lane blocks hold at most 32 edges");
    const SegGeo q = seg_geo<1>(it);
    LaneRaw<VT, BOX, HASW, P> r;
    LaneVals<VT, CHECK, BOX, HASW, P> v;
    // (rows beyond LDS gather lam with a second load per row: smaller tiles)
    constexpr int T0 = TAIL ? 8 : 16;
    constexpr int T = P < T0 ? P : T0;
    lane_load<0, T, 1>(g, q, r);
    __builtin_amdgcn_sched_barrier(0);
    lane_t<0, T, 1, VT, CHECK, TAIL>(g, s, q, r, v);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (P > T) {
        constexpr int T2 = P < 2 * T ? P : 2 * T;
        lane_load<T, T2, 1>(g, q, r);
        __builtin_amdgcn_sched_barrier(0);
        lane_t<T, T2, 1, VT, CHECK, TAIL>(g, s, q, r, v);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (P > T2) {
            constexpr int T3 = P < 3 * T ? P : 3 * T;
            lane_load<T2, T3, 1>(g, q, r);
            __builtin_amdgcn_sched_barrier(0);
            lane_t<T2, T3, 1, VT, CHECK, TAIL>(g, s, q, r, v);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (P > T3) {
                lane_load<T3, P, 1>(g, q, r);
                __builtin_amdgcn_sched_barrier(0);
                lane_t<T3, P, 1, VT, CHECK, TAIL>(g, s, q, r, v);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    lane_project<1, VT, CHECK, HASW, TAIL, PJ, P>(g, s, q, gamma, ob, v);
}

// row class of a group: S = 1 by degree (FP64 storage: at most 8); S > 1 by
// rows per lane, 8 or the variant's largest
template <typename VT, bool HASW, bool TAIL>
__device__ __forceinline__ int lane_class(int d, int lg)
{
    constexpr int RMAX = seg_rmax(sizeof(VT) == 8, HASW, TAIL);
    if (lg == 0) {
        if (sizeof(VT) == 8) return d <= 4 ? 4 : 8;
        return d <= 4 ? 4 : d <= 8 ? 8 : d <= 12 ? 12 : d <= 16 ? 16 : d <= 24 ? 24 : 32;
    }
    const int R = (d + (1 << lg) - 1) >> lg;
    return R <= 8 ? 8 : RMAX;
}

// item r of a batch of 64 descriptors held one per lane
__device__ __forceinline__ Item item_at(const Item& mine, int r)
{
    Item it;
    it.base = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(mine.base >> 32), r) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)mine.base, r));
    it.d = __builtin_amdgcn_readlane(mine.d, r);
    const int pk = __builtin_amdgcn_readlane((int)mine.nb | ((int)mine.lg << 8) | ((int)mine.kind << 16) |
                                                 ((int)mine.proj << 24),
                                             r);
    it.nb = (uint8_t)(pk & 0xFF);
    it.lg = (uint8_t)((pk >> 8) & 0xFF);
    it.kind = (uint8_t)((pk >> 16) & 0xFF);
    it.proj = (uint8_t)((pk >> 24) & 0xFF);
    return it;
}

// a run of groups of one class (S, P, projection) starting at batch entry r:
// the next group's loads are in flight while the current group projects.
// Passes that read lam from LDS issue them before the t phase; passes that
// gather lam from memory issue the gathers first, then the prefetch, so that
// waiting for the gathers (older in the in-order memory counter) never waits
// for the prefetch as well.  Returns the first entry not processed.
template <int S, typename VT, bool CHECK, bool HASW, bool TAIL, int PJ, int P>
__device__ __forceinline__ int lane_run(const GradArgs& g, const Item& mine, int r, const int rn, const Lds& s,
                                        double gamma, Obj& ob)
{
    constexpr bool BOX = pj_proj(PJ) != 0;
    static_assert(P <= 16, "pipelined lane runs hold at most 16 rows per group");
    constexpr int LG = S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : S == 8 ? 3 : S == 16 ? 4 : S == 32 ? 5 : 6;
    static_assert((1 << LG) == S, "S is a power of two up to 64");
    constexpr bool EARLY = !TAIL;   // lam from LDS
    SegGeo q = seg_geo<S>(item_at(mine, r));
    LaneRaw<VT, BOX, HASW, P> cur;
    lane_load<0, P, S>(g, q, cur);
#pragma unroll 1
    for (;;) {
        // the next group of this class, else the current one again (its
        // loads are in bounds and their values are never used)
        bool more = false;
        SegGeo qn = q;
        if (r + 1 < rn) {
            const Item nx = item_at(mine, r + 1);
            if (nx.proj == pj_proj(PJ) && nx.kind == ITEM_LANE && nx.lg == LG &&
                lane_class<VT, HASW, TAIL>(nx.d, LG) == P) {
                more = true;
                qn = seg_geo<S>(nx);
            }
        }
        LaneRaw<VT, BOX, HASW, P> nxt;
        LaneVals<VT, CHECK, BOX, HASW, P> v;
        __builtin_amdgcn_sched_barrier(0);
        if (EARLY) {
            lane_load<0, P, S>(g, qn, nxt);
            __builtin_amdgcn_sched_barrier(0);
            lane_t<0, P, S, VT, CHECK, TAIL>(g, s, q, cur, v);
        } else {
            double lam[P];
            lane_gather<VT, CHECK, TAIL>(g, s, cur, lam);
            __builtin_amdgcn_sched_barrier(0);
            lane_load<0, P, S>(g, qn, nxt);
            __builtin_amdgcn_sched_barrier(0);
            lane_t_gathered<S>(q, cur, lam, v);
        }
        __builtin_amdgcn_sched_barrier(0);
        lane_project<S, VT, CHECK, HASW, TAIL, PJ, P>(g, s, q, gamma, ob, v);
        if (!more) break;
        cur = nxt;
        q = qn;
        ++r;
    }
    return r + 1;
}

// ---------------------------------------------------------------------------
// WG items beyond 8 kWG edges: one workgroup per block of any degree, t
// recomputed on every pass (the block's data stays in L2 between passes)
// ---------------------------------------------------------------------------
template <typename VT, bool CHECK, bool HASW, bool TAIL>
__device__ __forceinline__ double edge_t(const GradArgs& g, const Lds& s, int64_t idx, double& w,
                                         double inv_g)
{
    const VT* __restrict__ A = (const VT*)g.A;
    const VT* __restrict__ C = (const VT*)g.C;
    const double a = (double)Val<VT>::ld(A, idx);
    const double c = (double)Val<VT>::ld(C, idx);
    const int j = g.dst[idx];
    w = HASW ? (double)g.IV[idx] * inv_g : inv_g;
    return -(c + a * get_lam<CHECK, TAIL>(s, g, j));
}

// three sums over the whole workgroup (all threads call it)
__device__ __forceinline__ void wg_sum3d(double& a, double& b, double& c, double* red)
{
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = a;
        red[kWaves + w] = b;
        red[2 * kWaves + w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int i = 0; i < kWaves; ++i) {
        a += red[i];
        b += red[kWaves + i];
        c += red[2 * kWaves + i];
    }
}

// capped-simplex threshold of a WG block held in registers (edge e = k kWG +
// tid); every thread gets the same sums, so the loop is uniform
template <int RW, bool HASW>
__device__ __forceinline__ double wg_cut_threshold(const double (&t)[RW], const float (&u)[RW],
                                                  const float (&wv)[HASW ? RW : 1], const double gamma,
                                                  const double inv_g, double* red)
{
    double s0 = 0.0, z0 = 0.0, z1 = 0.0;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const double w = HASW ? (double)wv[HASW ? k : 0] * inv_g : inv_g;
        const double z = w * t[k];
        s0 += z > 0.0 ? (z < (double)u[k] ? z : (double)u[k]) : 0.0;
    }
    wg_sum3d(s0, z0, z1, red);
    if (!(s0 > 1.0)) return 0.0;
    double lo = 0.0, hi = INFINITY, tau = 0.0;
#pragma unroll 1
    for (int rep = 0; rep < RW * kWG + 4; ++rep) {
        double sw = 0.0, swt = 0.0, su = 0.0;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const float wk = wv[HASW ? k : 0];
            const double w = HASW ? (double)wk * inv_g : inv_g;
            const bool fr = cut_free<HASW>(t[k], u[k], wk, gamma, lo, hi);
            const bool up = cut_upper<HASW>(t[k], u[k], wk, gamma, lo, hi);
            sw += fr ? w : 0.0;
            swt += fr ? w * t[k] : 0.0;
            su += up ? (double)u[k] : 0.0;
        }
        wg_sum3d(sw, swt, su, red);
        const double tf = sw > 0.0 ? (swt + su - 1.0) / sw : lo;
        double dn = 0.0, dup = 0.0, nv = 0.0;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const float wk = wv[HASW ? k : 0];
            const double w = HASW ? (double)wk * inv_g : inv_g;
            const bool fr = cut_free<HASW>(t[k], u[k], wk, gamma, lo, hi);
            const double z = w * (t[k] - tf);
            const bool below = fr && z < 0.0, above = fr && z > (double)u[k];
            dn += below ? -z : 0.0;
            dup += above ? z - (double)u[k] : 0.0;
            nv += (below || above) ? 1.0 : 0.0;
        }
        wg_sum3d(dn, dup, nv, red);
        tau = tf;
        if (nv == 0.0 || !(sw > 0.0)) break;
        if (dn >= dup) lo = fmax(lo, tf);
        else hi = fmin(hi, tf);
    }
    return tau;
}

// the same for WG blocks beyond the register form: t recomputed from memory
// on every pass (the block stays in L2 between passes); et(idx, w) returns
// t of stream position idx and sets w = 1/(gamma v^2)
template <bool HASW, typename ET>
__device__ __forceinline__ double wg_cut_threshold_fn(const GradArgs& g, ET et, const int64_t base, const int d,
                                                     const double gamma, double* red)
{
    double s0 = 0.0, z0 = 0.0, z1 = 0.0;
    for (int e = threadIdx.x; e < d; e += kWG) {
        double w;
        const double t = et(base + e, w);
        const double uu = (double)g.U[base + e];
        const double z = w * t;
        s0 += z > 0.0 ? (z < uu ? z : uu) : 0.0;
    }
    wg_sum3d(s0, z0, z1, red);
    if (!(s0 > 1.0)) return 0.0;
    double lo = 0.0, hi = INFINITY, tau = 0.0;
#pragma unroll 1
    for (int rep = 0; rep < d + 4; ++rep) {
        double sw = 0.0, swt = 0.0, su = 0.0;
        for (int e = threadIdx.x; e < d; e += kWG) {
            double w;
            const double t = et(base + e, w);
            const float uk = g.U[base + e];
            const float wk = HASW ? g.IV[base + e] : 1.0f;
            const bool fr = cut_free<HASW>(t, uk, wk, gamma, lo, hi);
            const bool up = cut_upper<HASW>(t, uk, wk, gamma, lo, hi);
            sw += fr ? w : 0.0;
            swt += fr ? w * t : 0.0;
            su += up ? (double)uk : 0.0;
        }
        wg_sum3d(sw, swt, su, red);
        const double tf = sw > 0.0 ? (swt + su - 1.0) / sw : lo;
        double dn = 0.0, dup = 0.0, nv = 0.0;
        for (int e = threadIdx.x; e < d; e += kWG) {
            double w;
            const double t = et(base + e, w);
            const float uk = g.U[base + e];
            const float wk = HASW ? g.IV[base + e] : 1.0f;
            const bool fr = cut_free<HASW>(t, uk, wk, gamma, lo, hi);
            const double z = w * (t - tf);
            const bool below = fr && z < 0.0, above = fr && z > (double)uk;
            dn += below ? -z : 0.0;
            dup += above ? z - (double)uk : 0.0;
            nv += (below || above) ? 1.0 : 0.0;
        }
        wg_sum3d(dn, dup, nv, red);
        tau = tf;
        if (nv == 0.0 || !(sw > 0.0)) break;
        if (dn >= dup) lo = fmax(lo, tf);
        else hi = fmin(hi, tf);
    }
    return tau;
}
template <typename VT, bool CHECK, bool HASW, bool TAIL>
__device__ __forceinline__ double wg_cut_threshold_mem(const GradArgs& g, const Lds& s, const int64_t base,
                                                      const int d, const double gamma, const double inv_g)
{
    auto et = [&](int64_t idx, double& w) { return edge_t<VT, CHECK, HASW, TAIL>(g, s, idx, w, inv_g); };
    return wg_cut_threshold_fn<HASW>(g, et, base, d, gamma, s.red);
}

template <typename VT, bool CHECK, bool HASW, bool TAIL, int PJ>
__device__ __forceinline__ void wg_block(const GradArgs& g, const Item& it, const Lds& s, double gamma, Obj& ob)
{
    constexpr bool BOX = pj_proj(PJ) != 0;
    constexpr bool DET = pj_det(PJ);
    const int d = uni(it.d);
    const int64_t base = uni64(it.base);
    const double inv_g = 1.0 / gamma;
    double tau = 0.0;
    if constexpr (pj_proj(PJ) == 2) tau = wg_cut_threshold_mem<VT, CHECK, HASW, TAIL>(g, s, base, d, gamma, inv_g);
    if (!BOX) {
        double s0 = 0.0, mx = -INFINITY;
        for (int e = threadIdx.x; e < d; e += kWG) {
            double w;
            const double t = edge_t<VT, CHECK, HASW, TAIL>(g, s, base + e, w, inv_g);
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
                const double t = edge_t<VT, CHECK, HASW, TAIL>(g, s, base + e, w, inv_g);
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
                    const double t = edge_t<VT, CHECK, HASW, TAIL>(g, s, base + e, w, inv_g);
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
    }
    const VT* __restrict__ A = (const VT*)g.A;
    const VT* __restrict__ C = (const VT*)g.C;
    for (int e = threadIdx.x; e < d; e += kWG) {
        const int64_t idx = base + e;
        double w;
        const double t = edge_t<VT, CHECK, HASW, TAIL>(g, s, idx, w, inv_g);
        const double x = xval<BOX>(t, w, tau, BOX ? g.U[idx] : 0.0f);
        if (x != 0.0) {
            const double a = (double)Val<VT>::ld(A, idx);
            const double q2 = HASW ? x * x / (double)g.IV[idx] : x * x;
            ob.ot += t * x;
            ob.oq += q2;
            const double cx = CHECK ? (double)Val<VT>::ld(C, idx) * x : 0.0;
            if (CHECK) ob.oc += cx;
            accum<CHECK, TAIL, DET>(s, g, g.dst[idx], a * x, cx, q2);
        }
        if (g.X) g.X[g.perm[idx]] = x;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Workgroup-sized simplex (uniform weights) and box blocks on one wave each:
// the block is streamed in steps of 64 U edges (the next step's loads in
// flight while the current one is reduced), so no workgroup barrier is
// needed and the eight waves of a workgroup work on different blocks.
// Simplex blocks: one streaming pass gathers the sum of the positive t, the
// two largest t and the edge of the largest; when the largest edge is the
// only one above tau_0 = max(0, max t - gamma) (or the only positive one
// when the sum is at most gamma) it is the whole active set and is added
// from registers.  Otherwise the threshold iteration of the one-lane blocks
// runs with one streaming pass per step, and a last pass adds the active
// edges (as it does when x is written out).
// ---------------------------------------------------------------------------
template <typename VT, bool BOX, bool HASW, int U>
struct WvRaw {
    VT a[U], c[U];
    int j[U];
    float u[BOX ? U : 1];
    float w[HASW ? U : 1];
};
template <int U, typename VT, bool BOX, bool HASW>
__device__ __forceinline__ void wv_load(const GradArgs& g, const int64_t base, const int d, const int e0,
                                        WvRaw<VT, BOX, HASW, U>& r)
{
    const VT* __restrict__ A = (const VT*)g.A + base;
    const VT* __restrict__ C = (const VT*)g.C + base;
    const int32_t* __restrict__ Dst = g.dst + base;
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int e = e0 + 64 * k + lane;
        const uint32_t off = (uint32_t)(e < d ? e : d - 1);
        r.a[k] = ldo(A, off);
        r.c[k] = ldo(C, off);
        r.j[k] = ldo(Dst, off);
        if (BOX) r.u[k] = ldo(g.U + base, off);
        if (HASW) r.w[k] = ldo(g.IV + base, off);
    }
}

// one streaming pass over a block: f(e, t, a, c, j, u, wv) for every edge e
template <int U, typename VT, bool CHECK, bool BOX, bool HASW, bool TAIL, typename F>
__device__ __forceinline__ void wv_stream(const GradArgs& g, const Lds& s, const int64_t base, const int d, F&& f)
{
    using R = typename Val<VT>::reg;
    const int lane = (int)(threadIdx.x & 63);
    WvRaw<VT, BOX, HASW, U> cur;
    wv_load<U>(g, base, d, 0, cur);
#pragma unroll 1
    for (int e0 = 0; e0 < d; e0 += 64 * U) {
        WvRaw<VT, BOX, HASW, U> nxt;
        double lam[U];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < U; ++k) lam[k] = get_lam<CHECK, TAIL>(s, g, cur.j[k]);
        __builtin_amdgcn_sched_barrier(0);
        // (the last step re-reads its own edges: in bounds, never used)
        wv_load<U>(g, base, d, e0 + 64 * U < d ? e0 + 64 * U : e0, nxt);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int e = e0 + 64 * k + lane;
            const R a = Val<VT>::cvt(cur.a[k]);
            const R c = Val<VT>::cvt(cur.c[k]);
            const double t = e < d ? -((double)c + (double)a * lam[k]) : -INFINITY;
            f(e, t, a, c, cur.j[k], BOX ? cur.u[k] : 0.0f, HASW ? cur.w[k] : 1.0f);
        }
        cur = nxt;
    }
}

template <typename VT, bool CHECK, bool HASW, bool TAIL, int PJ>
__device__ __forceinline__ void wave_block(const GradArgs& g, const Item& it, const Lds& s, const double gamma,
                                           Obj& ob)
{
    using R = typename Val<VT>::reg;
    constexpr bool BOX = pj_proj(PJ) == 1;
    constexpr bool DET = pj_det(PJ);
    constexpr int U = sizeof(VT) == 8 ? 4 : 8;
    static_assert(BOX || !HASW, "streamed simplex blocks have uniform weights");
    const int d = uni(it.d);
    const int64_t base = uni64(it.base);
    const double inv_g = 1.0 / gamma;
    // adds edge e's x (x != 0) to the objective parts and the row sums
    auto add = [&](double t, double x, R a, R c, int j, float wv) {
        const double q2 = HASW ? x * x / (double)wv : x * x;
        ob.ot += t * x;
        ob.oq += q2;
        const double cx = CHECK ? (double)c * x : 0.0;
        if (CHECK) ob.oc += cx;
        accum<CHECK, TAIL, DET>(s, g, j, (double)a * x, cx, q2);
    };
    if constexpr (BOX) {
        wv_stream<U, VT, CHECK, true, HASW, TAIL>(g, s, base, d, [&](int e, double t, R a, R c, int j, float u,
                                                                     float wv) {
            const double w = HASW ? (double)wv * inv_g : inv_g;
            const double x = xval<true>(t, w, 0.0, u);
            if (x != 0.0) add(t, x, a, c, j, wv);
            if (g.X && e < d) g.X[g.perm[base + e]] = x;
        });
        return;
    } else {
        // pass 1: sum of positive t, two largest t, the largest edge's values
        double sp = 0.0, m1 = -INFINITY, m2 = -INFINITY, at = 0.0;
        R aa = 0, ac = 0;
        int aj = 0;
        wv_stream<U, VT, CHECK, false, false, TAIL>(g, s, base, d, [&](int, double t, R a, R c, int j, float,
                                                                       float) {
            sp += t > 0.0 ? t : 0.0;
            const bool gt = t > m1;
            m2 = gt ? m1 : fmax(m2, t);
            m1 = gt ? t : m1;
            at = gt ? t : at;
            aa = gt ? a : aa;
            ac = gt ? c : ac;
            aj = gt ? j : aj;
        });
        const double lm1 = m1;
        sp = wave_sum(sp);
        wave_top2(m1, m2);
        // the threshold, as on one-lane blocks of uniform weight
        double tau = 0.0;
        bool single = false;   // active set = the largest edge alone
        if (sp > gamma) {
            tau = m1 - gamma > 0.0 ? m1 - gamma : 0.0;
            single = !(m2 > tau);
        } else {
            // sum of x = sum t+ / gamma <= 1: every positive t is active
            single = !(m2 > 0.0);
        }
        if (sp > gamma && !single) {
            double st = 0.0;
            int n = 0;
            wv_stream<U, VT, CHECK, false, false, TAIL>(g, s, base, d, [&](int, double t, R, R, int, float,
                                                                           float) {
                st += t > tau ? t : 0.0;
                n += t > tau ? 1 : 0;
            });
            st = wave_sum(st);
            n = grp_sum_i<64>(n);
#pragma unroll 1
            for (int rep = 0; rep < 2 * d + 4; ++rep) {
                const double tn = (st - gamma) / (double)n;
                double st2 = 0.0;
                int n2 = 0;
                wv_stream<U, VT, CHECK, false, false, TAIL>(g, s, base, d, [&](int, double t, R, R, int, float,
                                                                               float) {
                    st2 += t > tn ? t : 0.0;
                    n2 += t > tn ? 1 : 0;
                });
                st2 = wave_sum(st2);
                n2 = grp_sum_i<64>(n2);
                tau = tn;
                if (n2 >= n || n2 == 0) break;
                st = st2;
                n = n2;
            }
        }
        if (single && !g.X) {
            // the lane holding the largest t adds it (the first such lane)
            const uint64_t m = __builtin_amdgcn_ballot_w64(lm1 == m1 && m1 > tau);
            if (m != 0 && (int)(threadIdx.x & 63) == (int)__builtin_ctzll(m)) {
                const double x = xval<false>(at, inv_g, tau, 0.0f);
                if (x != 0.0) add(at, x, aa, ac, aj, 1.0f);
            }
            return;
        }
        wv_stream<U, VT, CHECK, false, false, TAIL>(g, s, base, d, [&](int e, double t, R a, R c, int j, float,
                                                                       float) {
            const double x = xval<false>(t, inv_g, tau, 0.0f);
            if (x != 0.0) add(t, x, a, c, j, 1.0f);
            if (g.X && e < d) g.X[g.perm[base + e]] = x;
        });
    }
}

// WG items of up to kWG * RW edges with the block in registers: edge
// e = k kWG + tid, k < RW; all loads of a block issued at once, then the
// threshold by workgroup reductions (every thread gets the same sums, so the
// loop is uniform across the workgroup).  Runs of blocks of one class are
// pipelined like the lane runs: the next block's loads are in flight while
// the current block is reduced.
template <int RW, typename VT, bool BOX, bool HASW>
__device__ __forceinline__ void wg_load(const GradArgs& g, const int64_t base, const int d,
                                        LaneRaw<VT, BOX, HASW, RW>& r)
{
    const VT* __restrict__ A = (const VT*)g.A + base;
    const VT* __restrict__ C = (const VT*)g.C + base;
    const int32_t* __restrict__ Dst = g.dst + base;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const int e = k * kWG + (int)threadIdx.x;
        const uint32_t off = (uint32_t)(e < d ? e : d - 1);
        r.a[k] = ldo(A, off);
        r.c[k] = ldo(C, off);
        r.j[k] = ldo(Dst, off);
        if (BOX) r.u[k] = ldo(g.U + base, off);
        if (HASW) r.w[k] = ldo(g.IV + base, off);
    }
}

template <int RW, typename VT, bool CHECK, bool BOX, bool HASW>
__device__ __forceinline__ void wg_t(const int d, const LaneRaw<VT, BOX, HASW, RW>& r, const double (&lam)[RW],
                                     LaneVals<VT, CHECK, BOX, HASW, RW>& v)
{
    using R = typename Val<VT>::reg;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        v.a[k] = Val<VT>::cvt(r.a[k]);
        const R c = Val<VT>::cvt(r.c[k]);
        v.j[k] = r.j[k];
        if (BOX) v.u[k] = r.u[k];
        if (HASW) v.w[k] = r.w[k];
        const double tk = -((double)c + (double)v.a[k] * lam[k]);
        v.t[k] = k * kWG + (int)threadIdx.x < d ? tk : -INFINITY;
        if (CHECK) v.c[k] = c;
    }
}

template <int RW, typename VT, bool CHECK, bool HASW, bool TAIL, int PJ>
__device__ __forceinline__ void wg_project(const GradArgs& g, const Lds& s, const int64_t base, const int d,
                                           const double gamma, Obj& ob, const LaneVals<VT, CHECK, pj_proj(PJ) != 0, HASW, RW>& v)
{
    constexpr bool BOX = pj_proj(PJ) != 0;
    constexpr bool DET = pj_det(PJ);
    const double inv_g = 1.0 / gamma;
    const double* t = v.t;
    double tau = 0.0;
    if constexpr (pj_proj(PJ) == 2) tau = wg_cut_threshold<RW, HASW>(v.t, v.u, v.w, gamma, inv_g, s.red);
    if (!BOX) {
        // uniform weights: the two largest t; with the second at most tau_0 =
        // max t - 1/w only the largest is active and tau_0 is the threshold
        double s0 = 0.0, mx = -INFINITY, m2 = -INFINITY;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
            const double z = w * t[k];
            s0 += z > 0.0 ? z : 0.0;
            if (HASW) {
                mx = fmax(mx, t[k] - 1.0 / w);
            } else {
                m2 = fmax(m2, fmin(mx, t[k]));
                mx = fmax(mx, t[k]);
            }
        }
        if (HASW) {
            wg_sum_max(s0, mx, s.red);
        } else {
            wg_sum_top2(s0, mx, m2, s.red);
            mx = mx - 1.0 / inv_g;
        }
        if (s0 > 1.0) tau = mx > 0.0 ? mx : 0.0;
        if (s0 > 1.0 && (HASW || m2 > tau)) {
            double sw = 0.0, swt = 0.0;
            int n = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
                const bool in = t[k] > tau;
                sw += in ? w : 0.0;
                swt += in ? w * t[k] : 0.0;
                n += in ? 1 : 0;
            }
            wg_sum3(sw, swt, n, s.red);
#pragma unroll 1
            for (int rep = 0; rep < 2 * d + 4; ++rep) {
                const double tn = (swt - 1.0) / sw;
                double sw2 = 0.0, swt2 = 0.0;
                int n2 = 0;
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
                    const bool in = t[k] > tn;
                    sw2 += in ? w : 0.0;
                    swt2 += in ? w * t[k] : 0.0;
                    n2 += in ? 1 : 0;
                }
                wg_sum3(sw2, swt2, n2, s.red);
                tau = tn;
                if (n2 >= n || n2 == 0) break;
                sw = sw2;
                swt = swt2;
                n = n2;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const double w = HASW ? (double)v.w[k] * inv_g : inv_g;
        const double x = xval<BOX>(t[k], w, tau, BOX ? v.u[k] : 0.0f);
        if (x != 0.0) {
            const double q2 = HASW ? x * x / (double)v.w[k] : x * x;
            ob.ot += t[k] * x;
            ob.oq += q2;
            const double cx = CHECK ? (double)v.c[k] * x : 0.0;
            if (CHECK) ob.oc += cx;
            accum<CHECK, TAIL, DET>(s, g, v.j[k], (double)v.a[k] * x, cx, q2);
        }
        const int e = k * kWG + (int)threadIdx.x;
        if (g.X && e < d) g.X[g.perm[base + e]] = x;
    }
}

__device__ __forceinline__ int wg_class(int d) { return d <= 2 * kWG ? 2 : d <= 4 * kWG ? 4 : 8; }

// descriptor i of a WG item.  The item table is read-only while a kernel
// runs: loading it through the constant address space, as four dwords (a
// scalar load has no byte form), gives scalar loads, counted apart from the
// vector memory operations, so reading a descriptor never waits for
// outstanding prefetches or global atomics (a vector load of it would, its
// value being needed in scalar registers).
__device__ __forceinline__ Item wg_item(const GradArgs& g, const int i)
{
    typedef const __attribute__((address_space(4))) uint32_t CU32;
    const CU32* p = (CU32*)(g.items + i);
    const uint32_t w0 = p[0], w1 = p[1], w2 = p[2], w3 = p[3];
    Item it;
    it.base = (int64_t)(((uint64_t)w1 << 32) | w0);
    it.d = (int32_t)w2;
    it.nb = (uint8_t)(w3 & 0xFF);
    it.lg = (uint8_t)((w3 >> 8) & 0xFF);
    it.kind = (uint8_t)((w3 >> 16) & 0xFF);
    it.proj = (uint8_t)(w3 >> 24);
    return it;
}

// WG items i, i+1, ... of class RW and one projection type; returns the first
// item not processed
template <int RW, typename VT, bool CHECK, bool HASW, bool TAIL, int PJ>
__device__ __forceinline__ int wg_run(const GradArgs& g, int i, const int i1, const Lds& s, double gamma, Obj& ob)
{
    constexpr bool BOX = pj_proj(PJ) != 0;
    constexpr bool EARLY = !TAIL;   // lam from LDS
    Item it = wg_item(g, i);
    int64_t base = uni64(it.base);
    int d = uni(it.d);
    LaneRaw<VT, BOX, HASW, RW> cur;
    wg_load<RW>(g, base, d, cur);
#pragma unroll 1
    for (;;) {
        bool more = false;
        int64_t bn = base;
        int dn = d;
        if (i + 1 < i1) {
            const Item nx = wg_item(g, i + 1);
            const int nd = uni(nx.d);
            if (nx.proj == pj_proj(PJ) && nd <= 8 * kWG && wg_class(nd) == RW) {
                more = true;
                bn = uni64(nx.base);
                dn = nd;
            }
        }
        LaneRaw<VT, BOX, HASW, RW> nxt;
        LaneVals<VT, CHECK, BOX, HASW, RW> v;
        double lam[RW];
        __builtin_amdgcn_sched_barrier(0);
        if (EARLY) {
            wg_load<RW>(g, bn, dn, nxt);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < RW; ++k) lam[k] = get_lam<CHECK, TAIL>(s, g, cur.j[k]);
        } else {
#pragma unroll
            for (int k = 0; k < RW; ++k) lam[k] = get_lam<CHECK, TAIL>(s, g, cur.j[k]);
            __builtin_amdgcn_sched_barrier(0);
            wg_load<RW>(g, bn, dn, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
        wg_t<RW>(d, cur, lam, v);
        wg_project<RW, VT, CHECK, HASW, TAIL, PJ>(g, s, base, d, gamma, ob, v);
        if (!more) break;
        cur = nxt;
        base = bn;
        d = dn;
        ++i;
    }
    __syncthreads();
    return i + 1;
}

// ---------------------------------------------------------------------------
// the fused gradient kernel: one workgroup per chunk
// ---------------------------------------------------------------------------
// lane items from batch entry r on; returns the first entry not processed
template <typename VT, bool CHECK, bool HASW, bool TAIL, int PJ, bool ODD>
__device__ __forceinline__ int lane_dispatch(const GradArgs& g, const Item& mine, const int r, const int rn,
                                             const Item& it, const Lds& s, double gamma, Obj& ob)
{
    // FP64 storage keeps blocks of at most 8 edges in lanes (register budget);
    // per-edge weights (and rows beyond LDS) need more registers, so their
    // pipelined runs stop at smaller classes and their one-lane blocks at 16
    // edges (the layout guarantees d <= CAP for S = 1 and R <= RMAX for S > 1)
    constexpr bool W8 = sizeof(VT) == 8;
    // capped-simplex blocks: at most kCutLaneCap edges on one lane and
    // kCutRmax rows per lane of a segment (the layout guarantees it), which
    // keeps their threshold loops within the register budget
    constexpr int RMAX = pj_proj(PJ) == 2 ? (seg_rmax(W8, HASW, TAIL) < kCutRmax ? seg_rmax(W8, HASW, TAIL) : kCutRmax)
                                 : seg_rmax(W8, HASW, TAIL);
    constexpr int CAP = pj_proj(PJ) == 2 ? (lane_cap(W8, HASW, TAIL) < kCutLaneCap ? lane_cap(W8, HASW, TAIL) : kCutLaneCap)
                                : lane_cap(W8, HASW, TAIL);
    const int cls = lane_class<VT, HASW, TAIL>(it.d, it.lg);
    // blocks on S = 2^lg lanes: the host picks the S that pads a block's
    // degree least (S times the row class) among lg = 1..6 for the ordinary
    // kernels (ODD), among lg = 2, 4, 6 for those of problems with capped
    // blocks or in deterministic mode (their code stays smaller)
    switch (it.lg) {
    case 1:
        if constexpr (ODD) {
            if (cls == 8) return lane_run<2, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
            return lane_run<2, VT, CHECK, HASW, TAIL, PJ, RMAX>(g, mine, r, rn, s, gamma, ob);
        }
        break;
    case 2:
        if (cls == 8) return lane_run<4, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
        return lane_run<4, VT, CHECK, HASW, TAIL, PJ, RMAX>(g, mine, r, rn, s, gamma, ob);
    case 3:
        if constexpr (ODD) {
            if (cls == 8) return lane_run<8, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
            return lane_run<8, VT, CHECK, HASW, TAIL, PJ, RMAX>(g, mine, r, rn, s, gamma, ob);
        }
        break;
    case 4:
        if (cls == 8) return lane_run<16, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
        return lane_run<16, VT, CHECK, HASW, TAIL, PJ, RMAX>(g, mine, r, rn, s, gamma, ob);
    case 5:
        if constexpr (ODD) {
            if (cls == 8) return lane_run<32, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
            return lane_run<32, VT, CHECK, HASW, TAIL, PJ, RMAX>(g, mine, r, rn, s, gamma, ob);
        }
        break;
    case 6:
        if (cls == 8) return lane_run<64, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
        return lane_run<64, VT, CHECK, HASW, TAIL, PJ, RMAX>(g, mine, r, rn, s, gamma, ob);
    default:
        break;
    }
    switch (cls) {
    case 4: return lane_run<1, VT, CHECK, HASW, TAIL, PJ, 4>(g, mine, r, rn, s, gamma, ob);
    case 8: return lane_run<1, VT, CHECK, HASW, TAIL, PJ, 8>(g, mine, r, rn, s, gamma, ob);
    case 12:
        if constexpr (RMAX >= 12) return lane_run<1, VT, CHECK, HASW, TAIL, PJ, W8 ? 8 : 12>(g, mine, r, rn, s, gamma, ob);
        lane_group<VT, CHECK, HASW, TAIL, PJ, W8 ? 8 : 12>(g, it, s, gamma, ob);
        return r + 1;
    case 16:
        if constexpr (RMAX >= 16) return lane_run<1, VT, CHECK, HASW, TAIL, PJ, W8 ? 8 : 16>(g, mine, r, rn, s, gamma, ob);
        lane_group<VT, CHECK, HASW, TAIL, PJ, W8 ? 8 : 16>(g, it, s, gamma, ob);
        return r + 1;
    case 24:
        if constexpr (CAP > 16) lane_group<VT, CHECK, HASW, TAIL, PJ, 24>(g, it, s, gamma, ob);
        return r + 1;
    default:
        if constexpr (CAP > 24) lane_group<VT, CHECK, HASW, TAIL, PJ, 32>(g, it, s, gamma, ob);
        return r + 1;
    }
}

template <typename VT, bool CHECK, bool HASW, bool TAIL, bool CUT, bool DET>
__device__ __forceinline__ void grad_body(const GradArgs& g, const int chunk)
{
    if (g.done && *g.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    Lds s;
    s.lam_rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)g.lam, (short)0, g.J * 8, 0x00020000);
    s.red = (double*)smem;
    unsigned char* p = smem + 4 * kWaves * sizeof(double);
    const int K = g.K;
    // rows of the c x and v^2 x^2 sums in LDS (check passes)
    const int KC = CHECK ? g.Kc : 0;
    // bytes of one LDS sum: f32, or a 64-bit integer in deterministic mode
    constexpr size_t es = DET ? 8 : 4;
    constexpr int D4 = DET ? 4 : 0;   // the deterministic bit of the projection codes
    constexpr bool LAM_LDS = !(CHECK && TAIL);
    s.lam = nullptr;
    if (LAM_LDS) {
        s.lam = (double*)p;
        p += (size_t)K * sizeof(double);
    }
    // ordinary passes of problems without rows beyond LDS (outside
    // deterministic mode) keep the a x sums in FP64
    constexpr bool WIDE = !CHECK && !DET && !TAIL;
    s.hg = (float*)p;
    s.hgd = WIDE ? (double*)p : nullptr;
    p += (size_t)K * (WIDE ? sizeof(double) : es);
    s.hc = s.hq = nullptr;
    if (CHECK) {
        s.hc = (float*)p;
        p += (size_t)KC * es;
        s.hq = (float*)p;
    }
    const double gamma = g.gamma_ptr ? *g.gamma_ptr : g.gamma_val;
    // LDS rows: lam (8 rows per thread in flight at once) and zeroed sums
    {
        int j = threadIdx.x;
        if (LAM_LDS) {
            for (; j + 7 * kWG < K; j += 8 * kWG) {
                double l[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) l[u] = g.lam[j + u * kWG];
#pragma unroll
                for (int u = 0; u < 8; ++u) s.lam[j + u * kWG] = l[u];
            }
            for (; j < K; j += kWG) s.lam[j] = g.lam[j];
        }
        if constexpr (DET) {
            for (j = threadIdx.x; j < K; j += kWG) ((unsigned long long*)s.hg)[j] = 0ull;
            if (CHECK)
                for (j = threadIdx.x; j < KC; j += kWG) {
                    ((unsigned long long*)s.hc)[j] = 0ull;
                    ((unsigned long long*)s.hq)[j] = 0ull;
                }
        } else if constexpr (WIDE) {
            for (j = threadIdx.x; j < K; j += kWG) s.hgd[j] = 0.0;
        } else {
            for (j = threadIdx.x; j < K; j += kWG) s.hg[j] = 0.0f;
            if (CHECK)
                for (j = threadIdx.x; j < KC; j += kWG) {
                    s.hc[j] = 0.0f;
                    s.hq[j] = 0.0f;
                }
        }
    }
    __syncthreads();

    const Chunk ch = g.chunks[chunk];
    Obj ob = {0.0, 0.0, 0.0};
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // this wave's share of the chunk's lane items (bounds read with scalar
    // loads); their descriptors arrive 64 at a time (lane r holds item r of
    // the batch) and are broadcast with readlane, so a group waits on its
    // data only
    {
        typedef const __attribute__((address_space(4))) int32_t CI32;
        const CI32* wb = (CI32*)&g.chunks[chunk].w[0];
        const bool strided = wb[0] < 0;
        const int i0 = strided ? ch.a0 + wave : wb[wave];
        const int step = strided ? kWaves : 1;
        const int nmine = strided ? (ch.a1 - ch.a0 > wave ? (ch.a1 - ch.a0 - wave + kWaves - 1) / kWaves : 0)
                                  : wb[wave + 1] - i0;
        for (int r0 = 0; r0 < nmine; r0 += 64) {
            const int lane = threadIdx.x & 63;
            const int my = i0 + (r0 + lane) * step;
            Item mine = {0, 0, 0, 0, 0, 0};
            if (r0 + lane < nmine) mine = g.items[my];
            const int rn = nmine - r0 < 64 ? nmine - r0 : 64;
            for (int r = 0; r < rn;) {
                const Item it = item_at(mine, r);
                constexpr bool ODD = !CUT && !DET;
                if (it.proj == 1) {
                    r = lane_dispatch<VT, CHECK, HASW, TAIL, 1 | D4, ODD>(g, mine, r, rn, it, s, gamma, ob);
                } else if (it.proj == 2) {
                    // capped blocks exist only in problems launched with CUT
                    if constexpr (CUT)
                        r = lane_dispatch<VT, CHECK, HASW, TAIL, 2 | D4, ODD>(g, mine, r, rn, it, s, gamma, ob);
                    else r = rn;
                } else {
                    r = lane_dispatch<VT, CHECK, HASW, TAIL, 0 | D4, ODD>(g, mine, r, rn, it, s, gamma, ob);
                }
            }
        }
    }
    // WG items of box blocks and of simplex blocks with uniform weights: one
    // wave per block, the waves independent (items wave, wave + kWaves, ...)
    auto streamed = [&](const Item& it) { return it.proj == 1 || (it.proj == 0 && !HASW); };
    for (int i = ch.b0 + wave; i < ch.b1; i += kWaves) {
        const Item it = wg_item(g, i);
        if (it.proj == 1) wave_block<VT, CHECK, HASW, TAIL, 1 | D4>(g, it, s, gamma, ob);
        else if constexpr (!HASW) {
            if (it.proj == 0) wave_block<VT, CHECK, false, TAIL, 0 | D4>(g, it, s, gamma, ob);
        }
    }
    // the others (capped blocks, simplex blocks with per-edge weights) on the
    // whole workgroup
    for (int i = ch.b0; i < ch.b1;) {
        const Item it = wg_item(g, i);
        if (streamed(it)) {
            ++i;
            continue;
        }
        const int d = uni(it.d);
        if (d > 8 * kWG) {
            if (it.proj == 1) wg_block<VT, CHECK, HASW, TAIL, 1 | D4>(g, it, s, gamma, ob);
            else if (it.proj == 0) wg_block<VT, CHECK, HASW, TAIL, 0 | D4>(g, it, s, gamma, ob);
            else if constexpr (CUT) wg_block<VT, CHECK, HASW, TAIL, 2 | D4>(g, it, s, gamma, ob);
            ++i;
            continue;
        }
        const int rw = wg_class(d);
        if (it.proj == 1) {
            if (rw == 2) i = wg_run<2, VT, CHECK, HASW, TAIL, 1 | D4>(g, i, ch.b1, s, gamma, ob);
            else if (rw == 4) i = wg_run<4, VT, CHECK, HASW, TAIL, 1 | D4>(g, i, ch.b1, s, gamma, ob);
            else i = wg_run<8, VT, CHECK, HASW, TAIL, 1 | D4>(g, i, ch.b1, s, gamma, ob);
        } else if (it.proj == 2) {
            if constexpr (CUT) {
                if (rw == 2) i = wg_run<2, VT, CHECK, HASW, TAIL, 2 | D4>(g, i, ch.b1, s, gamma, ob);
                else if (rw == 4) i = wg_run<4, VT, CHECK, HASW, TAIL, 2 | D4>(g, i, ch.b1, s, gamma, ob);
                else i = wg_run<8, VT, CHECK, HASW, TAIL, 2 | D4>(g, i, ch.b1, s, gamma, ob);
            } else {
                i = ch.b1;
            }
        } else {
            if (rw == 2) i = wg_run<2, VT, CHECK, HASW, TAIL, 0 | D4>(g, i, ch.b1, s, gamma, ob);
            else if (rw == 4) i = wg_run<4, VT, CHECK, HASW, TAIL, 0 | D4>(g, i, ch.b1, s, gamma, ob);
            else i = wg_run<8, VT, CHECK, HASW, TAIL, 0 | D4>(g, i, ch.b1, s, gamma, ob);
        }
    }
    __syncthreads();

    // flush: this chunk's row of partial sums, and its objective part
    const int64_t plane = (int64_t)g.nchunks * K;
    if constexpr (DET) {
        unsigned long long* row = (unsigned long long*)g.part + (int64_t)chunk * K;
        for (int j = threadIdx.x; j < K; j += kWG) row[j] = ((const unsigned long long*)s.hg)[j];
        if (CHECK)
            for (int j = threadIdx.x; j < KC; j += kWG) {
                row[plane + j] = ((const unsigned long long*)s.hc)[j];
                row[2 * plane + j] = ((const unsigned long long*)s.hq)[j];
            }
    } else {
        float* row = g.part + (int64_t)chunk * K;
        if constexpr (WIDE)
            for (int j = threadIdx.x; j < K; j += kWG) row[j] = (float)s.hgd[j];
        else
            for (int j = threadIdx.x; j < K; j += kWG) row[j] = s.hg[j];
        if (CHECK)
            for (int j = threadIdx.x; j < KC; j += kWG) {
                row[plane + j] = s.hc[j];
                row[2 * plane + j] = s.hq[j];
            }
    }
    ob.ot = wave_sum(ob.ot);
    ob.oq = wave_sum(ob.oq);
    ob.oc = wave_sum(ob.oc);
    if ((threadIdx.x & 63) == 0) {
        s.red[threadIdx.x >> 6] = ob.ot;
        s.red[kWaves + (threadIdx.x >> 6)] = ob.oq;
        s.red[2 * kWaves + (threadIdx.x >> 6)] = ob.oc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            a += s.red[i];
            b += s.red[kWaves + i];
            c += s.red[2 * kWaves + i];
        }
        g.obj_part[3 * chunk] = a;
        g.obj_part[3 * chunk + 1] = b;
        g.obj_part[3 * chunk + 2] = c;
    }
}

template <typename VT, bool CHECK, bool HASW, bool TAIL, bool CUT, bool DET>
__global__ __launch_bounds__(kWG) void grad_kernel(GradArgs g)
{
    grad_body<VT, CHECK, HASW, TAIL, CUT, DET>(g, blockIdx.x);
}

// batched form: workgroup b runs chunk ct[b].y of problem ct[b].x
template <typename VT, bool CHECK, bool HASW, bool TAIL, bool CUT, bool DET>
__global__ __launch_bounds__(kWG) void grad_kernel_batch(const GradArgs* __restrict__ tab,
                                                          const int2* __restrict__ ct)
{
    const int2 e = ct[blockIdx.x];
    const GradArgs g = tab[e.x];
    grad_body<VT, CHECK, HASW, TAIL, CUT, DET>(g, e.y);
}

template <typename VT, bool CHECK, bool HASW, bool TAIL, bool CUT, bool DET>
static hipError_t launch_grad_t(const GradArgs& a, hipStream_t s)
{
    const size_t lds = grad_lds_bytes(a.K, a.Kc, CHECK, TAIL, DET);
    hipLaunchKernelGGL((grad_kernel<VT, CHECK, HASW, TAIL, CUT, DET>), dim3(a.nchunks), dim3(kWG), lds, s, a);
    return hipGetLastError();
}

template <typename VT, bool CUT, bool DET>
hipError_t launch_grad_vt(const GradArgs& a, bool check, bool has_w, hipStream_t s)
{
    const bool tail = a.K < a.J;
#define DL_L(C, W, T) if (check == C && has_w == W && tail == T) return launch_grad_t<VT, C, W, T, CUT, DET>(a, s);
    DL_L(false, false, false) DL_L(false, false, true) DL_L(false, true, false) DL_L(false, true, true)
    DL_L(true, false, false) DL_L(true, false, true) DL_L(true, true, false) DL_L(true, true, true)
#undef DL_L
    return hipErrorInvalidValue;
}

template <typename VT, bool CHECK, bool HASW, bool TAIL, bool CUT, bool DET>
static hipError_t launch_grad_batch_t(const GradArgs* tab, const int2* ct, int nblocks, size_t lds,
                                      hipStream_t s)
{
    hipLaunchKernelGGL((grad_kernel_batch<VT, CHECK, HASW, TAIL, CUT, DET>), dim3(nblocks), dim3(kWG), lds, s, tab,
                       ct);
    return hipGetLastError();
}

template <typename VT, bool CUT, bool DET>
hipError_t launch_grad_batch_vt(const GradArgs* tab, const int2* ct, int nblocks, size_t lds, bool check,
                                bool has_w, bool tail, hipStream_t s)
{
#define DL_L(C, W, T) \
    if (check == C && has_w == W && tail == T) return launch_grad_batch_t<VT, C, W, T, CUT, DET>(tab, ct, nblocks, lds, s);
    DL_L(false, false, false) DL_L(false, false, true) DL_L(false, true, false) DL_L(false, true, true)
    DL_L(true, false, false) DL_L(true, false, true) DL_L(true, true, false) DL_L(true, true, true)
#undef DL_L
    return hipErrorInvalidValue;
}

template <typename VT, bool CUT, bool DET>
hipError_t set_grad_attributes_vt(size_t lds)
{
    hipError_t e = hipSuccess, r;
#define DL_A(C, W, T)                                                                        \
    r = hipFuncSetAttribute((const void*)grad_kernel<VT, C, W, T, CUT, DET>,                     \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
    if (r != hipSuccess) e = r;                                                              \
    r = hipFuncSetAttribute((const void*)grad_kernel_batch<VT, C, W, T, CUT, DET>,               \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
    if (r != hipSuccess) e = r;
    DL_A(false, false, false) DL_A(false, false, true) DL_A(false, true, false) DL_A(false, true, true)
    DL_A(true, false, false) DL_A(true, false, true) DL_A(true, true, false) DL_A(true, true, true)
#undef DL_A
    return e;
}

// CUT: the variant that also handles capped-simplex blocks; DET: the variant
// with fixed-point integer sums (deterministic mode, instantiated with CUT).
// Each variant is compiled in its own translation unit, so problems of one
// kind never carry the code (and register pressure) of the others.
#define DL_INSTANTIATE_GRAD(VT, CUT, DET)                                                    \
    template hipError_t launch_grad_vt<VT, CUT, DET>(const GradArgs&, bool, bool, hipStream_t); \
    template hipError_t launch_grad_batch_vt<VT, CUT, DET>(const GradArgs*, const int2*, int, size_t, bool, \
                                                           bool, bool, hipStream_t);         \
    template hipError_t set_grad_attributes_vt<VT, CUT, DET>(size_t);


}  // namespace dl
