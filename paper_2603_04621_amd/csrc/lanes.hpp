// Cross-lane reductions shared by the HIP kernels of libdualip.
#pragma once
#include <hip/hip_runtime.h>

namespace dl {

// ---------------------------------------------------------------------------
// wave / workgroup reductions.  Within a row of 16 lanes they use DPP lane
// moves (quad_perm [1,0,3,2] and [2,3,0,1], row half-mirror, row mirror):
// each step adds a lane's partner value, the partners compute the same sum,
// so every lane of an aligned group of S lanes ends with the same bits.  Rows
// are combined with readlane (wave-uniform).  A reduction must be reached by
// every lane of the wave (no divergent exec mask), which all callers keep.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dpp32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp32<CTRL>((int)b);
    const int hi = dpp32<CTRL>((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double rdlane64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within 16

// sums / max over aligned groups of S lanes (S a power of two up to 64)
template <int S>
__device__ __forceinline__ double grp_sum(double v)
{
    if (S >= 2) v += dpp64<kDppXor1>(v);
    if (S >= 4) v += dpp64<kDppXor2>(v);
    if (S >= 8) v += dpp64<kDppHalfMirror>(v);
    if (S >= 16) v += dpp64<kDppMirror>(v);
    if (S == 32) {
        const double r0 = rdlane64(v, 0), r1 = rdlane64(v, 16), r2 = rdlane64(v, 32), r3 = rdlane64(v, 48);
        v = (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
    } else if (S == 64) {
        const double r0 = rdlane64(v, 0), r1 = rdlane64(v, 16), r2 = rdlane64(v, 32), r3 = rdlane64(v, 48);
        v = (r0 + r1) + (r2 + r3);
    }
    return v;
}
template <int S>
__device__ __forceinline__ double grp_max(double v)
{
    if (S >= 2) v = fmax(v, dpp64<kDppXor1>(v));
    if (S >= 4) v = fmax(v, dpp64<kDppXor2>(v));
    if (S >= 8) v = fmax(v, dpp64<kDppHalfMirror>(v));
    if (S >= 16) v = fmax(v, dpp64<kDppMirror>(v));
    if (S == 32) {
        const double r0 = rdlane64(v, 0), r1 = rdlane64(v, 16), r2 = rdlane64(v, 32), r3 = rdlane64(v, 48);
        v = (threadIdx.x & 32) ? fmax(r2, r3) : fmax(r0, r1);
    } else if (S == 64) {
        const double r0 = rdlane64(v, 0), r1 = rdlane64(v, 16), r2 = rdlane64(v, 32), r3 = rdlane64(v, 48);
        v = fmax(fmax(r0, r1), fmax(r2, r3));
    }
    return v;
}
// largest and second largest value (with multiplicity) over aligned groups of
// S lanes; every lane enters its own top two (m1 >= m2)
__device__ __forceinline__ void top2_merge(double& m1, double& m2, const double p1, const double p2)
{
    m2 = fmax(fmin(m1, p1), fmax(m2, p2));
    m1 = fmax(m1, p1);
}
template <int CTRL>
__device__ __forceinline__ void top2_step(double& m1, double& m2)
{
    const double p1 = dpp64<CTRL>(m1), p2 = dpp64<CTRL>(m2);
    top2_merge(m1, m2, p1, p2);
}
template <int S>
__device__ __forceinline__ void grp_top2(double& m1, double& m2)
{
    if (S >= 2) top2_step<kDppXor1>(m1, m2);
    if (S >= 4) top2_step<kDppXor2>(m1, m2);
    if (S >= 8) top2_step<kDppHalfMirror>(m1, m2);
    if (S >= 16) top2_step<kDppMirror>(m1, m2);
    if (S >= 32) {
        double a1 = rdlane64(m1, 0), a2 = rdlane64(m2, 0);
        double b1 = rdlane64(m1, 16), b2 = rdlane64(m2, 16);
        top2_merge(a1, a2, b1, b2);
        double c1 = rdlane64(m1, 32), c2 = rdlane64(m2, 32);
        const double d1 = rdlane64(m1, 48), d2 = rdlane64(m2, 48);
        top2_merge(c1, c2, d1, d2);
        if (S == 64) {
            top2_merge(a1, a2, c1, c2);
            m1 = a1;
            m2 = a2;
        } else {
            const bool hi = (threadIdx.x & 32) != 0;
            m1 = hi ? c1 : a1;
            m2 = hi ? c2 : a2;
        }
    }
}
template <int S>
__device__ __forceinline__ int grp_sum_i(int v)
{
    if (S >= 2) v += dpp32<kDppXor1>(v);
    if (S >= 4) v += dpp32<kDppXor2>(v);
    if (S >= 8) v += dpp32<kDppHalfMirror>(v);
    if (S >= 16) v += dpp32<kDppMirror>(v);
    if (S == 32) {
        const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
        const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
        v = (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
    } else if (S == 64) {
        v = (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
            (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
    }
    return v;
}
__device__ __forceinline__ double wave_sum(double v) { return grp_sum<64>(v); }
__device__ __forceinline__ double wave_max(double v) { return grp_max<64>(v); }
__device__ __forceinline__ void wave_top2(double& m1, double& m2) { grp_top2<64>(m1, m2); }
__device__ __forceinline__ int wave_sum_i(int v) { return grp_sum_i<64>(v); }

}  // namespace dl
