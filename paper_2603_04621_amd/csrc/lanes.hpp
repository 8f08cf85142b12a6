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
__device__ __forceinline__ int wave_sum_i(int v) { return grp_sum_i<64>(v); }

}  // namespace dl
