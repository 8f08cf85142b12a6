// Internal layout shared by the host code and the HIP kernels of libdualip.
//
// Device layout of one problem (built once by dl_problem_create):
//
//   Edge stream.  Every primal variable (edge e = (source i, destination j))
//   sits at one stream position holding a_e, c_e (storage type), dst_e (int32,
//   destination after relabelling), and when needed u_e (box bound, f32),
//   iv_e = 1/v_e^2 (primal scale, f32) and perm_e (original column, int64,
//   only read when x is requested).
//
//   Work items.  Blocks are grouped by projection type and degree d into
//   LANE items: groups of nb blocks of one exact degree, each block on
//   S = 2^lg consecutive lanes of a wave (S = 1 up to d <= lane_cap, else
//   the smallest S in {4, 16, 64} with ceil(d/S) <= seg_rmax rows per lane),
//   edge k S + s of block b at base + k nb S + b S + s for the full rows and
//   the last row compacted (see grad_impl.hpp), so every load of a row is
//   one contiguous run and the projection runs in registers with reductions
//   over the block's lanes.  Blocks longer than 64 seg_rmax edges are WG
//   items: one workgroup per block, edge k at base + k.
//
//   Chunks.  The workgroups of the fused gradient kernel each take one
//   chunk: the LANE items dealt round-robin in (S, projection, degree) order,
//   and likewise the WG items, so every chunk gets the same mix of sizes.
//   Each chunk owns one row of the per-destination partial-sum buffer, so
//   results do not depend on timing.
//
//   Destinations.  Relabelled by descending degree; the first K (lds_rows)
//   live in LDS during the gradient pass (lam in FP64 and f32 partial sums),
//   the rest read lam from global memory and add to FP64 global accumulators.
#pragma once
#include <stdint.h>

namespace dl {

constexpr int kWG = 512;                // threads of a gradient workgroup
constexpr int kWaves = kWG / 64;
constexpr int kLaneMaxDeg = 32;         // one-lane blocks (registers: 32 edges per lane)
constexpr int kLaneMaxDegF64 = 8;       // one-lane blocks with FP64 storage

// Largest degree of a one-lane block (S = 1): 8 with FP64 storage; 16 when
// per-edge weights or rows beyond LDS add registers (the 24- and 32-edge
// groups would spill there), else 32.  The host lays the stream out with it
// and the kernel variant of the same (storage, weights, tail) compiles only
// these classes.
constexpr int lane_cap(bool f64, bool has_w, bool tail)
{
    return f64 ? kLaneMaxDegF64 : ((has_w || tail) ? 16 : kLaneMaxDeg);
}
// Largest rows per lane of a multi-lane block (S > 1); blocks longer than
// 64 * seg_rmax edges are WG items.
constexpr int seg_rmax(bool f64, bool has_w, bool tail)
{
    return f64 ? 8 : (has_w ? 8 : (tail ? 12 : 16));
}

// Capped-simplex blocks take at most kCutLaneCap edges on one lane and
// kCutRmax rows per lane of a segment (their threshold loop keeps bounds and
// a bracket beside the values; larger classes would spill registers).
constexpr int kCutLaneCap = 16;
constexpr int kCutRmax = 8;

// Columns with several entries (several matching families, dense rows): at
// most kMfPlanes entries per column; blocks take at most kMfLaneCap edges on
// one lane and kMfRmax rows per lane (the entries multiply the registers per
// edge).
constexpr int kMfPlanes = 4;
constexpr int kMfLaneCap = 8;
constexpr int kMfRmax = 8;

enum ItemKind : uint8_t { ITEM_LANE = 0, ITEM_WG = 2 };

struct Item {                // 16 bytes
    int64_t base;            // first stream position
    int32_t d;               // degree (edges per block)
    uint8_t nb;              // blocks in the group (LANE), 1 otherwise
    uint8_t lg;              // log2 of lanes per block (LANE)
    uint8_t kind;            // ItemKind
    uint8_t proj;            // dl_proj
};
static_assert(sizeof(Item) == 16, "Item layout");

struct Chunk {               // lane items [a0, a1), workgroup blocks [b0, b1)
    int32_t a0, a1, b0, b1;
    // lane items of wave q of the one-entry kernels: [w[q], w[q + 1]), a
    // contiguous share of [a0, a1) (items of one class stay together, so a
    // wave's prefetch pipeline seldom restarts at a class change); w[0] < 0:
    // items a0 + q, a0 + q + kWaves, ... instead
    int32_t w[kWaves + 1];
};
// layouts with at most this many lane-item classes use the strided shares
constexpr int kStridedClasses = 12;

// Scalars of the iteration that live on the device (one per solve slot).
struct SolveState {
    double gamma, eta, eta_cap, tm;
    double g, P, rel_gap, max_infeas, gnorm, obj;
    double gamma_eval;       // gamma of the last evaluation
    int64_t k, ks;
    int64_t kmax;            // iteration cap of the solve (set at init)
    int32_t stage, done, converged, status;
    int32_t stage_eval, pad;
    // the step the scalar kernel chose for the row kernel
    double step_eta, step_beta;
    int32_t step_adv, step_stop;
};

// Constant parameters of a solve (kernel argument).
struct SolveParams {
    double gamma0, gamma_final, stage_tol, tol, max_step, init_step;
    int64_t stage_iters, max_iters, check_every;
    int32_t n_stages, momentum, adaptive, pad;
};

// Number of per-block FP64 sums written by the reduction kernel.
constexpr int kRedStride = 8;
// 0: sum lam_j b_j   1: |G'|^2   2: |G'-G'_prev|^2   3: |y'-y'_prev|^2
// 4: gap correction sum_j (s_j-1) C_j + gamma/2 (s_j^2-1) Q_j   5: max infeasibility

}  // namespace dl
