// Kernel arguments and launchers of libdualip (host and device see these).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace dl {

// Fused dual-gradient pass: t = -(c + a lam_dst), blockwise projection,
// per-destination sums of a x (and c x, v^2 x^2 on check passes), and the
// per-edge part of the dual objective, sum_e c x + gamma/2 v^2 x^2.
struct GradArgs {
    const void* A;           // [n] storage type
    const void* C;           // [n] storage type
    const int32_t* dst;      // [n] relabelled destination
    const float* U;          // [n] box bounds or null (no box block)
    const float* IV;         // [n] 1/v^2 or null (v = 1)
    const int64_t* perm;     // [n] original column of each stream position
    double* X;               // [n] x output (original column order) or null
    const Item* items;
    const Chunk* chunks;
    const double* lam;       // [J] lam in caller units, internal row order
    const double* gamma_ptr; // device scalar, or null to use gamma_val
    double gamma_val;
    const int32_t* done;     // early-exit flag or null
    int32_t J, K;            // rows; rows kept in LDS
    int32_t nchunks;
    int32_t Kc;              // check passes: rows whose c x and v^2 x^2 sums stay in LDS
    float* part;             // [planes][nchunks][K] (64-bit integers when det)
    double* tail;            // [3][J] FP64 accumulators of rows beyond LDS (integers when det)
    double* obj_part;        // [nchunks][3]: sum t x, sum v^2 x^2, sum c x (check)
    int32_t det, pad_det;    // deterministic mode: fixed-point integer sums
    double qs[3];            // their scales (a x, c x, v^2 x^2)
    // columns with several entries (grad_mf_kernel): planes 1..nf-1 of the
    // coefficients and rows (plane 0 is A, dst)
    const void* A2[kMfPlanes - 1];
    const int32_t* dst2[kMfPlanes - 1];
    int32_t nf;              // entries per column (1: the one-family kernels)
    int32_t restore;         // restoration pass of the gap (see grad_mf.hpp)
    int32_t dense_f;         // plane whose row is the same for every column (a dense
                             // row such as the count row), -1: none
    int32_t dense_row;       // that row (internal order)
    const double* srow;      // [J] min(1, b_j / (A x)_j), internal row order
    double* corr_part;       // [nchunks] restoration correction of P
};

// Per-destination combination of the chunk partial sums.
struct ReduceArgs {
    const float* part;
    int32_t nchunks, K, J, check, mode;   // mode 0: solve (lam' space), 1: evaluation
    int32_t Kc;              // rows whose c x and v^2 x^2 partials are in `part`
    double* tail;
    const double* b;         // [J] internal order
    const double* D;         // [J] row scale
    const double* lam;       // [J] the point evaluated, caller units
    const double* y;         // solve: y', y'_prev, G'_prev
    const double* yp;
    const double* Gp;
    double* G;               // solve: out G' = D (A x - b)
    const int32_t* orig;     // evaluation: original row of internal row j
    double* grad_out;        // evaluation: out (A x - b) in original row order
    const double* gamma_ptr;
    double gamma_val;
    const int32_t* done;
    double* blockpart;       // [gridDim.x][kRedStride]
    int32_t det, pad_det;    // partials and accumulators are 64-bit integers
    double iqs[3];           // their inverse scales
    double* srow;            // check passes of multi-entry columns: out s_j, or null
};

struct AgdArgs {
    SolveState* st;
    SolveParams prm;
    int32_t check, nchunks, nblk, J;
    const double* obj_part;
    const double* blockpart;
    double* lam;
    double* y;
    double* yp;
    double* G;
    double* Gp;
    double* lam_eval;
    const double* D;
    double* trace;           // [max_iters][6] or null
    const double* corr_part; // [nchunks] restoration corrections (multi-entry columns), or null
};

// dynamic LDS of a gradient launch.  Ordinary passes: lam (FP64) and the
// a x sums of K rows.  Check passes of problems without tail rows: the same
// plus the c x and v^2 x^2 sums of Kc rows; with tail rows (lam read from
// memory): the a x sums of K rows and the other two of Kc rows.  A sum is an
// f32, or a 64-bit integer in deterministic mode.
size_t grad_lds_bytes(int K, int Kc, bool check, bool tail, bool det);

// storage: 0 f64, 1 f32, 2 bf16 (a, c); cut: the problem has capped-simplex
// blocks (the kernel variant that handles them); a.det selects the
// deterministic variant
hipError_t launch_grad(const GradArgs& a, int storage, bool check, bool has_w, bool cut, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, int nblk, hipStream_t s);
hipError_t launch_agd(const AgdArgs& a, hipStream_t s);
hipError_t launch_permute_in(const double* src, const int32_t* orig, int J, double* dst,
                             hipStream_t s);
hipError_t launch_eval_finish(const double* obj_part, int nchunks, const double* blockpart,
                              int nblk, int check, double gamma, double* out6, hipStream_t s,
                              const double* corr_part = nullptr);
// multi-entry columns: the fused gradient pass (or, with a.restore, the
// restoration pass); storage as launch_grad
hipError_t launch_grad_mf(const GradArgs& a, int storage, bool has_w, hipStream_t s);
hipError_t launch_solve_init(SolveState* st, SolveParams prm, const double* lam_in,
                             const int32_t* orig, const double* D, int J, double* lam, double* y,
                             double* yp, double* G, double* Gp, double* lam_eval, hipStream_t s);
hipError_t launch_solve_final(const SolveState* st, const double* y, const double* yp,
                              const int32_t* orig, const double* D, int J, double* lam_out,
                              hipStream_t s);
hipError_t set_grad_attributes(size_t max_lds);

// batched forms: tables of per-problem argument blocks in device memory
hipError_t launch_grad_batch(const GradArgs* tab, const int2* ct, int nblocks, size_t lds, int storage,
                             bool check, bool has_w, bool tail, bool cut, bool det, hipStream_t s);
hipError_t launch_reduce_batch(const ReduceArgs* tab, const int2* rt, int nblocks, hipStream_t s);
hipError_t launch_agd_batch(const AgdArgs* tab, int count, hipStream_t s);
hipError_t launch_count_done(const AgdArgs* tab, int count, int* out, hipStream_t s);
hipError_t launch_gather_states(const AgdArgs* tab, int count, SolveState* out, hipStream_t s);

}  // namespace dl
