// Host-side state of a created problem and helpers shared by the ABI files.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dualip.h"
#include "common.hpp"
#include "kernels.hpp"

struct dl_problem {
    int device = 0;
    int64_t m = 0, n = 0, nblocks = 0;
    int storage = 1;
    int has_box = 0, has_w = 0, solve_ok = 1;
    int has_cut = 0;                   // some block is a capped simplex
    int nf = 1;                        // entries per column (several families, dense rows)
    int dense_f = -1, dense_row = 0;   // plane holding one row for every column, and that row
    void* A2[dl::kMfPlanes - 1] = {};  // planes 1..nf-1 of the coefficients
    int32_t* dst2[dl::kMfPlanes - 1] = {};   // and their rows (internal order)
    double* srow = nullptr;            // [J] restoration ratios (nf > 1)
    double* corr_part = nullptr;       // [nchunks] restoration partials (nf > 1)
    int det = 0;                       // deterministic mode: fixed-point sums
    double qs[3] = {1.0, 1.0, 1.0};    // their scales (a x, c x, v^2 x^2)
    double anorm2 = 1.0;               // |A'|^2 of the iteration matrix (presets)
    int J = 0, K = 0;                  // rows; rows resident in LDS
    int Kc = 0;                        // rows of the check-pass c x, v^2 x^2 sums in LDS
    int nchunks = 0, nitems = 0, nblk2 = 0;
    int64_t n_lane = 0, n_seg = 0, n_wg = 0;
    int lane_cap = 0, seg_rmax = 0, chunk_mult = 1, wg_min = 0, tuned = 0;   // work layout
    int64_t stream_bytes = 0;
    size_t device_bytes = 0;
    // edge stream
    void* A = nullptr;
    void* C = nullptr;
    int32_t* dst = nullptr;
    float* U = nullptr;
    float* IV = nullptr;
    int64_t* perm = nullptr;
    dl::Item* items = nullptr;
    dl::Chunk* chunks = nullptr;
    // rows (internal order)
    double* b = nullptr;
    double* D = nullptr;
    int32_t* orig = nullptr;
    // scratch of one evaluation
    float* part = nullptr;
    double* tail = nullptr;
    double* obj_part = nullptr;
    double* blockpart = nullptr;
    double* lam_int = nullptr;
    double* eval6 = nullptr;
    // solve state
    double *lam = nullptr, *y = nullptr, *yp = nullptr, *G = nullptr, *Gp = nullptr,
           *lam_eval = nullptr;
    dl::SolveState* st = nullptr;
    dl::SolveState* st_host = nullptr;   // pinned mirror (2 slots)
    std::vector<void*> allocs;
    // the last solve's graph of `seg` iterations, replayed by later solves
    // with the same parameters (no trace); freed with the problem
    struct {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t ev[2] = {nullptr, nullptr};
        int64_t seg = 0, check_every = 0;
        dl::SolveParams prm;
    } gc;
};

namespace dlh {

void set_error(const char* fmt, ...);
dl_status hip_fail(hipError_t e, const char* what);

// gradient + reduction of one pass (mode 0: solve, 1: evaluation)
dl::GradArgs grad_args(const dl_problem* p, const double* lam, const double* gamma_ptr,
                       double gamma_val, const int32_t* done, double* X);
dl::ReduceArgs reduce_args(const dl_problem* p, int check, int mode, const double* lam,
                           const double* gamma_ptr, double gamma_val, const int32_t* done,
                           double* grad_out);
dl::AgdArgs agd_args(const dl_problem* p, const dl::SolveParams& prm, int check, double* trace);

// enqueues one full iteration (gradient, reduction, ascent step)
hipError_t enqueue_iteration(dl_problem* p, const dl::SolveParams& prm, int check, double* trace,
                             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);

// frees a problem whose device work the caller has already waited for
// (no device-wide synchronization, unlike dl_problem_destroy)
void destroy_idle(dl_problem* p);

// raises the gradient kernels' dynamic-LDS limit to the device maximum, once
// per device (thread-safe)
hipError_t ensure_grad_attributes(int device);

dl_status check_solve_opts(const dl_solve_opts* o);
// dl_problem_validate that also reports the most entries in one column
dl_status validate_desc(const dl_problem_desc* d, const dl_problem_opts* o, int* col_entries);
// solve parameters of problem p (its preset resolved with p's |A'|^2)
dl::SolveParams make_params(const dl_solve_opts* o, const dl_problem* p);
bool is_check_iter(const dl_solve_opts* o, int64_t k);

}  // namespace dlh
