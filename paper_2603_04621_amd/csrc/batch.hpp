// Batched iteration over several problems: one fused gradient launch per
// kernel-variant group (storage, primal scale, rows beyond LDS, capped
// blocks, deterministic sums), one reduction launch and one ascent launch
// per iteration, all driven by per-problem argument tables on the device.
// Each problem keeps its own chunking, reduction order and FP64 state, so a
// problem's iterates are the same alone and in a batch.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "problem.hpp"

namespace dlh {

class BatchRunner {
public:
    ~BatchRunner() { release(); }
    // Builds the tables for `probs` (solve mode) with parameters prm[k].
    dl_status build(const std::vector<dl_problem*>& probs, const std::vector<dl::SolveParams>& prm,
                    hipStream_t s);
    // Enqueues one iteration of every problem (check pass when check != 0).
    hipError_t enqueue_iteration(int check, hipStream_t s) const;
    // Number of finished problems (waits for the stream).
    hipError_t count_done(hipStream_t s, int* ndone);
    // Copies all states to host (waits for the stream).
    hipError_t states(hipStream_t s, std::vector<dl::SolveState>& out);
    void release();
    int count() const { return (int)probs_.size(); }

private:
    struct Group {
        int storage, has_w, tail, cut, det;
        int c0, nblocks;
        size_t lds;
    };
    std::vector<dl_problem*> probs_;
    std::vector<Group> groups_;
    dl::GradArgs* gtab_ = nullptr;
    dl::ReduceArgs* rtab_[2] = {nullptr, nullptr};
    dl::AgdArgs* atab_[2] = {nullptr, nullptr};
    int2* ctab_ = nullptr;
    int2* rbt_ = nullptr;
    int nrb_ = 0;
    int* ndone_dev_ = nullptr;
    int* ndone_host_ = nullptr;
    dl::SolveState* st_dev_ = nullptr;
    dl::SolveState* st_host_ = nullptr;   // pinned copy of st_dev_
    size_t st_cap_ = 0;
    size_t cap_[7] = {0, 0, 0, 0, 0, 0, 0};   // allocated entries of the seven tables
};

}  // namespace dlh
