// Register-blocked float32 cell Sinkhorn for 8 x 8 X blocks (declarations).
#pragma once

#include <vector>

#include "sinkhorn.hpp"

namespace dd {

// Launch split of one solve on the register-blocked path.
struct FastInfo {
    int n_wave = 0;   // cells solved by one wave (long box side <= 32)
    int n_group = 0;  // cells solved by a workgroup of four waves
    int lds_wave = 0, lds_group = 0;  // LDS bytes of one cell slice per class
    // batch rule: launches (all of them), their summed duration and LSE terms per class
    // (0: one wave per cell, 1: a workgroup per cell)
    int launches[2] = {0, 0};
    double ms[2] = {0.0, 0.0};
    double terms[2] = {0.0, 0.0};
};

// True when the batch runs on the register-blocked path: float32 terms, 8 x 8 X blocks,
// every box side at most kFastMaxSide, and the path not switched off (DD_FAST=0).
bool fast_eligible(const SkBatch& p, const std::vector<int32_t>& hd);
constexpr int kFastMaxSide = 512;

// The float32 phase of a solve (the caller runs the float64 finish): writes f to p.a, g to
// p.b, per-cell iterations, errors and masses (w.cell_mass), and the control words read by
// the statistics (done iteration ctrl[2], converged ctrl[4]).  Same options and stopping
// rules as the general kernels, except that the batch rule is tested every
// max(1, o.check_every)-th iteration.
Status fast_solve(const SkBatch& p, const dd_sinkhorn_opts& o, hipStream_t st, SkWork& w,
                  const std::vector<int32_t>& hd, int32_t* iters, double* errs, FastInfo* info);

}  // namespace dd
