// Register-blocked float32 cell Sinkhorn for 8 x 8 X blocks (declarations).
#pragma once

#include <vector>

#include "sinkhorn.hpp"

namespace dd {

// Launch split of one solve on the register-blocked path, per cell class (0: box long side
// <= 32, one wave per cell, log nu_J in registers; 1: the rest up to 2048 box entries, four
// waves per cell; 2: larger boxes, eight waves per cell).
constexpr int kClasses = 3;
struct FastInfo {
    int n[kClasses] = {0, 0, 0};    // cells
    int lds[kClasses] = {0, 0, 0};  // LDS bytes per workgroup
    // batch rule: launches (all of them), their summed duration and LSE terms
    int launches[kClasses] = {0, 0, 0};
    double ms[kClasses] = {0.0, 0.0, 0.0};
    double terms[kClasses] = {0.0, 0.0, 0.0};
    int stop_it = 0;          // batch rule: the iteration the rule stopped at
    bool final_done = true;   // f and g of that iteration are in p.a, p.b
    double terms_per_it[kClasses] = {0.0, 0.0, 0.0};  // LSE terms of one iteration per class
    int spec_slots = 0;       // kFastSpec: event slots of the rounds enqueued
};

// fast_solve phases: the whole solve; rounds enqueued with no host wait (batch rule, the
// caller resumes if they were not enough); the resumption of such a solve
constexpr int kFastAll = 0, kFastSpec = 1, kFastResume = 2;

// An upper bound on the iterations kFastSpec's rounds run (stop tests `chunk` apart at least).
int fast_spec_max_iters(int chunk);

// True when the batch runs on the register-blocked path: float32 terms, 8 x 8 X blocks,
// every box side at most kFastMaxSide, every class's workgroup within the LDS of a CU, and
// the path not switched off (DD_FAST=0).
bool fast_eligible(const SkBatch& p, const std::vector<int32_t>& hd);

// Cell classes of the register-blocked path: boxes whose long side is at most wave_side get a
// wave each, boxes of more than big_entries entries eight waves, the rest four.
struct FastClasses {
    int wave_side = 32, big_entries = 2048;
};
// The classes for a batch: a forced pair (sinkhorn_set_classes), or the tuner's pick for the
// batch's key (the mode, the mean box area in powers of four, the cell count in powers of two);
// every
// candidate is tried once on consecutive solves of a key, then the one with the least float32
// time per LSE term stays.  Returns false when the batch does not take the register-blocked
// path.  `choice` / `key` identify the pick for fast_record.
bool fast_plan(const SkBatch& p, const std::vector<int32_t>& hd, const dd_sinkhorn_opts& o,
               FastClasses* cls, int* choice, int key[3]);
void fast_record(const int key[3], int choice, double ms_per_term);
void fast_force(int wave_side, int big_entries);
constexpr int kFastMaxSide = 512;

// The float32 phase of a solve (the caller runs the float64 finish): writes f to p.a, g to
// p.b, per-cell iterations, errors and masses (w.cell_mass), and the control words read by
// the statistics (done iteration ctrl[2], converged ctrl[4]).  Same options and stopping
// rules as the general kernels, except that the batch rule is tested at iterations the
// device chooses from the error's decay (at least max(1, o.check_every) apart), and that a
// tolerance solve aims at 0.85 o.tol (the float64 finish certifies o.tol).
// `ord`: the cells in order of decreasing work (each class keeps that order, most work first).
// `final_pass` (batch rule): end with the Y-update of the X potential whose error stopped the
// rule (f and g of that iteration in p.a, p.b); without it, when a float64 finish follows, p.a
// keeps the X-update of the last iteration (the start of the next one) and p.b is left to the
// finish, and every cell's iteration count is the float32 phase's.
Status fast_solve(const SkBatch& p, const dd_sinkhorn_opts& o, hipStream_t st, SkWork& w,
                  const std::vector<int32_t>& hd, const std::vector<int32_t>& ord,
                  int32_t* iters, double* errs, FastInfo* info, bool final_pass = true,
                  int32_t* h_ord = nullptr, FastClasses cls = FastClasses{},
                  int phase = kFastAll, int spec_rounds = 4);
// h_ord: pinned host room for n ints (the order is uploaded from there without waiting), or
// NULL (no-allocation mode: uploaded from a temporary, then waited for).
// phase kFastSpec (batch rule, not in no-allocation mode): enqueue spec_rounds (at most four) rounds and the
// per-cell counts of their stop iteration (0 if none) without a host wait, and return;
// kFastResume (same arguments, after the caller has waited and copied w.ctrl to w.h_ctl32):
// continue that solve from where the four rounds left it.

}  // namespace dd
