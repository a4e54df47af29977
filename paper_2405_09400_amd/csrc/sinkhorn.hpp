// Batched separable log-domain cell Sinkhorn on gfx950 (declarations).
#pragma once

#include <vector>

#include "common.hpp"

namespace dd {

// Device-side description of a batch of cell problems (see sinkhorn_batch in domdec.h).
// Inputs and potentials are float64; `prec` selects the arithmetic of the log-sum-exp terms.
struct SkBatch {
    int ncells = 0;
    int xside = 0;                   // X block side (2s)
    const int32_t* dims = nullptr;   // [ncells][2] W1, W2
    const int64_t* base = nullptr;   // [ncells] packed Y offset
    const int32_t* shift = nullptr;  // [ncells][2] E1, E2
    const double* logmu = nullptr;   // [ncells][xside^2]
    const double* lognu = nullptr;   // packed Y boxes
    double* a = nullptr;             // [ncells][xside^2] f, in/out
    double* b = nullptr;             // packed Y boxes, g out
    const int32_t* order = nullptr;  // processing order, most work first (set by sk_solve)
    double kappa = 1.0;
    int max_w1 = 0, max_w2 = 0;
    // set by sk_solve for each launch: the cells order[q_lo, q_hi) and their LDS tile bound,
    // and the per-cell global scratch offsets (in doubles) of boxes beyond the tile
    int q_lo = 0, q_hi = 0;
    int lw1 = 0, lw2 = 0;
    const int64_t* scr_off = nullptr;
    int prec = DD_PREC_F32;
};

// Scratch owned by the caller (reused across solves).
struct SkWork {
    double* a_alt = nullptr;    // second X-potential buffer for the batch rule
    size_t a_alt_n = 0;
    double* cell_err = nullptr; // [cap]
    double* cell_mass = nullptr;
    int32_t* cell_iters = nullptr;
    int32_t* iters64 = nullptr; // [cap] float64-finish iterations
    int* ctrl = nullptr;        // [16] device control words (queue, ticket, done, flags)
    int* ctrl64 = nullptr;      // [16] control words of a speculative float64 finish
    double* dtot = nullptr;     // [8] device totals
    void* big = nullptr;        // scratch for Y boxes beyond the LDS tile (g, z in global memory)
    size_t big_bytes = 0;
    int64_t* scr_off = nullptr; // [cap] per-cell scratch offsets
    int32_t* order = nullptr;   // processing order of the main run
    int order_cap = 0;
    int4* recs = nullptr;       // register-blocked path: per queue slot, the cell's record
    int recs_cap = 0;
    int32_t* order64 = nullptr; // processing order and scratch offsets of the float64 finish
    int64_t* scr_off64 = nullptr;
    int order64_cap = 0;
    int cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    hipEvent_t evj = nullptr;     // joins the caller's stream and `stream`
    hipEvent_t evf = nullptr, evj2 = nullptr;  // fork / join of `stream` and `stream2`
    hipStream_t stream = nullptr; // the solver's own streams (default priority): small cells
    hipStream_t stream2 = nullptr;  // and the other classes run side by side
    hipStream_t stream3 = nullptr;
    hipEvent_t evj3 = nullptr;
    hipEvent_t kev[3][2][4] = {};  // register-blocked path: start/end of each class's rounds
    // No-allocation mode: every buffer above is carved from a device arena the caller owns
    // (bump allocation from the start of the arena on every solve), all work runs on the
    // caller's stream, and no events, streams or graphs are created (statistics carry no
    // times).
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    Mem mem;  // supplier of the buffers above outside no-allocation mode
    // Pinned host staging (outside no-allocation mode): the launch plans are copied to the
    // device from here without waiting, and the statistics come back here; a solve's uploads
    // are complete before the next solve starts (every solve synchronises at least once).
    char* h_stage = nullptr;
    size_t h_stage_cap = 0;
    int* h_ctl = nullptr;       // [16] control words of the last solve
    int* h_ctl32 = nullptr;     // [16] a speculative solve's float32-phase control words
    int64_t waits = 0;          // host waits for the device so far (statistics)
    // float32 rounds a speculative solve enqueues, by batch size (the last four sizes seen)
    int spec_n[4] = {0, 0, 0, 0}, spec_r[4] = {0, 0, 0, 0}, spec_next = 0;
    double* h_tot = nullptr;    // [8] its totals
    // what a solve with deferred statistics leaves for sk_finish
    struct Pend {
        bool active = false, fast = false, run64 = false, tune = false;
        int ncells = 0, fixed_iters = 0, stop_rule = 0, choice = 0;
        int key[4] = {0, 0, 0, 0};
        int n[3] = {0, 0, 0}, lds[3] = {0, 0, 0}, launches[3] = {0, 0, 0};
        double ms[3] = {0.0, 0.0, 0.0}, terms[3] = {0.0, 0.0, 0.0};
        int n_big = 0, n_giant = 0, small_tile[2] = {0, 0}, big_tile[2] = {0, 0};
        size_t small_budget = 0, big_budget = 0;
        int fchoice = -1, fkey[3] = {0, 0, 0};  // register-blocked path: the tuner's pick
        int wave_side = 0, big_entries = 0;     // and the class thresholds used
        double terms32 = 0.0;                   // LSE terms of the float32 phase
        bool spec = false;                      // enqueued speculatively (see sk_solve)
        int spec_slots = 0;                     // its float32 rounds' event slots
        double tpi[3] = {0.0, 0.0, 0.0};        // and LSE terms per iteration per class
    } pend;
    // A speculative solve (sk_solve with spec): what its resumption needs, if the rounds and
    // float64 iterations enqueued without a host wait turn out not to be enough.
    struct Spec {
        bool need_resume = false;
        SkBatch p, q64;
        dd_sinkhorn_opts o{};
        std::vector<int32_t> hd, ord;
        std::vector<int64_t> cls64;  // the float64 finish's classes: mode, lo, hi, t0, t1, budget,
                                     // threads
        int wave_side = 0, big_entries = 0;
        int first64 = 2;  // float64-finish iterations launched speculatively
        int32_t* iters = nullptr;
        double* errs = nullptr;
        hipStream_t caller = nullptr;
    } spec;
};

// Carve n elements from the no-allocation arena (256-byte aligned); DD_EINVAL when the arena
// is too small for the batch.
template <typename P>
inline Status arena_take(SkWork& w, P*& p, size_t n) {
    Status st;
    const size_t bytes = ((n > 0 ? n : 1) * sizeof(P) + 255) & ~(size_t)255;
    if (w.arena_used + bytes > w.arena_bytes) {
        st.code = DD_EINVAL;
        st.msg = "sinkhorn: the batch needs more scratch than the no-allocation entry point's "
                 "fixed buffer holds";
        return st;
    }
    p = reinterpret_cast<P*>(w.arena + w.arena_used);
    w.arena_used += bytes;
    return st;
}

Status sk_work_reserve(SkWork& w, int ncells, size_t a_n);
void sk_work_release(SkWork& w);

// LDS bytes of the per-cell X arrays of one workgroup (every Y box fits: boxes beyond the
// LDS tile run from global scratch), or 0 when xside is out of range.
size_t sk_lds_bytes(int xside, int prec);

// host_dims: the cells' box dims already on the host ([ncells][2], as p.dims), or NULL to read
// them back.  defer: leave the statistics in w (pinned) and return without waiting for the
// solve; the caller synchronises its stream and then calls sk_finish, which also reports a
// stop that missed the tolerance.  Not in no-allocation mode.
//
// spec (with defer, on the register-blocked path under the batch rule): enqueue the whole solve
// without any host wait -- a fixed number of float32 rounds (the rounds after the stop exit
// at once), a device gate, and the first float64 finish iterations (which exit at once when
// the float32 phase has not stopped).  sk_finish then sets w.spec.need_resume when that was
// not enough; sk_resume continues the solve exactly where it stands (the same iterations and
// results as a solve without spec), after which the caller redoes whatever it enqueued
// behind the solve and calls sk_finish again.
Status sk_solve(const SkBatch& p, const dd_sinkhorn_opts& o, hipStream_t st, SkWork& w,
                dd_batch_stats* stats, int32_t* cell_iters_out, double* cell_err_out,
                const int32_t* host_dims = nullptr, bool defer = false, bool spec = false);
Status sk_finish(SkWork& w, dd_batch_stats* stats);
Status sk_resume(SkWork& w);

// iters[c] = ctrl[2] (the batch rule's stop iteration) for every cell
void launch_done_iters(int ncells, int32_t* iters, const int* ctrl, hipStream_t st);

// Algorithmic work of one iteration of one cell (for the statistics).
inline double sk_cell_terms(int a, int W1, int W2) {
    return (double)a * W2 * (a + W1) + (double)a * W1 * (W2 + a);
}

}  // namespace dd
