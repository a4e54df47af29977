// The domain-decomposition context (opaque dd_ctx of the C ABI).
#pragma once

#include <string>
#include <vector>

#include "cells.hpp"
#include "dual.hpp"
#include "sinkhorn.hpp"

struct FlowState;
struct dd_net;

struct dd_ctx {
    // multiscale: coarser layers below the finest, the current layer (0 = coarsest) and the
    // marginals of every layer (host, [0] coarsest ... [levels] finest)
    int levels = 0, layer = 0;
    std::vector<std::vector<double>> pyr_mu, pyr_nu;
    // problem (of the current layer)
    int N = 0, s = 0, n = 0, nI = 0, AS = 0, prec = DD_PREC_F32;
    double h = 0.0, trunc = 1e-15;
    hipStream_t st = nullptr;
    dd::Mem mem;  // device-memory supplier of every buffer below and of the workspaces
    std::vector<int32_t> h_dims;  // composite box dims of the current iteration (host)
    int64_t* h_small = nullptr;   // pinned: sizes read back at the end of an iteration
    std::string err;
    std::vector<double> m;  // basic cell masses (host copy)
    std::vector<int32_t> pmembers[2], pxorig[2];
    double* d_mu = nullptr;
    double* d_nu = nullptr;
    double* d_lognu_glob = nullptr;
    double* d_m = nullptr;
    // partitions and their persistent X potentials (warm start)
    dd::PartDev part[2];
    double* d_logmu[2] = {nullptr, nullptr};
    double* d_a[2] = {nullptr, nullptr};
    int32_t* d_gst[2] = {nullptr, nullptr};
    bool visited[2] = {false, false};
    double kappa_a[2] = {1.0, 1.0};
    // state
    dd::BoxSet S, S2;
    // composite work of the current / last iteration
    dd::CompDev C;
    double* d_nuJ = nullptr;
    size_t nuJ_cap = 0;
    double* d_lognu = nullptr;
    size_t lognu_cap = 0;
    double* d_b = nullptr;
    size_t b_cap = 0;
    double* d_tmp = nullptr;
    size_t tmp_cap = 0;
    double* d_py2 = nullptr;
    int64_t* d_nsize = nullptr;
    int32_t* d_flags = nullptr;
    int32_t* d_iters = nullptr;
    double* d_cerr = nullptr;
    double* d_scratch = nullptr;
    double* d_cell_out = nullptr;
    double* d_basic_out = nullptr;
    double* d_eval = nullptr;
    dd::SkWork skw;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // composite box dims of both partitions, computed on the device at the end of the last
    // iteration from the state it left and copied to pinned memory with its final wait, so
    // that the next iteration plans its solve without waiting; valid until anything else
    // changes the state (dd_forget_pred)
    int32_t* d_pred[2] = {nullptr, nullptr};  // [cells][2]
    int32_t* h_pred[2] = {nullptr, nullptr};  // pinned copies
    bool pred_ok[2] = {false, false};
    int32_t* d_pcheck = nullptr;  // [1] set on the device when a prediction was wrong
    int last_part = -1;
    double last_eps = 0.0;
    int last_mw1 = 0, last_mw2 = 0;
    int untruncated_cells = 0;
    FlowState* flow = nullptr;
    // learned warm start (borrowed net) and its per-cell buffers
    dd_net* net = nullptr;
    float* d_nx = nullptr;  // [cells][8][32][32] features
    size_t nx_cap = 0;
    float* d_ng = nullptr;  // [cells][32][32] predicted corrections of the Y potential
    size_t ng_cap = 0;
    double* d_a0 = nullptr;  // [cells][xside^2] previous-iterate start of the last iteration
    size_t a0_cap = 0;
    dd::DualWork dual;
    // sequential batches of composite cells (bounding-box clusters; domdec_set_clusters)
    int clusters = 1;
    struct Batch {
        dd::CompDev C;                 // the batch's composite boxes ([cap] cells)
        int32_t* idx = nullptr;        // [cap] composite cells of the batch (partition ids)
        int32_t* members = nullptr;    // [cap][4]
        int32_t* xorig = nullptr;      // [cap][2]
        int32_t* gst = nullptr;        // [cap][2]
        double* a = nullptr;           // [cap][xside^2] X potentials
        double* logmu = nullptr;       // [cap][xside^2]
        int32_t* list = nullptr;       // [4 cap] basic cells of the batch
        int64_t* lsize = nullptr;      // [4 cap + 1] their sizes, then prefix sums
        int cap = 0;
        int64_t* stage_base = nullptr; // [nI] staging offset of every basic cell
        double* staging = nullptr;     // truncated boxes of all batches, batch after batch
        size_t staging_cap = 0;
        int64_t peak_entries = 0;      // largest batch of the last iteration (composite entries)
        int count = 0;                 // batches of the last iteration
    } bt;
    // one saved copy of the mutable state (domdec_save / domdec_restore)
    struct Snap {
        bool valid = false;
        int32_t* box = nullptr;
        int64_t* base = nullptr;
        double* data = nullptr;
        size_t data_cap = 0;
        int64_t ntot = 0;
        double* a[2] = {nullptr, nullptr};
        int32_t* gst[2] = {nullptr, nullptr};
        bool visited[2] = {false, false};
        double kappa_a[2] = {1.0, 1.0};
    } snap;
};

void dd_ctx_release(dd_ctx* c);
// Called by every entry point that changes the state other than an iteration.
inline void dd_forget_pred(dd_ctx* c) { c->pred_ok[0] = c->pred_ok[1] = false; }
// Evaluation reductions of the last iteration's composite plans; with pix_out ([N*N][3]) also
// the per-pixel X moments of the plans.
void dd_eval_cells(dd_ctx* c, double* pix_out = nullptr);
void flow_release(dd_ctx* c);
