// Stitched global dual point of a domain-decomposition state (declarations).
#pragma once

#include "common.hpp"

namespace dd {

struct DualArgs {
    int N = 0, s = 0, xside = 0;
    int ncell[2] = {0, 0};
    const int32_t* members[2] = {nullptr, nullptr};  // host [ncell][4] basic ids (-1 absent)
    const int32_t* xorig[2] = {nullptr, nullptr};    // device [ncell][2] X block origins
    const double* a[2] = {nullptr, nullptr};         // device [ncell][xside^2] potentials f
    const int32_t* gst[2] = {nullptr, nullptr};      // device [ncell][2] gauge offsets G
    double kappa[2] = {1.0, 1.0};                    // kappa of each partition's last solve
    double kappa_eval = 1.0, eps = 1.0;
    const double* mu = nullptr;                      // device [N*N]
    const double* nu = nullptr;                      // device [N*N]
};

struct DualWork {
    double* buf = nullptr;   // [5][N*N]
    double* d = nullptr;     // [nI]
    int32_t* own = nullptr;  // [nI]
    double* sA = nullptr;    // [ncell A]
    double* part = nullptr;  // partial sums
    Mem mem;                 // supplier of the buffers above
};

// alpha+ / eps_eval on every pixel (device [N*N], inside w): the A cells' potentials with the
// breadth-first offsets; valid until the next call on w.
Status stitched_alpha(const DualArgs& a, DualWork& w, hipStream_t st, const double** fdag);
// D = eps (<alpha+/eps, mu> + <beta+/eps, nu>) of the stitched dual point.
Status stitched_dual(const DualArgs& a, DualWork& w, hipStream_t st, double* D);
void dual_release(DualWork& w);

}  // namespace dd
