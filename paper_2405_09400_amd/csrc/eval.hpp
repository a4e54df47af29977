// Float64 quality reductions and per-cell moments (declarations).
#pragma once

#include "common.hpp"

namespace dd {

struct EvalArgs {
    using T = double;
    int ncell = 0, xside = 0, s = 0, maxw1 = 0, maxw2 = 0, N = 0;
    const int32_t *members = nullptr, *xorig = nullptr, *cdims = nullptr, *corig = nullptr,
                  *cshift = nullptr, *gofs = nullptr;
    const int64_t* cbase = nullptr;
    const T *logmu = nullptr, *a = nullptr, *b = nullptr, *lognuJ = nullptr;
    const double *nuJ = nullptr, *lognu_glob = nullptr;
    double kappa = 1.0;
    double* cell_out = nullptr;   // [ncell][4]: E/eps part, <c,pi> (pixel units), X err, mass
    double* basic_out = nullptr;  // [nI][3]: sum m0, sum |x|^2 m0, sum <x,y> pi (pixel units), may be null
    double* totals = nullptr;     // [4] sums of cell_out columns
    double* pix_out = nullptr;    // [N*N][3]: per X pixel with mass, sum_y pi(x,y) and
                                  // sum_y (y_k + 1/2) pi(x,y) (pixel units), may be null
};

void launch_fill(double* p, size_t n, double v, hipStream_t st);
void launch_ymarg(int nI, const int32_t* box, const int64_t* base, const double* data, int N,
                  double* acc, const double* nu, double* out, hipStream_t st);
void launch_basic_mass(int nI, const int64_t* base, const double* data, const double* m,
                       double* per_cell, double* out, hipStream_t st);
size_t cell_eval_lds(int xside, int maxw1, int maxw2, size_t elem);
void launch_cell_eval(const EvalArgs& e, hipStream_t st);

}  // namespace dd
