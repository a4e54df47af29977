// Basic/composite cell-marginal kernels of one domain-decomposition iteration (declarations).
#pragma once

#include "common.hpp"

namespace dd {

// Static geometry of a composite partition on the device.
struct PartDev {
    int ncell = 0;
    int32_t* members = nullptr;  // [ncell][4] basic ids, -1 if absent; slot k = (dr, dc) = (k>>1, k&1)
    int32_t* xorig = nullptr;    // [ncell][2] X block origin pixel (may be -s for B)
};

// Current basic-cell Y-marginals nu_i in bounding-box form.
struct BoxSet {
    int32_t* box = nullptr;   // [nI][4] o1, o2, w1, w2
    int64_t* base = nullptr;  // [nI + 1]
    double* data = nullptr;   // packed row-major boxes
    size_t cap = 0;           // entries allocated in data
};

// Composite-cell work arrays of one iteration.
struct CompDev {
    int32_t* dims = nullptr;   // [ncell][2] W1, W2
    int32_t* orig = nullptr;   // [ncell][2] Y box origin pixel
    int32_t* shift = nullptr;  // [ncell][2] gauge E
    int32_t* gofs = nullptr;   // [ncell][2] G = pX - pY - E of this solve
    int64_t* size = nullptr;   // [ncell] W1*W2
    int64_t* base = nullptr;   // [ncell + 1]
    int32_t* info = nullptr;   // [8] totals read back by the host
};

void launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st);
void launch_comp_boxes(const PartDev& P, const BoxSet& S, int xside, CompDev& C, hipStream_t st);
void launch_scan(const int64_t* in, int64_t* out, int n, hipStream_t st);
void launch_comp_max(const CompDev& C, int ncell, hipStream_t st);
// dims[J] = (W1, W2) of every composite cell of P over the basic boxes `box`, as
// launch_comp_boxes computes them
void launch_comp_dims(const PartDev& P, const int32_t* box, int32_t* dims, hipStream_t st);
// flag[0] = 1 where a[k] != b[k] for some k < n (flag is not cleared)
void launch_dims_check(int n, const int32_t* a, const int32_t* b, int32_t* flag, hipStream_t st);

void launch_b2c(const PartDev& P, const BoxSet& S, const CompDev& C, double* nuJ, double* lognu,
                hipStream_t st);

void launch_warm_start(const PartDev& P, const CompDev& C, int xside, double* a, int32_t* g_stored,
                       double kappa_old, double kappa_new, int use_prev, hipStream_t st);

// c2b needs an upper bound maxw2 of the box widths (sizes its LDS tiles).
void launch_c2b(const PartDev& P, const CompDev& C, int xside, int s, int maxw2, const double* a,
                const double* logmu, const double* nuJ, double kappa, double h, double* tmp,
                double* py2, hipStream_t st);

void launch_balance(const PartDev& P, const CompDev& C, const double* m, double* tmp,
                    hipStream_t st);

void launch_trunc_boxes(const PartDev& P, const CompDev& C, const double* tmp, double trunc,
                        int nI, int32_t* nbox, int64_t* nsize, int32_t* flags, hipStream_t st);

void launch_compact(const PartDev& P, const CompDev& C, const double* tmp, double trunc,
                    const int32_t* nbox, const int64_t* nbase, const int32_t* flags,
                    double* ndata, hipStream_t st);

// Coarse-to-fine refinement (multiscale DD): fine basic-cell boxes and sizes from the coarse
// boxes (nf, nc basic cells per side), the refined values, and the interpolated potentials
// of one partition (fc: the coarse stitched potential on the Nc x Nc grid).
void launch_refine_boxes(int nf, int nc, const int32_t* cbox, int32_t* fbox, int64_t* fsize,
                         hipStream_t st);
void launch_refine_values(int nf, int nc, int Nc, const BoxSet& C, const double* cm,
                          const double* cnu, const int64_t* fbase, const double* fm,
                          const double* fnu, double* fdata, hipStream_t st);
void launch_refine_alpha(const PartDev& P, int xside, int Nc, const double* fc, double* a,
                         hipStream_t st);

// Sequential batches of one partition's composite cells: gathers of per-cell rows into a
// batch's own arrays (and back), and the staging of the truncated basic-cell boxes of each
// batch, copied to their place in the new state once every batch is done.
void launch_gather_rows(int n, const int32_t* idx, int width, const double* src, double* dst,
                        hipStream_t st);
void launch_scatter_rows(int n, const int32_t* idx, int width, const double* src, double* dst,
                         hipStream_t st);
void launch_gather_rows_i32(int n, const int32_t* idx, int width, const int32_t* src, int32_t* dst,
                            int back, hipStream_t st);
void launch_list_sizes(int n, const int32_t* list, const int64_t* nsize, int64_t* out,
                       hipStream_t st);
void launch_stage_base(int n, const int32_t* list, const int64_t* local, int64_t offset,
                       int64_t* stage_base, hipStream_t st);
void launch_unstage(int nI, const int64_t* nsize, const int64_t* stage_base, const double* staging,
                    const int64_t* nbase, double* ndata, hipStream_t st);

}  // namespace dd
