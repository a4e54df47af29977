// Learned warm start for the cell Sinkhorn: a small convolutional net (declarations).
//
// The net maps a 32x32 window of the cell -- centred on the X block in the box-local
// coordinates of the cell problem, so that window position w and X pixel i are at cost
// |o + i - w|^2 / kappa with o = (32 - xside)/2 -- to a correction of the Y potential on
// that window.  Its base is the previous-iterate start f0 (the X potential of the last
// visit of the partition): g0(w) = -LSE_i [f0(i) + log mu(i) - C(i, w)], made mean-free
// under the weights nu_J / m_J.  The X potential used to start Sinkhorn is one exact
// X-update, over the whole box, of the corrected potential g0 + dg (dg on the window part
// of the box, made mean-free the same way; g0 elsewhere):
//   f(i) = -LSE_j [g(j) + log nu_J(j) - C(i, j)],
// which is the slot for the initial alpha of the cell solve (App. A.1, Alg. "SinkhornGPU"
// input alpha_init).  With dg = 0 this is exactly one Sinkhorn iteration from f0.  The
// stopping rule of the solve is untouched, so the prediction only changes where the
// iteration starts.
//
// Layers (3x3 kernels, 32 channels, BF16 weights, FP32 accumulation, ReLU between):
//   L1  8 -> 32, stride 2      32x32 -> 16x16
//   L2 32 -> 32, dilation 1    16x16
//   L3 32 -> 32, dilation 2    16x16
//   L4 32 -> 32, dilation 4    16x16
//   L5 32 -> 4,  dilation 1    16x16, pixel-shuffled to the 32x32 output (no ReLU)
// Input channels: nu_J feature and support, mu feature and support, two window coordinates,
// g0 / 8 on the support of nu_J, and on the X block the change f1 - f0 of one Sinkhorn
// iteration from f0 (f1 = the X-update of g0), where mu > 0.
#pragma once

#include "common.hpp"

namespace dd {

constexpr int kNetWin = 32;          // window side
constexpr int kNetCin = 8;           // input channels
constexpr int kNetCh = 32;           // hidden channels
constexpr int kNetLayers = 5;

struct ConvDesc {
    int cin, cout, hin, win, hout, wout, stride, dil, pad, relu;
    int64_t woff, boff;  // offsets of the weights [cout][cin][3][3] and bias [cout]
};

// Layer table and parameter count.
const ConvDesc* net_layers();
int64_t net_param_count();

// Cell features of a composite batch (box-local window) from the start f0 (a0 [ncell]
// [xside^2]), and optionally the training target (the solved g minus g0, both mean-free
// under the weights) and the weights nu_J / m_J.
void launch_net_features(int ncell, int xside, const int32_t* dims, const int32_t* shift,
                         const int64_t* base, const double* logmu, const double* lognu,
                         const double* a0, double kappa, const double* b, float* x, float* tgt,
                         float* wgt, hipStream_t st);

// The learned start from the previous-iterate start f0 (in a, overwritten) and the net's
// correction dg on the window: g = g0 + (dg - its weighted mean) on the window part of the
// box, g0 elsewhere, written with log nu_J added to v (float scratch packed like log nu_J);
// then f(i) = -LSE_j [g(j) + log nu_J(j) - C(i, j)] over the whole box, into a.  Also
// records the gauge offsets of this solve (as the zero / previous-iterate start does).
void launch_net_start(int ncell, int xside, const int32_t* dims, const int32_t* shift,
                      const int64_t* base, const double* logmu, const double* lognu,
                      const int32_t* gofs, const float* dg, double kappa, float* v, double* a,
                      int32_t* g_stored, hipStream_t st);

}  // namespace dd

// The opaque net of the C ABI.
struct dd_net {
    float* master = nullptr;  // FP32 master parameters
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;
    uint16_t* wbf = nullptr;  // BF16 copy used by the kernels (weights; biases stay FP32)
    float* wfwd = nullptr;    // the BF16 weights widened to FP32, [ci][tap][co] per layer,
                              // for the forward kernels (read as wave-uniform loads)
    uint2* wfrag = nullptr;   // the BF16 weights in the matrix-core operand order of the
                              // inference kernel (B fragments per layer, K step and lane)
    float* part = nullptr;    // weight-gradient partials [blocks][layer params]
    size_t part_cap = 0;
    float* act = nullptr;     // activations of the last forward (training) [4][n][32][256]
    float* ga = nullptr;      // gradient buffers [2][n][32][256]
    float* out = nullptr;     // output of the last forward [n][1024]
    float* loss_b = nullptr;  // per-sample loss [n]
    int cap_n = 0;
    int64_t step = 0;
    std::string err;
};

// Forward pass on n samples (x [n][8][32][32] -> y [n][32][32]); keeps the activations.
dd::Status net_forward(dd_net* net, int n, const float* x, float* y, hipStream_t st);
// the same net with the 32-channel layers on the matrix cores (inputs rounded to BF16): the
// learned start of domdec_iterate
dd::Status net_infer(dd_net* net, int n, const float* x, float* y, hipStream_t st);
