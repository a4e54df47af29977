// Learned warm start: conv-net inference and training kernels, cell features and the
// X-update that turns a predicted Y potential into the initial X potential.
//
// Inference (the learned start of the cell solves) is one kernel for the whole net: one
// workgroup per cell, every layer on the matrix cores (BF16 operands, FP32 accumulation),
// the activations kept in LDS between layers.  Training runs direct 3x3 convolutions on the
// vector ALUs: one workgroup of 256 lanes per sample, one output pixel per lane (every layer
// has a 16x16 output), FP32 accumulation.  The training forward kernel stages the sample's
// input in LDS and reads the weights (the BF16 values widened to FP32 after every update, laid
// out [ci][tap][co]) with wave-uniform loads from global memory, so they arrive through the
// scalar cache and feed the multiply-adds as scalar operands instead of occupying LDS
// bandwidth.  The backward kernels stage the weights in LDS.  Training keeps FP32 master
// weights with Adam and refreshes the BF16 copy after every step.  The weight gradients are
// reduced over the batch in a fixed order (per-workgroup partials, then one reduction), so
// training is deterministic.
#include "net.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace dd {

namespace {

constexpr int kT = 256;   // lanes per workgroup == output pixels per layer (16 x 16)
constexpr int kPix = 256;

ConvDesc make_layers_table(ConvDesc* L) {
    const int cin[kNetLayers] = {kNetCin, kNetCh, kNetCh, kNetCh, kNetCh};
    const int cout[kNetLayers] = {kNetCh, kNetCh, kNetCh, kNetCh, 4};
    const int hin[kNetLayers] = {kNetWin, 16, 16, 16, 16};
    const int stride[kNetLayers] = {2, 1, 1, 1, 1};
    const int dil[kNetLayers] = {1, 1, 2, 4, 1};
    int64_t off = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        ConvDesc& d = L[l];
        d.cin = cin[l];
        d.cout = cout[l];
        d.hin = d.win = hin[l];
        d.hout = d.wout = 16;
        d.stride = stride[l];
        d.dil = dil[l];
        d.pad = dil[l];
        d.relu = l < kNetLayers - 1;
        d.woff = off;
        off += (int64_t)d.cout * d.cin * 9;
        d.boff = off;
        off += d.cout;
    }
    return L[0];
}

struct Table {
    ConvDesc L[kNetLayers];
    int64_t n;
    Table() {
        make_layers_table(L);
        n = L[kNetLayers - 1].boff + L[kNetLayers - 1].cout;
    }
};
const Table& table() {
    static const Table t;
    return t;
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// y = act(conv(x) + b); for the last layer the 4 output channels are pixel-shuffled into
// the 32x32 output: y[2*oy + a][2*ox + c] = channel 2a + c.
template <int CO>
__global__ void __launch_bounds__(kT)
    conv_fwd_kernel(ConvDesc d, int n, const float* __restrict__ x,
                    const float* __restrict__ wfwd, const float* __restrict__ params,
                    float* __restrict__ y, int shuffle) {
    extern __shared__ float sm[];
    const int xin = d.cin * d.hin * d.win;
    float* xs = sm;
    const float* __restrict__ ws = wfwd + d.woff;  // [ci][tap][co]
    const int p = threadIdx.x;
    const int oy = p / d.wout, ox = p % d.wout;
    float bias[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) bias[co] = params[d.boff + co];
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        __syncthreads();
        for (int k = threadIdx.x; k < xin; k += blockDim.x) xs[k] = x[(int64_t)b * xin + k];
        __syncthreads();
        float acc[CO];
#pragma unroll
        for (int co = 0; co < CO; ++co) acc[co] = bias[co];
        for (int ci = 0; ci < d.cin; ++ci)
            for (int ky = 0; ky < 3; ++ky) {
                const int iy = oy * d.stride + ky * d.dil - d.pad;
                if (iy < 0 || iy >= d.hin) continue;
                for (int kx = 0; kx < 3; ++kx) {
                    const int ix = ox * d.stride + kx * d.dil - d.pad;
                    if (ix < 0 || ix >= d.win) continue;
                    const float v = xs[(ci * d.hin + iy) * d.win + ix];
                    const float* wr = ws + (ci * 9 + ky * 3 + kx) * CO;
#pragma unroll
                    for (int co = 0; co < CO; ++co) acc[co] = fmaf(v, wr[co], acc[co]);
                }
            }
        if (!shuffle) {
#pragma unroll
            for (int co = 0; co < CO; ++co)
                y[((int64_t)b * CO + co) * kPix + p] = d.relu ? fmaxf(acc[co], 0.f) : acc[co];
        } else {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    y[(int64_t)b * kNetWin * kNetWin + (2 * oy + a) * kNetWin + 2 * ox + c] =
                        acc[(2 * a + c) % CO];
        }
    }
}

// Operand layouts of v_mfma_f32_32x32x8 bf16 (checked on the device): A[m][k] in lane
// m + 32 (k / 4), element k % 4; B[k][n] in lane n + 32 (k / 4), element k % 4; D[m][n] in
// lane n + 32 ((m / 4) % 2), element 4 (m / 8) + m % 4.
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// The whole net's inference for one cell per workgroup, every layer on the matrix cores, the
// activations kept in LDS between layers (BF16, channel innermost).  Per layer the product
// D[p][co] = sum_k A[p][k] B[k][co] over the 256 output pixels (8 tiles of 32 rows; wave w
// takes tiles w and w + 4, two independent accumulators), k = tap * CIN + ci.  The B
// fragments come from a table in the instruction's operand order (one 8-byte load per lane
// and K step, see frag_kernel); the last layer's 4 output channels fill columns 0..3 of the
// tile (the rest are zero weights) and are pixel-shuffled into the 32x32 output.  The input of
// every layer is rounded to BF16; products are summed in FP32; bias and ReLU are applied in
// FP32 before the rounding.
constexpr int kAStr = 36;  // LDS stride of a pixel's 32 channels (BF16): 72 bytes, so the
                           // 8-byte reads of 32 consecutive pixels hit 64 distinct banks
constexpr int kFragSteps = (kNetCin * 9 + (kNetLayers - 1) * kNetCh * 9) / 8;

template <int CIN, int S, int DIL, int HIN, int ISTR, int COUT>
__device__ __forceinline__ void infer_layer(const uint16_t* __restrict__ in,
                                            const uint2* __restrict__ frag,
                                            const float* __restrict__ bias,
                                            uint16_t* __restrict__ out, float* __restrict__ y,
                                            int wv, int lane) {
    constexpr int kGroups = CIN / 8;  // K steps per tap
    const int half = lane >> 5, col = lane & 31;
    const int pa = wv * 32 + col, pb = pa + 128;
    const int oya = pa >> 4, oxa = pa & 15, oyb = pb >> 4, oxb = pb & 15;
    f32x16 acc0 = {}, acc1 = {};
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = (tap / 3 - 1) * DIL, dx = (tap % 3 - 1) * DIL;
        const int iya = oya * S + dy, ixa = oxa * S + dx;
        const int iyb = oyb * S + dy, ixb = oxb * S + dx;
        const bool ina = (unsigned)iya < (unsigned)HIN && (unsigned)ixa < (unsigned)HIN;
        const bool inb = (unsigned)iyb < (unsigned)HIN && (unsigned)ixb < (unsigned)HIN;
        const uint16_t* ra = in + (ina ? (iya * HIN + ixa) * ISTR : 0) + 4 * half;
        const uint16_t* rb = in + (inb ? (iyb * HIN + ixb) * ISTR : 0) + 4 * half;
        const uint2* ft = frag + tap * kGroups * 64 + lane;
        uint2 w[kGroups];
#pragma unroll
        for (int g = 0; g < kGroups; ++g) w[g] = ft[g * 64];
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
            bf4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
            if (ina) a0 = *reinterpret_cast<const bf4*>(ra + 8 * g);
            if (inb) a1 = *reinterpret_cast<const bf4*>(rb + 8 * g);
            bf4 bw;
            bw[0] = (short)(w[g].x & 0xffffu);
            bw[1] = (short)(w[g].x >> 16);
            bw[2] = (short)(w[g].y & 0xffffu);
            bw[3] = (short)(w[g].y >> 16);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a0, bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, bw, acc1, 0, 0, 0);
        }
    }
    // row m = 8 (j / 4) + 4 half + j % 4 of the tile: a per-lane base plus a constant offset
    if (COUT == kNetCh) {
        const float bv = bias[col];
        uint16_t* ob = out + (wv * 32 + 4 * half) * kAStr + col;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int mo = 8 * (j / 4) + j % 4;
            ob[mo * kAStr] = f2bf(fmaxf(acc0[j] + bv, 0.f));
            ob[(128 + mo) * kAStr] = f2bf(fmaxf(acc1[j] + bv, 0.f));
        }
    } else if (col < COUT) {
        // channel 2 a + c of output pixel p = (oy, ox) -> y[2 oy + a][2 ox + c]; with
        // p = 32 w + m: oy = 2 w + j / 8, ox = 8 ((j / 4) % 2) + 4 half + j % 4
        const float bv = bias[col];
        const int a = col >> 1, c = col & 1;
        float* yb = y + (4 * wv + a) * kNetWin + 8 * half + c;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int yo = 2 * (j / 8) * kNetWin + 2 * (8 * ((j / 4) % 2) + j % 4);
            yb[yo] = acc0[j] + bv;
            yb[16 * kNetWin + yo] = acc1[j] + bv;  // tile w + 4: oy + 8
        }
    }
}

struct InferBias {
    int64_t boff[kNetLayers];
};

__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(4)))
    net_infer_kernel(int n, const float* __restrict__ x, const uint2* __restrict__ frag,
                     const float* __restrict__ params, InferBias ib, float* __restrict__ y) {
    static_assert(kNetWin * kNetWin * kNetCin <= kPix * kAStr, "input fits the second buffer");
    __shared__ __align__(16) uint16_t buf0[kPix * kAStr];
    __shared__ __align__(16) uint16_t buf1[kPix * kAStr];  // also the 32x32x8 input
    constexpr int W2 = kNetWin * kNetWin;
    constexpr int o2 = kNetCin * 9 / 8, o3 = o2 + kNetCh * 9 / 8, o4 = o3 + kNetCh * 9 / 8,
                  o5 = o4 + kNetCh * 9 / 8;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        const float* xb = x + (int64_t)b * kNetCin * W2;
        __syncthreads();  // the previous cell's last layer has read buf1
        for (int pix = threadIdx.x; pix < W2; pix += kT) {
            uint4 w;
            w.x = f2bf(xb[0 * W2 + pix]) | ((uint32_t)f2bf(xb[1 * W2 + pix]) << 16);
            w.y = f2bf(xb[2 * W2 + pix]) | ((uint32_t)f2bf(xb[3 * W2 + pix]) << 16);
            w.z = f2bf(xb[4 * W2 + pix]) | ((uint32_t)f2bf(xb[5 * W2 + pix]) << 16);
            w.w = f2bf(xb[6 * W2 + pix]) | ((uint32_t)f2bf(xb[7 * W2 + pix]) << 16);
            *reinterpret_cast<uint4*>(&buf1[pix * kNetCin]) = w;
        }
        __syncthreads();
        infer_layer<kNetCin, 2, 1, kNetWin, kNetCin, kNetCh>(buf1, frag, params + ib.boff[0],
                                                             buf0, nullptr, wv, lane);
        __syncthreads();
        infer_layer<kNetCh, 1, 1, 16, kAStr, kNetCh>(buf0, frag + o2 * 64, params + ib.boff[1],
                                                     buf1, nullptr, wv, lane);
        __syncthreads();
        infer_layer<kNetCh, 1, 2, 16, kAStr, kNetCh>(buf1, frag + o3 * 64, params + ib.boff[2],
                                                     buf0, nullptr, wv, lane);
        __syncthreads();
        infer_layer<kNetCh, 1, 4, 16, kAStr, kNetCh>(buf0, frag + o4 * 64, params + ib.boff[3],
                                                     buf1, nullptr, wv, lane);
        __syncthreads();
        infer_layer<kNetCh, 1, 1, 16, kAStr, 4>(buf1, frag + o5 * 64, params + ib.boff[4],
                                                nullptr, y + (int64_t)b * W2, wv, lane);
    }
}

// The B-fragment table of net_infer_kernel: entry (step s of layer l, lane L) holds
// B[k][n] = W[n][ci][tap] for n = L % 32, k = 8 s + 4 (L / 32) + e, e = 0..3 (packed BF16,
// e in the low half first), k = tap * cin + ci; zero for n >= cout.
struct FragDesc {
    int64_t woff[kNetLayers];
    int cin[kNetLayers], cout[kNetLayers], soff[kNetLayers + 1];
};

__global__ void frag_kernel(FragDesc fd, const uint16_t* __restrict__ wbf,
                            uint2* __restrict__ frag) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= fd.soff[kNetLayers] * 64) return;
    const int gs = idx >> 6, lane = idx & 63;
    int l = 0;
    while (gs >= fd.soff[l + 1]) ++l;
    const int s = gs - fd.soff[l], nn = lane & 31, cin = fd.cin[l];
    uint32_t h[4];
    for (int e = 0; e < 4; ++e) {
        const int k = 8 * s + 4 * (lane >> 5) + e, tap = k / cin, ci = k % cin;
        h[e] = nn < fd.cout[l] ? wbf[fd.woff[l] + ((int64_t)nn * cin + ci) * 9 + tap] : 0u;
    }
    frag[idx] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

// Gradient with respect to the input of a stride-1 layer:
// dX[ci][iy][ix] = sum_co sum_tap dZ[co][iy - ky*dil + pad][ix - kx*dil + pad] W[co][ci][tap],
// dZ = dA * [A > 0] for a ReLU layer (A = the layer's output), dZ = dA otherwise.
template <int CI>
__global__ void __launch_bounds__(kT)
    conv_bwd_data_kernel(ConvDesc d, int n, const float* __restrict__ dA,
                         const float* __restrict__ A, const uint16_t* __restrict__ wbf,
                         float* __restrict__ dX) {
    extern __shared__ float sm[];
    float* zs = sm;                       // [cout][256]
    float* ws = sm + d.cout * kPix;       // [co][tap][ci]
    for (int k = threadIdx.x; k < d.cout * 9 * CI; k += blockDim.x) {
        const int ci = k % CI, t = (k / CI) % 9, co = k / (9 * CI);
        ws[k] = bf2f(wbf[d.woff + ((int64_t)co * CI + ci) * 9 + t]);
    }
    const int p = threadIdx.x;
    const int iy = p / d.win, ix = p % d.win;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        __syncthreads();
        for (int k = threadIdx.x; k < d.cout * kPix; k += blockDim.x) {
            const int64_t g = (int64_t)b * d.cout * kPix + k;
            zs[k] = (d.relu && !(A[g] > 0.f)) ? 0.f : dA[g];
        }
        __syncthreads();
        float acc[CI];
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) acc[ci] = 0.f;
        for (int co = 0; co < d.cout; ++co)
            for (int ky = 0; ky < 3; ++ky) {
                const int oy = iy - ky * d.dil + d.pad;
                if (oy < 0 || oy >= d.hout) continue;
                for (int kx = 0; kx < 3; ++kx) {
                    const int ox = ix - kx * d.dil + d.pad;
                    if (ox < 0 || ox >= d.wout) continue;
                    const float z = zs[co * kPix + oy * d.wout + ox];
                    const float* wr = ws + (co * 9 + ky * 3 + kx) * CI;
#pragma unroll
                    for (int ci = 0; ci < CI; ++ci) acc[ci] = fmaf(z, wr[ci], acc[ci]);
                }
            }
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) dX[((int64_t)b * CI + ci) * kPix + p] = acc[ci];
    }
}

// Per-workgroup partial weight and bias gradients of one layer over its share of the batch:
// dW[co][ci][tap] = sum_b sum_p dZ[co][p] X[ci][in(p, tap)], db[co] = sum_b sum_p dZ[co][p].
constexpr int kMaxE = (kNetCh * kNetCh * 9 + kNetCh + kT - 1) / kT;

__global__ void __launch_bounds__(kT)
    conv_bwd_w_kernel(ConvDesc d, int n, const float* __restrict__ X,
                      const float* __restrict__ dA, const float* __restrict__ A,
                      float* __restrict__ part) {
    extern __shared__ float sm[];
    const int xin = d.cin * d.hin * d.win;
    float* xs = sm;
    float* zs = sm + xin;
    const int ne = d.cout * d.cin * 9, np = ne + d.cout;
    float acc[kMaxE];
#pragma unroll
    for (int k = 0; k < kMaxE; ++k) acc[k] = 0.f;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        __syncthreads();
        for (int k = threadIdx.x; k < xin; k += blockDim.x) xs[k] = X[(int64_t)b * xin + k];
        for (int k = threadIdx.x; k < d.cout * kPix; k += blockDim.x) {
            const int64_t g = (int64_t)b * d.cout * kPix + k;
            zs[k] = (d.relu && !(A[g] > 0.f)) ? 0.f : dA[g];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxE; ++k) {
            const int e = threadIdx.x + k * kT;
            if (e < ne) {
                const int co = e / (d.cin * 9), r = e - co * d.cin * 9;
                const int ci = r / 9, t = r - ci * 9, ky = t / 3, kx = t - ky * 3;
                const float* z = zs + co * kPix;
                const float* xc = xs + ci * d.hin * d.win;
                float s = 0.f;
                for (int oy = 0; oy < d.hout; ++oy) {
                    const int iy = oy * d.stride + ky * d.dil - d.pad;
                    if (iy < 0 || iy >= d.hin) continue;
                    for (int ox = 0; ox < d.wout; ++ox) {
                        const int ix = ox * d.stride + kx * d.dil - d.pad;
                        if (ix < 0 || ix >= d.win) continue;
                        s = fmaf(z[oy * d.wout + ox], xc[iy * d.win + ix], s);
                    }
                }
                acc[k] += s;
            } else if (e < np) {
                const float* z = zs + (e - ne) * kPix;
                float s = 0.f;
                for (int q = 0; q < kPix; ++q) s += z[q];
                acc[k] += s;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kMaxE; ++k) {
        const int e = threadIdx.x + k * kT;
        if (e < np) part[(int64_t)blockIdx.x * np + e] = acc[k];
    }
}

// grad[e] = sum over workgroups of the partials, in workgroup order.
__global__ void reduce_part_kernel(int nblk, int np, const float* __restrict__ part,
                                   float* __restrict__ grad) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < np; e += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int k = 0; k < nblk; ++k) s += part[(int64_t)k * np + e];
        grad[e] = s;
    }
}

// Gauge-invariant weighted squared error of the predicted Y potential (a constant shift of
// g changes nothing in the cell problem):
//   loss_b = sum_w omega (y - t - c)^2,  c = sum_w omega (y - t) / sum_w omega,
// with the gradient 2 omega (y - t - c) / n written un-shuffled into the L5 gradient layout.
__global__ void __launch_bounds__(kT)
    loss_kernel(int n, const float* __restrict__ y, const float* __restrict__ tgt,
                const float* __restrict__ wgt, float* __restrict__ dA5, float* __restrict__ loss_b) {
    __shared__ double red[8];
    constexpr int W2 = kNetWin * kNetWin;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        const int64_t o = (int64_t)b * W2;
        double sw = 0.0, swr = 0.0;
        for (int k = threadIdx.x; k < W2; k += kT) {
            const double w = wgt[o + k];
            sw += w;
            swr += w * ((double)y[o + k] - tgt[o + k]);
        }
        sw = block_sum(sw, red);
        swr = block_sum(swr, red);
        const double c = sw > 0.0 ? swr / sw : 0.0;
        double l = 0.0;
        for (int k = threadIdx.x; k < W2; k += kT) {
            const double w = wgt[o + k];
            const double r = (double)y[o + k] - tgt[o + k] - c;
            l += w * r * r;
            const int Y = k / kNetWin, Xp = k % kNetWin;
            const int ch = 2 * (Y & 1) + (Xp & 1);
            dA5[((int64_t)b * 4 + ch) * kPix + (Y >> 1) * 16 + (Xp >> 1)] =
                (float)(2.0 * w * r / n);
        }
        l = block_sum(l, red);
        if (threadIdx.x == 0) loss_b[b] = (float)l;
    }
}

__global__ void adam_kernel(int64_t np, float* __restrict__ th, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ g,
                            uint16_t* __restrict__ wbf, float lr, float c1, float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < np;
         k += (int64_t)gridDim.x * blockDim.x) {
        const float gk = g[k];
        const float mk = b1 * m[k] + (1.f - b1) * gk;
        const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        const float t = th[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
        th[k] = t;
        wbf[k] = f2bf(t);
    }
}

__global__ void to_bf16_kernel(int64_t np, const float* __restrict__ th, uint16_t* __restrict__ wbf) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < np;
         k += (int64_t)gridDim.x * blockDim.x)
        wbf[k] = f2bf(th[k]);
}

// wfwd[ci][tap][co] = the BF16 weight W[co][ci][tap] as FP32, for one layer
__global__ void widen_kernel(ConvDesc d, const uint16_t* __restrict__ wbf,
                             float* __restrict__ wfwd) {
    const int nw = d.cout * d.cin * 9;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nw; k += gridDim.x * blockDim.x) {
        const int co = k % d.cout, t = (k / d.cout) % 9, ci = k / (9 * d.cout);
        wfwd[d.woff + k] = bf2f(wbf[d.woff + ((int64_t)co * d.cin + ci) * 9 + t]);
    }
}

__device__ __forceinline__ float feat(double lv, double lm) {
    return (float)(fmax(lv - lm + 16.0, 0.0) * 0.25);
}

// Separable pieces of the X <-> Y log-sum-exps of the learned start.  The cost splits into
// c(i1 - j1 + E1) + c(i2 - j2 + E2) with c(d) = d^2 / kappa, so an LSE over the X block (or
// over the box) is two LSEs over one axis each, the first into LDS.  Each row of the
// two-pass LSE takes its maximum in the precision of its inputs and sums the exponentials in
// FP32 relative to it.
constexpr int kRows = 64;  // box rows per pass of the Y-side kernels

// row LSE of fx[.][i2] (double, X block) against the column cost of one box row:
//   t = LSE_{i1} [fx(i1, i2) - c(i1 - j1 + E1)]
__device__ __forceinline__ double lse_xcol(const double* fx, int xside, int i2, int dj,
                                           float invk) {
    double mx = kNegD;
    for (int i1 = 0; i1 < xside; ++i1) {
        const double d = i1 + dj;
        mx = fmax(mx, fx[i1 * xside + i2] - d * d * invk);
    }
    float sm = 0.f;
    for (int i1 = 0; i1 < xside; ++i1) {
        const double d = i1 + dj;
        sm += __expf((float)(fx[i1 * xside + i2] - d * d * invk - mx));
    }
    return mx + log((double)sm);
}

// Features of cell J on the 32x32 window; window position w maps to box-local j = w - o + E
// and to X pixel i = w - o (o = (32 - xside)/2).  One workgroup per cell:
//   1. the cell's mass m_J, and f0 + log mu on the X block (LDS);
//   2. g0(w) = -LSE_i [f0(i) + log mu(i) - C(i, w)] on the support of nu_J in the window,
//      separably: LSE over i1 for every window row and X column into LDS, then over i2;
//   3. its mean under the weights nu_J / m_J, taken out;
//   4. f1(i) = -LSE_w [g0(w) + log nu_J(w) - C(i, w)] on the X block, separably: LSE over
//      w2 for every window row and X column into LDS, then over w1 (four lanes per X point,
//      a quarter of the rows each), and the channels.
__global__ void __launch_bounds__(kT)
    net_features_kernel(int ncell, int xside, const int32_t* __restrict__ dims,
                        const int32_t* __restrict__ shift, const int64_t* __restrict__ base,
                        const double* __restrict__ logmu, const double* __restrict__ lognu,
                        const double* __restrict__ a0, float invk, const double* __restrict__ b,
                        float* __restrict__ x, float* __restrict__ tgt, float* __restrict__ wgt) {
    __shared__ double red[8];
    __shared__ double fx[64];         // f0 + log mu on the X block (kNegD without mass)
    __shared__ float gv[kNetWin * kNetWin];  // g0 + log nu_J - lm (kNegF off the support)
    __shared__ float gs[kNetWin * kNetWin];  // g0 (raw)
    __shared__ float df[64];          // f1 - f0
    __shared__ double tw[kNetWin * 8];  // LSE over i1, per window row and X column
    __shared__ float sw1[kNetWin * 8];  // LSE over w2, per window row and X column
    constexpr int W2 = kNetWin * kNetWin;
    const int N2 = xside * xside, o = (kNetWin - xside) / 2;
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        double m = 0.0;
        for (int i = threadIdx.x; i < N2; i += kT) {
            const double l = logmu[(int64_t)J * N2 + i];
            const bool h = l > kZeroMassLog;
            if (h) m += exp(l);
            fx[i] = h ? a0[(int64_t)J * N2 + i] + l : kNegD;
        }
        m = block_sum(m, red);  // synchronises, so fx is complete
        const double lm = log(m);
        for (int k = threadIdx.x; k < kNetWin * xside; k += kT) {
            const int w1 = k / xside, i2 = k - w1 * xside;
            tw[k] = lse_xcol(fx, xside, i2, o - w1, invk);
        }
        __syncthreads();
        const int W1 = dims[2 * J], Wd2 = dims[2 * J + 1];
        const int E1 = shift[2 * J], E2 = shift[2 * J + 1];
        const int64_t bs = base[J];
        double sw = 0.0, swp = 0.0, swg = 0.0;
        for (int k = threadIdx.x; k < W2; k += kT) {
            const int w1 = k / kNetWin, w2 = k % kNetWin;
            const int j1 = w1 - o + E1, j2 = w2 - o + E2;
            const bool inbox = j1 >= 0 && j1 < W1 && j2 >= 0 && j2 < Wd2;
            const double ln = inbox ? lognu[bs + (int64_t)j1 * Wd2 + j2] : kNegD;
            const bool has = ln > kZeroMassLog;
            double g = 0.0;
            if (has) {
                const double* t = tw + w1 * xside;
                double mx = kNegD;
                for (int i2 = 0; i2 < xside; ++i2) {
                    const double d = o + i2 - w2;
                    mx = fmax(mx, t[i2] - d * d * invk);
                }
                float sm = 0.f;
                for (int i2 = 0; i2 < xside; ++i2) {
                    const double d = o + i2 - w2;
                    sm += __expf((float)(t[i2] - d * d * invk - mx));
                }
                g = -(mx + log((double)sm));
            }
            const double wt = has ? exp(ln - lm) : 0.0;
            gs[k] = (float)g;
            gv[k] = has ? (float)(g + ln - lm) : kNegF;
            sw += wt;
            swp += wt * g;
            if (tgt) {
                swg += has ? wt * b[bs + (int64_t)j1 * Wd2 + j2] : 0.0;
                wgt[(int64_t)J * W2 + k] = (float)wt;
            }
        }
        sw = block_sum(sw, red);
        swp = block_sum(swp, red);
        const double gpm = sw > 0.0 ? swp / sw : 0.0;
        // f1 on the X block: the LSE over w2 per window row and X column (block_sum above
        // synchronised, so gv is complete), then lane t takes X point t / 4 and the window
        // rows q = t % 4 (mod 4)
        for (int k = threadIdx.x; k < kNetWin * xside; k += kT) {
            const int w1 = k / xside, i2 = k - w1 * xside;
            const float* row = gv + w1 * kNetWin;
            float rm = kNegF;
            for (int w2 = 0; w2 < kNetWin; ++w2) {
                const float d = (float)(o + i2 - w2);
                rm = fmaxf(rm, row[w2] - d * d * invk);
            }
            float rs = 0.f;
            if (rm > 0.5f * kNegF)
                for (int w2 = 0; w2 < kNetWin; ++w2) {
                    const float d = (float)(o + i2 - w2);
                    rs += __expf(row[w2] - d * d * invk - rm);
                }
            sw1[k] = rm > 0.5f * kNegF ? rm + __logf(rs) : kNegF;
        }
        __syncthreads();
        {
            const int i = threadIdx.x >> 2, q = threadIdx.x & 3;
            const bool live = i < N2;
            const int i1 = live ? i / xside : 0, i2 = live ? i % xside : 0;
            float mx = kNegF, sm = 0.f;
            for (int w1 = q; w1 < kNetWin; w1 += 4) {
                const float s = sw1[w1 * xside + i2];
                if (!(s > 0.5f * kNegF)) continue;
                const float d = (float)(o + i1 - w1);
                const float x = s - d * d * invk;
                if (x > mx) {
                    sm = sm * __expf(mx - x) + 1.f;
                    mx = x;
                } else {
                    sm += __expf(x - mx);
                }
            }
            for (int k = 1; k < 4; k <<= 1) {
                const float mo = __shfl_xor(mx, k, 64), so = __shfl_xor(sm, k, 64);
                const float mn = fmaxf(mx, mo);
                sm = (mx > 0.5f * kNegF ? sm * __expf(mx - mn) : 0.f) +
                     (mo > 0.5f * kNegF ? so * __expf(mo - mn) : 0.f);
                mx = mn;
            }
            if (live && q == 0) {
                // f1 = -(lm + mx + log sm); the gauge of g0 cancels in f1 - f0
                const bool ok = fx[i] > 0.5 * kNegD && mx > 0.5f * kNegF && sm > 0.f;
                const double f0 = ok ? fx[i] - logmu[(int64_t)J * N2 + i] : 0.0;
                df[i] = ok ? (float)(-(lm + (double)mx + log((double)sm)) - f0) : 0.f;
            }
        }
        if (tgt) {
            swg = block_sum(swg, red);  // also makes df visible
        } else {
            __syncthreads();
        }
        const double gm = sw > 0.0 ? swg / sw : 0.0;
        float* xc = x + (int64_t)J * kNetCin * W2;
        for (int k = threadIdx.x; k < W2; k += kT) {
            const int w1 = k / kNetWin, w2 = k % kNetWin;
            const int j1 = w1 - o + E1, j2 = w2 - o + E2;
            const bool inbox = j1 >= 0 && j1 < W1 && j2 >= 0 && j2 < Wd2;
            const double ln = inbox ? lognu[bs + (int64_t)j1 * Wd2 + j2] : kNegD;
            const bool has = ln > kZeroMassLog;
            const int i1 = w1 - o, i2 = w2 - o;
            const bool inx = i1 >= 0 && i1 < xside && i2 >= 0 && i2 < xside;
            const double lmu = inx ? logmu[(int64_t)J * N2 + i1 * xside + i2] : kNegD;
            const bool hmu = lmu > kZeroMassLog;
            const float gc = has ? (float)((double)gs[k] - gpm) : 0.f;
            xc[0 * W2 + k] = has ? feat(ln, lm) : 0.f;
            xc[1 * W2 + k] = has ? 1.f : 0.f;
            xc[2 * W2 + k] = hmu ? feat(lmu, lm) : 0.f;
            xc[3 * W2 + k] = hmu ? 1.f : 0.f;
            xc[4 * W2 + k] = (w1 - 15.5f) * (1.f / 16.f);
            xc[5 * W2 + k] = (w2 - 15.5f) * (1.f / 16.f);
            xc[6 * W2 + k] = gc * 0.125f;
            xc[7 * W2 + k] = hmu ? df[i1 * xside + i2] : 0.f;
            if (tgt)
                tgt[(int64_t)J * W2 + k] =
                    has ? (float)(b[bs + (int64_t)j1 * Wd2 + j2] - gm) - gc : 0.f;
        }
        __syncthreads();
    }
}

// Y potential of the learned start on every box entry j (with nu_J > 0):
//   g(j) = -LSE_i [f0(i) + log mu(i) - C(i, j)] + [j in the window] (dg(w) - mean dg),
// with C(i, j) = ((i1 - j1 + E1)^2 + (i2 - j2 + E2)^2) / kappa and the mean of dg under the
// weights nu_J / m_J on the window (the net's output has no fixed constant; inside and outside
// the window the base is the same g0).  v = g + log nu_J is written packed like log nu_J
// (float; -inf where nu_J = 0).  Separable: t(j1, i2) = LSE_{i1} [...] for a pass of box
// rows into LDS, then g(j1, j2) = -LSE_{i2} [t(j1, i2) - c(i2 - j2 + E2)].
__global__ void __launch_bounds__(kT)
    net_gbox_kernel(int ncell, int xside, const int32_t* __restrict__ dims,
                    const int32_t* __restrict__ shift, const int64_t* __restrict__ base,
                    const double* __restrict__ logmu, const double* __restrict__ lognu,
                    const double* __restrict__ a0, const float* __restrict__ dg, float invk,
                    float* __restrict__ v) {
    __shared__ double red[8];
    __shared__ double fx[64];
    __shared__ double tr[kRows * 8];
    constexpr int W2 = kNetWin * kNetWin;
    const int N2 = xside * xside, o = (kNetWin - xside) / 2;
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        double m = 0.0;
        for (int i = threadIdx.x; i < N2; i += kT) {
            const double l = logmu[(int64_t)J * N2 + i];
            const bool h = l > kZeroMassLog;
            if (h) m += exp(l);
            fx[i] = h ? a0[(int64_t)J * N2 + i] + l : kNegD;
        }
        m = block_sum(m, red);
        const double lm = log(m);
        const int W1 = dims[2 * J], Wd2 = dims[2 * J + 1];
        const int E1 = shift[2 * J], E2 = shift[2 * J + 1];
        const int64_t bs = base[J];
        double sw = 0.0, swd = 0.0;
        for (int k = threadIdx.x; k < W2; k += kT) {
            const int j1 = k / kNetWin - o + E1, j2 = k % kNetWin - o + E2;
            const bool inbox = j1 >= 0 && j1 < W1 && j2 >= 0 && j2 < Wd2;
            const double ln = inbox ? lognu[bs + (int64_t)j1 * Wd2 + j2] : kNegD;
            if (ln > kZeroMassLog) {
                const double wt = exp(ln - lm);
                sw += wt;
                swd += wt * dg[(int64_t)J * W2 + k];
            }
        }
        sw = block_sum(sw, red);
        swd = block_sum(swd, red);
        const double dm = sw > 0.0 ? swd / sw : 0.0;
        for (int r0 = 0; r0 < W1; r0 += kRows) {
            const int nr = min(kRows, W1 - r0);
            for (int k = threadIdx.x; k < nr * xside; k += kT) {
                const int j1 = r0 + k / xside, i2 = k % xside;
                tr[k] = lse_xcol(fx, xside, i2, E1 - j1, invk);
            }
            __syncthreads();
            for (int e = threadIdx.x; e < nr * Wd2; e += kT) {
                const int r = e / Wd2, j1 = r0 + r, j2 = e - r * Wd2;
                const int64_t at = bs + (int64_t)j1 * Wd2 + j2;
                const double ln = lognu[at];
                float out = kNegF;
                if (ln > kZeroMassLog) {
                    const double* t = tr + r * xside;
                    double mx = kNegD;
                    for (int i2 = 0; i2 < xside; ++i2) {
                        const double d = i2 - j2 + E2;
                        mx = fmax(mx, t[i2] - d * d * invk);
                    }
                    float sm = 0.f;
                    for (int i2 = 0; i2 < xside; ++i2) {
                        const double d = i2 - j2 + E2;
                        sm += __expf((float)(t[i2] - d * d * invk - mx));
                    }
                    double g = -(mx + log((double)sm));
                    const int w1 = j1 + o - E1, w2 = j2 + o - E2;
                    if (w1 >= 0 && w1 < kNetWin && w2 >= 0 && w2 < kNetWin)
                        g += (double)dg[(int64_t)J * W2 + w1 * kNetWin + w2] - dm;
                    out = (float)(g + ln);
                }
                v[at] = out;
            }
            __syncthreads();
        }
    }
}

// The learned start: f(i) = -LSE_j [v(j) - C(i, j)] over the whole box (an exact X-update of
// the corrected Y potential).  Separable: s(j1, i2) = LSE_{j2} [v(j1, j2) - c(i2 - j2 + E2)]
// for a pass of box rows into LDS, then four lanes per X point fold the pass's rows
// (j1 = q mod 4) into an online maximum and sum, f = -LSE_{j1} [s(j1, i2) - c(i1 - j1 + E1)].
// Also records the gauge offsets of this solve (as the zero / previous-iterate start does).
__global__ void __launch_bounds__(kT)
    net_fbox_kernel(int ncell, int xside, const int32_t* __restrict__ dims,
                    const int32_t* __restrict__ shift, const int64_t* __restrict__ base,
                    const int32_t* __restrict__ gofs, const float* __restrict__ v, float invk,
                    double* __restrict__ a, int32_t* __restrict__ g_stored) {
    __shared__ float sr[kRows * 8];
    const int N2 = xside * xside;
    const int i = threadIdx.x >> 2, q = threadIdx.x & 3;
    const bool live = i < N2;
    const int i1 = live ? i / xside : 0, i2 = live ? i % xside : 0;
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int W1 = dims[2 * J], Wd2 = dims[2 * J + 1];
        const int E1 = shift[2 * J], E2 = shift[2 * J + 1];
        const int64_t bs = base[J];
        float mx = kNegF, sm = 0.f;
        for (int r0 = 0; r0 < W1; r0 += kRows) {
            const int nr = min(kRows, W1 - r0);
            for (int k = threadIdx.x; k < nr * xside; k += kT) {
                const int r = k / xside, c = k - r * xside;
                const float* row = v + bs + (int64_t)(r0 + r) * Wd2;
                float rm = kNegF;
                for (int j2 = 0; j2 < Wd2; ++j2) {
                    const float d = (float)(c - j2 + E2);
                    rm = fmaxf(rm, row[j2] - d * d * invk);
                }
                float rs = 0.f;
                if (rm > 0.5f * kNegF)
                    for (int j2 = 0; j2 < Wd2; ++j2) {
                        const float d = (float)(c - j2 + E2);
                        rs += __expf(row[j2] - d * d * invk - rm);
                    }
                sr[k] = rm > 0.5f * kNegF ? rm + __logf(rs) : kNegF;
            }
            __syncthreads();
            for (int r = q; r < nr; r += 4) {
                const float s = sr[r * xside + i2];
                if (!(s > 0.5f * kNegF)) continue;
                const float d = (float)(i1 - (r0 + r) + E1);
                const float x = s - d * d * invk;
                if (x > mx) {
                    sm = sm * __expf(mx - x) + 1.f;
                    mx = x;
                } else {
                    sm += __expf(x - mx);
                }
            }
            __syncthreads();
        }
        // combine the four partial (max, sum) pairs of an X point
        for (int k = 1; k < 4; k <<= 1) {
            const float mo = __shfl_xor(mx, k, 64), so = __shfl_xor(sm, k, 64);
            const float mn = fmaxf(mx, mo);
            sm = (mx > 0.5f * kNegF ? sm * __expf(mx - mn) : 0.f) +
                 (mo > 0.5f * kNegF ? so * __expf(mo - mn) : 0.f);
            mx = mn;
        }
        if (live && q == 0)
            a[(int64_t)J * N2 + i] = (mx > 0.5f * kNegF && sm > 0.f)
                                         ? -((double)mx + log((double)sm))
                                         : 0.0;
        if (threadIdx.x == 0) {
            g_stored[2 * J] = gofs[2 * J];
            g_stored[2 * J + 1] = gofs[2 * J + 1];
        }
    }
}

int grid_n(int n, int cap) { return std::max(1, std::min(n, cap)); }

template <typename K>
void lds_attr(K k, size_t bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t fwd_lds(const ConvDesc& d) { return sizeof(float) * (size_t)d.cin * d.hin * d.win; }

void launch_fwd(const ConvDesc& d, int n, const float* x, const float* wfwd,
                const float* params, float* y, int shuffle, hipStream_t st) {
    const size_t lds = fwd_lds(d);
    const int g = grid_n(n, 2048);
    if (d.cout == kNetCh) {
        lds_attr(conv_fwd_kernel<kNetCh>, lds);
        conv_fwd_kernel<kNetCh><<<g, kT, lds, st>>>(d, n, x, wfwd, params, y, shuffle);
    } else {
        lds_attr(conv_fwd_kernel<4>, lds);
        conv_fwd_kernel<4><<<g, kT, lds, st>>>(d, n, x, wfwd, params, y, shuffle);
    }
}

// refresh the forward kernels' FP32 weights and the inference kernel's fragment table from
// the BF16 copy
void widen_weights(dd_net* net, hipStream_t st) {
    const ConvDesc* L = table().L;
    FragDesc fd;
    fd.soff[0] = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        const int nw = L[l].cout * L[l].cin * 9;
        widen_kernel<<<(nw + 255) / 256, 256, 0, st>>>(L[l], net->wbf, net->wfwd);
        fd.woff[l] = L[l].woff;
        fd.cin[l] = L[l].cin;
        fd.cout[l] = L[l].cout;
        fd.soff[l + 1] = fd.soff[l] + L[l].cin * 9 / 8;
    }
    frag_kernel<<<(kFragSteps * 64 + 255) / 256, 256, 0, st>>>(fd, net->wbf, net->wfrag);
}

// the layer table is the one net_infer_kernel is written for
bool infer_shapes_match() {
    const ConvDesc* L = table().L;
    const int st[kNetLayers] = {2, 1, 1, 1, 1}, dl[kNetLayers] = {1, 1, 2, 4, 1};
    for (int l = 0; l < kNetLayers; ++l)
        if (L[l].stride != st[l] || L[l].dil != dl[l] || L[l].pad != dl[l] ||
            L[l].hout != 16 || L[l].wout != 16 || L[l].cout != (l + 1 < kNetLayers ? kNetCh : 4))
            return false;
    return L[0].cin == kNetCin && L[0].hin == kNetWin;
}

}  // namespace

const ConvDesc* net_layers() { return table().L; }
int64_t net_param_count() { return table().n; }

void launch_net_features(int ncell, int xside, const int32_t* dims, const int32_t* shift,
                         const int64_t* base, const double* logmu, const double* lognu,
                         const double* a0, double kappa, const double* b, float* x, float* tgt,
                         float* wgt, hipStream_t st) {
    if (ncell <= 0) return;
    net_features_kernel<<<grid_n(ncell, 4096), kT, 0, st>>>(ncell, xside, dims, shift, base,
                                                            logmu, lognu, a0,
                                                            (float)(1.0 / kappa), b, x, tgt,
                                                            wgt);
}

void launch_net_start(int ncell, int xside, const int32_t* dims, const int32_t* shift,
                      const int64_t* base, const double* logmu, const double* lognu,
                      const int32_t* gofs, const float* dg, double kappa, float* v, double* a,
                      int32_t* g_stored, hipStream_t st) {
    if (ncell <= 0) return;
    const float invk = (float)(1.0 / kappa);
    net_gbox_kernel<<<grid_n(ncell, 4096), kT, 0, st>>>(ncell, xside, dims, shift, base, logmu,
                                                        lognu, a, dg, invk, v);
    net_fbox_kernel<<<grid_n(ncell, 4096), kT, 0, st>>>(ncell, xside, dims, shift, base, gofs, v,
                                                        invk, a, g_stored);
}

}  // namespace dd

using dd::Status;

namespace {

Status net_reserve(dd_net* net, int n) {
    Status st;
    if (n <= net->cap_n) return st;
    const int cap = std::max(n, 256);
    if (net->act) (void)hipFree(net->act);
    if (net->ga) (void)hipFree(net->ga);
    if (net->out) (void)hipFree(net->out);
    if (net->loss_b) (void)hipFree(net->loss_b);
    net->act = net->ga = net->out = net->loss_b = nullptr;
    net->cap_n = 0;
    const size_t per = (size_t)dd::kNetCh * dd::kPix;
    DD_HIP(hipMalloc(&net->act, 4 * per * cap * sizeof(float)), st);
    DD_HIP(hipMalloc(&net->ga, 2 * per * cap * sizeof(float)), st);
    DD_HIP(hipMalloc(&net->out, (size_t)cap * dd::kNetWin * dd::kNetWin * sizeof(float)), st);
    DD_HIP(hipMalloc(&net->loss_b, cap * sizeof(float)), st);
    net->cap_n = cap;
    return st;
}

}  // namespace

Status net_infer(dd_net* net, int n, const float* x, float* y, hipStream_t st) {
    Status s;
    if (n == 0) return s;
    const dd::ConvDesc* L = dd::net_layers();
    if (!dd::infer_shapes_match()) {
        s.code = DD_EINVAL;
        s.msg = "net_infer: layer table differs from the inference kernel";
        return s;
    }
    dd::InferBias ib;
    for (int l = 0; l < dd::kNetLayers; ++l) ib.boff[l] = L[l].boff;
    dd::net_infer_kernel<<<dd::grid_n(n, 4096), dd::kT, 0, st>>>(n, x, net->wfrag, net->master,
                                                                 ib, y);
    DD_HIP(hipGetLastError(), s);
    return s;
}

Status net_forward(dd_net* net, int n, const float* x, float* y, hipStream_t st) {
    Status s = net_reserve(net, n);
    if (s.code || n == 0) return s;
    const dd::ConvDesc* L = dd::net_layers();
    const size_t per = (size_t)dd::kNetCh * dd::kPix * n;
    const float* in = x;
    for (int l = 0; l < dd::kNetLayers; ++l) {
        const bool last = l == dd::kNetLayers - 1;
        float* o = last ? y : net->act + l * per;
        dd::launch_fwd(L[l], n, in, net->wfwd, net->master, o, last ? 1 : 0, st);
        in = o;
    }
    DD_HIP(hipGetLastError(), s);
    return s;
}

namespace {

dd_status net_fail(dd_net* net, dd_status code, const std::string& msg) {
    if (net) net->err = msg;
    dd::set_global_error(msg);
    return code;
}

Status net_train(dd_net* net, int n, const float* x, const float* tgt, const float* wgt,
                 float lr, hipStream_t st, double* loss) {
    using namespace dd;
    Status s = net_reserve(net, n);
    if (s.code) return s;
    s = net_forward(net, n, x, net->out, st);
    if (s.code) return s;
    const ConvDesc* L = net_layers();
    const size_t per = (size_t)kNetCh * kPix * n;
    float* A[4] = {net->act, net->act + per, net->act + 2 * per, net->act + 3 * per};
    float* G[2] = {net->ga, net->ga + per};
    loss_kernel<<<grid_n(n, 2048), kT, 0, st>>>(n, net->out, tgt, wgt, G[0], net->loss_b);
    // weight-gradient partials: one slot per workgroup of the largest layer
    const int gw = grid_n(n, 512);
    const size_t need = (size_t)gw * (kNetCh * kNetCh * 9 + kNetCh);
    if (need > net->part_cap) {
        if (net->part) (void)hipFree(net->part);
        net->part = nullptr;
        DD_HIP(hipMalloc(&net->part, need * sizeof(float)), s);
        net->part_cap = need;
    }
    int cur = 0;  // G[cur] holds the gradient w.r.t. the output of layer l
    for (int l = kNetLayers - 1; l >= 0; --l) {
        const ConvDesc& d = L[l];
        const float* X = l == 0 ? x : A[l - 1];
        const float* Aout = l == kNetLayers - 1 ? nullptr : A[l];
        const size_t wl = sizeof(float) * ((size_t)d.cin * d.hin * d.win + (size_t)d.cout * kPix);
        lds_attr(conv_bwd_w_kernel, wl);
        conv_bwd_w_kernel<<<gw, kT, wl, st>>>(d, n, X, G[cur], Aout, net->part);
        const int np = d.cout * d.cin * 9 + d.cout;
        reduce_part_kernel<<<(np + 255) / 256, 256, 0, st>>>(gw, np, net->part,
                                                             net->grad + d.woff);
        if (l > 0) {
            const size_t dl = sizeof(float) * ((size_t)d.cout * kPix + (size_t)d.cout * 9 * d.cin);
            lds_attr(conv_bwd_data_kernel<kNetCh>, dl);
            conv_bwd_data_kernel<kNetCh><<<grid_n(n, 2048), kT, dl, st>>>(d, n, G[cur], Aout,
                                                                          net->wbf, G[1 - cur]);
            cur = 1 - cur;
        }
    }
    net->step += 1;
    const float c1 = 1.f - std::pow(0.9f, (float)net->step);
    const float c2 = 1.f - std::pow(0.999f, (float)net->step);
    const int64_t np = net_param_count();
    adam_kernel<<<(int)std::min<int64_t>((np + 255) / 256, 1024), 256, 0, st>>>(
        np, net->master, net->adam_m, net->adam_v, net->grad, net->wbf, lr, c1, c2);
    dd::widen_weights(net, st);
    DD_HIP(hipGetLastError(), s);
    if (loss) {
        std::vector<float> lb(n);
        DD_HIP(hipMemcpyAsync(lb.data(), net->loss_b, n * sizeof(float), hipMemcpyDeviceToHost, st),
               s);
        DD_HIP(hipStreamSynchronize(st), s);
        double t = 0.0;
        for (float v : lb) t += v;
        *loss = n > 0 ? t / n : 0.0;
    }
    return s;
}

}  // namespace

extern "C" int64_t dd_net_param_count(void) { return dd::net_param_count(); }

extern "C" dd_status dd_net_create(const float* params, dd_net** out) {
    if (!params || !out) return net_fail(nullptr, DD_EINVAL, "dd_net_create: null argument");
    *out = nullptr;
    const int64_t np = dd::net_param_count();
    for (int64_t k = 0; k < np; ++k)
        if (!std::isfinite(params[k]))
            return net_fail(nullptr, DD_EINVAL, "dd_net_create: non-finite parameter");
    dd_net* net = new dd_net();
    Status s;
    auto bail = [&](const Status& e) {
        dd_net_free(net);
        return net_fail(nullptr, e.code, e.msg);
    };
    if (hipMalloc(&net->master, np * sizeof(float)) != hipSuccess ||
        hipMalloc(&net->adam_m, np * sizeof(float)) != hipSuccess ||
        hipMalloc(&net->adam_v, np * sizeof(float)) != hipSuccess ||
        hipMalloc(&net->grad, np * sizeof(float)) != hipSuccess ||
        hipMalloc(&net->wbf, np * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&net->wfwd, np * sizeof(float)) != hipSuccess ||
        hipMalloc(&net->wfrag, (size_t)dd::kFragSteps * 64 * sizeof(uint2)) != hipSuccess) {
        s.code = DD_ENOMEM;
        s.msg = "dd_net_create: device allocation failed";
        return bail(s);
    }
    if (hipMemcpy(net->master, params, np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->adam_m, 0, np * sizeof(float)) != hipSuccess ||
        hipMemset(net->adam_v, 0, np * sizeof(float)) != hipSuccess) {
        s.code = DD_EDEVICE;
        s.msg = "dd_net_create: upload failed";
        return bail(s);
    }
    dd::to_bf16_kernel<<<(int)std::min<int64_t>((np + 255) / 256, 1024), 256>>>(np, net->master,
                                                                              net->wbf);
    dd::widen_weights(net, nullptr);
    if (hipDeviceSynchronize() != hipSuccess) {
        s.code = DD_EDEVICE;
        s.msg = "dd_net_create: kernel failed";
        return bail(s);
    }
    *out = net;
    return DD_OK;
}

extern "C" dd_status dd_net_params(dd_net* net, float* out) {
    if (!net || !out) return net_fail(net, DD_EINVAL, "dd_net_params: null argument");
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(out, net->master, dd::net_param_count() * sizeof(float),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return net_fail(net, DD_EDEVICE, "dd_net_params: copy failed");
    return DD_OK;
}

extern "C" dd_status dd_net_forward(dd_net* net, int32_t n, const float* x, float* y,
                                    void* stream) {
    if (!net || n < 0 || (n > 0 && (!x || !y)))
        return net_fail(net, DD_EINVAL, "dd_net_forward: bad argument");
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Status s = net_forward(net, n, x, y, st);
    if (s.code) return net_fail(net, s.code, s.msg);
    if (hipStreamSynchronize(st) != hipSuccess)
        return net_fail(net, DD_EDEVICE, "dd_net_forward: kernel failed");
    return DD_OK;
}

extern "C" dd_status dd_net_infer(dd_net* net, int32_t n, const float* x, float* y,
                                  void* stream) {
    if (!net || n < 0 || (n > 0 && (!x || !y)))
        return net_fail(net, DD_EINVAL, "dd_net_infer: bad argument");
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Status s = net_infer(net, n, x, y, st);
    if (s.code) return net_fail(net, s.code, s.msg);
    if (hipStreamSynchronize(st) != hipSuccess)
        return net_fail(net, DD_EDEVICE, "dd_net_infer: kernel failed");
    return DD_OK;
}

extern "C" dd_status dd_net_train_step(dd_net* net, int32_t n, const float* x, const float* tgt,
                                       const float* wgt, float lr, void* stream, double* loss) {
    if (!net || n < 1 || !x || !tgt || !wgt || !(lr > 0.f))
        return net_fail(net, DD_EINVAL, "dd_net_train_step: bad argument");
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Status s = net_train(net, n, x, tgt, wgt, lr, st, loss);
    if (s.code) return net_fail(net, s.code, s.msg);
    if (hipStreamSynchronize(st) != hipSuccess)
        return net_fail(net, DD_EDEVICE, "dd_net_train_step: kernel failed");
    return DD_OK;
}

extern "C" void dd_net_free(dd_net* net) {
    if (!net) return;
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)net->master, (void*)net->adam_m, (void*)net->adam_v, (void*)net->grad,
                    (void*)net->wbf, (void*)net->wfwd, (void*)net->wfrag, (void*)net->part, (void*)net->act, (void*)net->ga,
                    (void*)net->out, (void*)net->loss_b})
        if (p) (void)hipFree(p);
    delete net;
}

extern "C" const char* dd_net_strerror(const dd_net* net) {
    return net ? net->err.c_str() : dd::global_error();
}
