// Register-blocked float32 cell Sinkhorn for 8 x 8 X blocks on gfx950.
//
// The iteration, the potentials (f = alpha/eps, g = beta/eps, reference measure
// mu_J (x) nu_J) and the precision split (float32 terms, float64 line offsets, potentials,
// errors and masses) are those of the general kernels: the cell problem of Alg.
// "DomDecIter" in the log domain, with the separable cost of App. A.1 evaluated as two 1D
// log-sum-exp passes per half-iteration, each as a stabilised kernel product (input shifted
// by its line maximum, the cost split at the input nearest to each output, so that the
// per-term work is one multiply-add against a kernel table built once per cell).
//
// What is specific to the common block side 2s = 8 is the mapping to the hardware:
//   * the 64 lanes of a wave form an 8 x 8 grid (r, c).  The lane (r, c) of the first wave
//     owns X point (r, c) (f, log mu, mu in registers); in the Y box it owns the rows
//     j1 = r + 8 (wave + waves * t) and the columns j2 = c + 8 u (+ 32 per column block);
//   * the Y-update of a box row is fused with the first pass of the X-update of that row:
//     g, g + log nu_J, the row maximum and exp(g + log nu_J - max) never leave registers.
//     The 8-wide kernel rows (Y-update over i1, X-update over i2) are vectors read once per
//     row or column as 128-bit LDS broadcasts, so a box entry costs 16 multiply-adds, one
//     log and one exp, and no LDS traffic of its own;
//   * row maxima and the reductions of the X-update over the 8 lanes of a row are DPP lane
//     permutations; the second X pass reduces across the rows through shuffles;
//   * a cell's box is transposed on load when it is wider than tall, so the long side is the
//     one split across lanes and waves;
//   * a box whose long side is at most 32 is solved by one wave (four cells per workgroup,
//     log nu_J in registers); larger boxes by a workgroup of four waves (log nu_J read from
//     global memory, L2-resident while the cell runs);
//   * an underflowed kernel-product sum (every input near the output negligible against the
//     line maximum) is recomputed for that output by an exact log-sum-exp in float64.
// The batch rule runs in rounds: one launch per cell class runs K iterations of each of its
// cells, and the last workgroup of the round (ticket shared by the classes) reduces the
// per-cell errors in fixed cell order, tests the rule, raises the device stop flag or sets K
// of the next round from the error's decay.  Rounds are plain launches queued a few at a time
// between host reads of the stop flag; a round queued after the stop exits at once.
#include "fastcell.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

namespace dd {
namespace {

constexpr int kA = 8;  // X block side
constexpr int kBlock = 256;
// largest move of f (in units of kT) tolerated between rebuilds of the absorbed profiles
constexpr double kProfileDrift = 32.0;
// Smallest kernel-product sum trusted without the exact fallback.  Every factor is at most 1,
// so the terms lost to float underflow (each below 1.2e-38, at most 512 of them) stay below
// 1e-9 of any sum above the floor.
constexpr float kFloorF = 1e-28f;
constexpr int kSolve = 0, kBatch = 1, kFinal = 2;

template <typename T>
using lds_p = __attribute__((address_space(3))) T*;
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------
// Lane permutations (all 64 lanes active).
// ---------------------------------------------------------------------------------------
constexpr int kDppXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppMirror8 = 0x141;  // row_half_mirror: lane i <-> 7 - i within 8
constexpr int kDppRor8 = 0x128;     // row_ror:8 within 16 lanes: lane i <-> i ^ 8

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// The value of lane ^ 32 or lane ^ 16 by gfx950's lane swaps (VALU, no LDS round trip):
// permlane32_swap(v, v) hands every lane l the pair (v[l & 31], v[(l & 31) + 32]),
// permlane16_swap(v, v) the pair (v[l & ~16], v[l | 16]).
template <int B>
__device__ __forceinline__ unsigned xoru(unsigned v) {
    static_assert(B == 16 || B == 32, "lane swaps of 16 or 32");
    const bool upper = (threadIdx.x & B) != 0;
    if constexpr (B == 32) {
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return upper ? p[0] : p[1];
    } else {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return upper ? p[0] : p[1];
    }
}
template <int B>
__device__ __forceinline__ double xord(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = xoru<B>((unsigned)u), hi = xoru<B>((unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// maximum over the aligned group of 8 lanes (same r); every lane gets the same result
__device__ __forceinline__ double max8(double v) {
    v = fmax(v, dppd<kDppXor1>(v));
    v = fmax(v, dppd<kDppXor2>(v));
    return fmax(v, dppd<kDppMirror8>(v));
}
// maximum over the 8 lanes with the same c (lane bits 3..5)
__device__ __forceinline__ double maxr(double v) {
    v = fmax(v, dppd<kDppRor8>(v));
    v = fmax(v, xord<16>(v));
    return fmax(v, xord<32>(v));
}
// sum / maximum over the wave (every lane gets the result): quads, then pairs of quads
// (lane i <-> 7 - i), of 8, of 16 and of 32 lanes
__device__ __forceinline__ double wsum(double v) {
    v += dppd<kDppXor1>(v);
    v += dppd<kDppXor2>(v);
    v += dppd<kDppMirror8>(v);
    v += dppd<kDppRor8>(v);
    v += xord<16>(v);
    return v + xord<32>(v);
}
__device__ __forceinline__ double wmax(double v) {
    v = fmax(v, dppd<kDppXor1>(v));
    v = fmax(v, dppd<kDppXor2>(v));
    v = fmax(v, dppd<kDppMirror8>(v));
    v = fmax(v, dppd<kDppRor8>(v));
    v = fmax(v, xord<16>(v));
    return fmax(v, xord<32>(v));
}
// Reduce-scatter of a[0..7] over the 8 lanes with the same r: lane c gets the sum over those
// lanes of a[c] (recursive halving with partners 7 - c, c ^ 2, c ^ 1).
__device__ __forceinline__ float rs8(const float (&a)[8], int c) {
    const bool b2 = (c & 4) != 0, b1 = (c & 2) != 0, b0 = (c & 1) != 0;
    float h[4], e[2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        h[q] = (b2 ? a[4 + q] : a[q]) + dppf<kDppMirror8>(b2 ? a[q] : a[4 + q]);
#pragma unroll
    for (int q = 0; q < 2; ++q)
        e[q] = (b1 ? h[2 + q] : h[q]) + dppf<kDppXor2>(b1 ? h[q] : h[2 + q]);
    return (b0 ? e[1] : e[0]) + dppf<kDppXor1>(b0 ? e[0] : e[1]);
}
// The same over the 8 lanes with the same c (float64): lane (r, c) gets the sum of a[r]
// (partners lane ^ 32, ^ 16, ^ 8).
__device__ __forceinline__ double rsrd(const double (&a)[8], int r) {
    const bool b2 = (r & 4) != 0, b1 = (r & 2) != 0, b0 = (r & 1) != 0;
    double h[4], e[2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        h[q] = (b2 ? a[4 + q] : a[q]) + xord<32>(b2 ? a[q] : a[4 + q]);
#pragma unroll
    for (int q = 0; q < 2; ++q)
        e[q] = (b1 ? h[2 + q] : h[q]) + xord<16>(b1 ? h[q] : h[2 + q]);
    return (b0 ? e[1] : e[0]) + dppd<kDppRor8>(b0 ? e[0] : e[1]);
}

template <int NW>
struct Team {
    __device__ static int wave() {
        return NW == 1 ? 0 : (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    }
    // a wave alone works from LDS only and its LDS operations complete in order: keeping the
    // compiler from moving memory operations across this point is all it needs
    __device__ static void sync() {
        if constexpr (NW == 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    }
};

__device__ __forceinline__ double uni(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// ---------------------------------------------------------------------------------------
// LDS slice of one cell (kernel frame: W1 >= W2 after the optional transposition).
//   fixed part: U1 [64] f64 = exp(f + log mu - phi(i2) - ry(i1)), ry [8] f64 (row maxima of
//               f + log mu - phi), red [8] f64 (shared scalars), phi [8], psi [8] f64
//               (profiles absorbed into the Y-update kernels), and for a workgroup team the
//               per-wave partials xd [NW][8] f64, xs [2][NW][64] f64;
//   row records (box row j1, 176 B): KY2 [8] f32 (Y-update pass over i1, inputs i1),
//               KX2 [8] f64 (X-update pass over j1, outputs i1), R [8] f64 (first X pass,
//               minus dx1(j1)^2 / kappa), sY2 f64 (shift of output j1 of the Y-update's
//               second pass), unc [8] u8 (R is only an upper bound, see below);
//   column records (box column j2, 224 B): KY1 [8] f64 (Y-update pass over i2, inputs i2),
//               KX1 [8] f32 (X-update pass over j2, outputs i2), U2 [8] f32 = exp(V - psi
//               - My) over i1, My f64, sY1 f64 (shift of output j2 of the Y-update's first
//               pass), V [8] f64 = LSE_i2 [f + log mu - cost] (for the exact fallback),
//               Myx f64 = My + dx2(j2)^2 / kappa.
// Kernel entries.  The potential f varies across the block by far more than float exp covers
// at small kappa, and g grows quadratically away from it, so each pass absorbs the bulk of
// its input's variation into its kernel (the stabilised-kernel idea, here once per launch):
//   * Y-update, pass over i2: the column profile phi(i2) = max_i1 (f + log mu) taken at the
//     cell's load, KY1[j2][i2] = exp(phi(i2) - (i2 - j2 + E2)^2 / kappa - tau1(j2)) with
//     tau1(j2) the maximum over i2 of the exponent, sY1 = -tau1;
//   * Y-update, pass over i1: the row profile psi(i1) = max_i2 (f + log mu - phi) at load,
//     KY2[j1][i1] = exp(psi(i1) - (i1 - j1 + E1)^2 / kappa - tau2(j1)), sY2 = -tau2, and the
//     pass's input is V - psi;
//   * X-update passes (box inputs, X outputs): each input is normalised at the X output
//     nearest to it, dn = dx(j) the distance of box line j to the block's range, whose
//     square / kappa is taken out of that input instead (the quadratic growth of g).
// Any profile gives the same sums.  The two passes over the X block's 8-wide lines (the first
// Y pass, the second X pass) run in float64 with a float exp split into an exponent and a
// fraction, so they cannot underflow; the two float32 passes over box lines fall back to
// exact sums when one underflows (rare with the profiles above), and the first X pass's
// underflowed outputs are first replaced by an upper bound that is kept whenever it cannot
// move the second pass's sums.
// ---------------------------------------------------------------------------------------
constexpr int kRowB = 176, kColB = 224;  // 16-byte multiples
constexpr int kOffU1 = 0, kOffRy = 512, kOffRed = 576, kOffPhi = 640, kOffPsi = 704,
              kOffXd = 768;
// row record fields
constexpr int kRKY2 = 0, kRKX2 = 32, kRR = 96, kRSY2 = 160, kRUnc = 168;
// column record fields
constexpr int kCKY1 = 0, kCKX1 = 64, kCU2 = 96, kCMy = 128, kCSY1 = 136, kCV = 144,
              kCMyx = 208;
// exp(x) for x <= 0 by the hardware's base-2 exponential (underflows to 0 below about -87,
// which no kept term reaches), and ln of a positive normal float to about 1e-7 absolute: the
// base-2 log of the mantissa in [0.5, 1) plus the exponent, combined in float64
__device__ __forceinline__ float fexp(float x) {
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}
__device__ __forceinline__ double klog(float x) {
    const float m = __builtin_amdgcn_frexp_mantf(x);
    const int e = __builtin_amdgcn_frexp_expf(x);
    return ((double)__builtin_amdgcn_logf(m) + (double)e) * 0.6931471805599453;
}
// exp of a float64 argument to float accuracy over the whole float64 range: 2^(x log2 e)
// split into an integer power and a fraction
__device__ __forceinline__ double exp_wide(double x) {
    const double t = x * 1.4426950408889634;
    const double k = fmin(fmax(floor(t), -2000.0), 1000.0);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(t - k)), (int)k);
}
// log of a positive float64 to float accuracy: mantissa and exponent separately
__device__ __forceinline__ double log_wide(double x) {
    int e;
    const double m = frexp(x, &e);
    return ((double)__builtin_amdgcn_logf((float)m) + (double)e) * 0.6931471805599453;
}

__host__ __device__ constexpr int fixed_bytes(int NW) {
    return NW > 1 ? kOffXd + 64 * NW + 1024 * NW : kOffXd;
}

__host__ __device__ inline size_t slice_bytes(int NW, int W1m, int W2m) {
    return (size_t)fixed_bytes(NW) + (size_t)kRowB * W1m + (size_t)kColB * W2m;
}

__device__ __forceinline__ void ld8(lds_p<float> p, float (&v)[8]) {
    const v4f a = *(lds_p<v4f>)p;
    const v4f b = *(lds_p<v4f>)(p + 4);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = b.x;
    v[5] = b.y;
    v[6] = b.z;
    v[7] = b.w;
}

// signed distance of box line j to the block's range [e, e + 8) along one axis
__device__ __forceinline__ int dx_block(int j, int e) { return j - min(max(j, e), e + kA - 1); }

typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void ld8d(lds_p<double> p, double (&v)[8]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const v2d a = *(lds_p<v2d>)(p + 2 * q);
        v[2 * q] = a.x;
        v[2 * q + 1] = a.y;
    }
}

struct FastArgs {
    SkBatch p;
    const int32_t* cells;  // the cells of this launch, most work first
    const int4* recs;      // per queue slot: {cell, W1, W2, -}, {shift 1, shift 2, base lo, hi}
    int n;
    int W1m, W2m;          // slice bounds (kernel frame)
    int mode;
    int limit, fixed, stall;  // kSolve
    int chunk, max_iter;      // kBatch: least iterations between two tests, iteration cap
    double tol;
    int nblocks;              // kBatch: workgroups of all the launches of one round
    int* ctrl;
    int qidx;                 // this launch's queue word
    int32_t* iters;
    double* err;
    double* mass;
    double* dtot;
    double* f_keep;           // kBatch / kFinal: f at the start of each cell's last iteration
};

// Exact log-sum-exp fallbacks, reached only when a kernel-product sum underflows (an output
// whose nearest inputs with mass are all negligible against the line maximum).
// LSE_k [in(k) - (k - q + e)^2 / kappa] over the 8 inputs of an X line.
template <typename F>
__device__ __forceinline__ double exact8(F in, int q, int e, double invk) {
    double m = -1e300;
#pragma unroll
    for (int k = 0; k < kA; ++k) {
        const double d = k - q + e;
        m = fmax(m, in(k) - d * d * invk);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kA; ++k) {
        const double d = k - q + e;
        s += fexp((float)(in(k) - d * d * invk - m));
    }
    return m + klog(s);
}
// Y-update, second pass, entry (j1, j2): LSE_i1 [V(i1, j2) - (i1 - j1 + E1)^2 / kappa].
__device__ __forceinline__ double exact_y2(lds_p<char> col, int j1, int E1, double invk) {
    const lds_p<double> V = (lds_p<double>)(col + kCV);
    return exact8([&](int k) { return V[k]; }, j1, E1, invk);
}
__device__ __noinline__ double exact_y2_call(lds_p<char> col, int j1, int E1, double invk) {
    return exact_y2(col, j1, E1, invk);
}
// X-update, second pass, output (i1, i2): LSE_j1 [R(j1, i2) - (j1 - i1 - E1)^2 / kappa], R
// the first pass's result (stored minus dx1(j1)^2 / kappa).
__device__ __noinline__ double exact_x2(lds_p<char> rows, int i1, int i2, int W1, int E1,
                                        double invk) {
    // (reached only when every term of the float64 pass is zero)
    auto term = [&](int j1) {
        const double d = j1 - i1 - E1, e = dx_block(j1, E1);
        return *((lds_p<double>)(rows + j1 * kRowB + kRR) + i2) + (e * e - d * d) * invk;
    };
    double m = -1e300;
    for (int j1 = 0; j1 < W1; ++j1) m = fmax(m, term(j1));
    float s = 0.f;
    for (int j1 = 0; j1 < W1; ++j1) s += fexp((float)(term(j1) - m));
    return m + klog(s);
}

// One cell: load, iterate, store.  NW waves per cell, RPL box rows per lane at most, RC rows
// per lane processed together; LNREG: log nu_J held in registers (NW == 1, box within
// 32 x 32).
template <int NW, int RPL, bool LNREG, int RC>
__device__ __forceinline__ void run_cell(const FastArgs& g, int q, lds_p<char> sb, int K) {
    using Tm = Team<NW>;
    const SkBatch& p = g.p;
    const int lane = threadIdx.x & 63, w = Tm::wave(), tl = w * 64 + lane;
    const int r = lane >> 3, c = lane & 7;
    // the slot's packed record: one load for everything the cell's other loads depend on
    const int4 ra = g.recs[2 * q], rb = g.recs[2 * q + 1];
    const int cell = ra.x;
    const int W1o = ra.y, W2o = ra.z;
    const bool T = W2o > W1o;
    const int W1 = T ? W2o : W1o, W2 = T ? W1o : W2o;
    if (W1o < 1 || W2o < 1 || W1o > p.max_w1 || W2o > p.max_w2 || W1 > g.W1m || W2 > g.W2m) {
        if (tl == 0) {
            atomicOr(&g.ctrl[3], 1);
            g.err[cell] = 0.0;
            g.mass[cell] = 0.0;
            if (g.mode != kBatch) g.iters[cell] = 0;
        }
        return;
    }
    const int E1 = T ? rb.y : rb.x, E2 = T ? rb.x : rb.y;
    const int64_t bse = (int64_t)(((uint64_t)(uint32_t)rb.w << 32) | (uint32_t)rb.z);
    const int s1 = T ? 1 : W2o, s2 = T ? W2o : 1;  // kernel-frame (j1, j2) -> packed offset
    const int xo = T ? c * kA + r : r * kA + c;    // this lane's X point (i1 = r, i2 = c)
    const double invk = 1.0 / p.kappa;
    const float invkf = (float)invk;
    const lds_p<double> U1 = (lds_p<double>)(sb + kOffU1);
    const lds_p<double> ry = (lds_p<double>)(sb + kOffRy);
    const lds_p<double> red = (lds_p<double>)(sb + kOffRed);
    const lds_p<int> ired = (lds_p<int>)(sb + kOffRed + 32);  // [8] shared ints
    const lds_p<double> phi = (lds_p<double>)(sb + kOffPhi);
    const lds_p<double> psi = (lds_p<double>)(sb + kOffPsi);
    const lds_p<double> xd = (lds_p<double>)(sb + kOffXd);
    const lds_p<double> xs = (lds_p<double>)(sb + kOffXd + 64 * NW);  // [2][NW][64]
    const lds_p<char> rows = sb + fixed_bytes(NW);
    const lds_p<char> cols = rows + kRowB * g.W1m;
    auto rowp = [&](int j) { return rows + j * kRowB; };
    auto colp = [&](int j) { return cols + j * kColB; };
    auto KY2 = [&](int j) { return (lds_p<float>)(rowp(j) + kRKY2); };
    auto KX2 = [&](int j) { return (lds_p<double>)(rowp(j) + kRKX2); };
    auto UNC = [&](int j) { return (lds_p<unsigned char>)(rowp(j) + kRUnc); };
    auto Rr = [&](int j) { return (lds_p<double>)(rowp(j) + kRR); };
    auto SY2 = [&](int j) { return (lds_p<double>)(rowp(j) + kRSY2); };
    auto KY1 = [&](int j) { return (lds_p<double>)(colp(j) + kCKY1); };
    auto KX1 = [&](int j) { return (lds_p<float>)(colp(j) + kCKX1); };
    auto U2 = [&](int j) { return (lds_p<float>)(colp(j) + kCU2); };
    auto My = [&](int j) { return (lds_p<double>)(colp(j) + kCMy); };
    auto SY1 = [&](int j) { return (lds_p<double>)(colp(j) + kCSY1); };
    auto Vc = [&](int j) { return (lds_p<double>)(colp(j) + kCV); };
    auto Myx = [&](int j) { return (lds_p<double>)(colp(j) + kCMyx); };

    // ---- load: X state (first wave), log nu_J, which X rows and columns carry mass --------
    // (every load of the visit is issued before the first wait: they all depend on the slot's
    // record only)
    const double* fsrc = g.mode == kFinal ? g.f_keep : p.a;
    double f = 0.0, lm = kNegD, mu = 0.0;
    if (w == 0) {
        f = fsrc[(int64_t)cell * 64 + xo];
        lm = p.logmu[(int64_t)cell * 64 + xo];
    }
    float lnr[LNREG ? RPL : 1][4];
    double lnref = 0.0;
    if constexpr (LNREG) {
        double v[RPL][4];
#pragma unroll
        for (int t = 0; t < RPL; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j1 = r + 8 * t, j2 = c + 8 * u;
                v[t][u] = (j1 < W1 && j2 < W2)
                              ? p.lognu[bse + (int64_t)j1 * s1 + (int64_t)j2 * s2]
                              : kNegD;
            }
        double m = kNegD;
#pragma unroll
        for (int t = 0; t < RPL; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (v[t][u] > kZeroMassLog) m = fmax(m, v[t][u]);
        lnref = uni(wmax(m));
        if (!(lnref > kZeroMassLog)) lnref = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                lnr[t][u] = v[t][u] > kZeroMassLog ? (float)(v[t][u] - lnref) : kNegF;
    }
    if (w == 0) mu = lm > kZeroMassLog ? exp(lm) : 0.0;
    if (tl == 0) ired[1] = 0;  // underflow flag of the first X pass
    Tm::sync();
    // X rows / columns with mass (kernel frame), and the cell's mass
    unsigned xrow = 0, xcol = 0;
    double mass_all = 0.0;
    if (w == 0) {
        const unsigned long long bm = __ballot(mu > 0.0);
        for (int k = 0; k < kA; ++k) {
            if ((bm >> (8 * k)) & 0xFFull) xrow |= 1u << k;
            if ((bm >> k) & 0x0101010101010101ull) xcol |= 1u << k;
        }
        mass_all = wsum(mu);
        if constexpr (NW > 1) {
            if (tl == 0) {
                ired[2] = (int)xrow;
                ired[3] = (int)xcol;
                red[1] = mass_all;
            }
        }
    }
    Tm::sync();
    if constexpr (NW > 1) {
        xrow = (unsigned)ired[2];
        xcol = (unsigned)ired[3];
        mass_all = red[1];
    }
    xrow = __builtin_amdgcn_readfirstlane(xrow);
    xcol = __builtin_amdgcn_readfirstlane(xcol);
    mass_all = uni(mass_all);
    // X-update kernel tables (fixed for the cell)
    for (int o = tl; o < W2 * 8; o += 64 * NW) {
        const int j2 = o >> 3, k = o & 7;
        const int dx = j2 - k - E2, dnx = dx_block(j2, E2);
        KX1(j2)[k] = fexp(-(float)(dx * dx - dnx * dnx) * invkf);
    }
    for (int o = tl; o < W1 * 8; o += 64 * NW) {
        const int j1 = o >> 3, k = o & 7;
        const int dx = j1 - k - E1, dnx = dx_block(j1, E1);
        KX2(j1)[k] = exp_wide(-(double)(dx * dx - dnx * dnx) * invk);
    }
    // Y-update kernel tables with the profiles of f + log mu absorbed (from f = fc)
    auto build_y = [&](double fc) {
        if (w == 0) {
            const bool has = mu > 0.0;
            const double w0 = has ? fc + lm : kNegD;
            const double ph = maxr(w0);  // over the rows, per column c
            const double ps = max8(has ? w0 - ph : kNegD);  // over the columns, per row r
            if (r == 0) phi[c] = ph;
            if (c == 0) psi[r] = ps;
        }
        Tm::sync();
        for (int o = tl; o < W2 * 8; o += 64 * NW) {
            const int j2 = o >> 3, k = o & 7;
            double tau = -1e300;
#pragma unroll
            for (int q = 0; q < kA; ++q) {
                const double d = q - j2 + E2;
                if ((xcol >> q) & 1u) tau = fmax(tau, phi[q] - d * d * invk);
            }
            if (!(tau > -1e299)) tau = 0.0;
            const double d = k - j2 + E2;
            const bool on = (xcol >> k) & 1u;
            KY1(j2)[k] = on ? exp_wide(phi[k] - d * d * invk - tau) : 0.0;
            if (k == 0) *SY1(j2) = -tau;
        }
        for (int o = tl; o < W1 * 8; o += 64 * NW) {
            const int j1 = o >> 3, k = o & 7;
            double tau = -1e300;
#pragma unroll
            for (int q = 0; q < kA; ++q) {
                const double d = q - j1 + E1;
                if ((xrow >> q) & 1u) tau = fmax(tau, psi[q] - d * d * invk);
            }
            if (!(tau > -1e299)) tau = 0.0;
            const double d = k - j1 + E1;
            const bool on = (xrow >> k) & 1u;
            KY2(j1)[k] = on ? fexp((float)(psi[k] - d * d * invk - tau)) : 0.f;
            if (k == 0) *SY2(j1) = -tau;
        }
        Tm::sync();
    };
    build_y(f);

    // number of rows t of this wave inside the box; column blocks of 32
    // rows of lane (r, c) of wave w: j1 = r + 8 (w + NW t), t < ntw (blocks of 8 rows dealt
    // round the waves; a wave with fewer blocks leaves its SIMD to the other workgroups)
    const int ntw = W1 > 8 * w ? min(RPL, (W1 - 8 * w + 8 * NW - 1) / (8 * NW)) : 0;
    const int nb = (W2 + 31) >> 5;

    // ---- Y-update, first part: U1, ry (first wave), then per column j2 (float64):
    //      V = LSE_i2 [f + log mu - cost], My = max_i1 (V - psi), U2 = exp(V - psi - My)
    auto y_first = [&](double fc) {
        if (w == 0) {
            const bool has = mu > 0.0;
            const double wv = has ? fc + lm - phi[c] : kNegD;
            const double ryv = max8(wv);
            U1[lane] = has ? exp_wide(wv - ryv) : 0.0;
            if (c == 0) ry[r] = ryv;
            if (tl == 0) ired[1] = 0;  // no first-X-pass output is uncertain yet
        }
        Tm::sync();
        // LPC aligned lanes share a column, each taking 8 / LPC rows i1
        constexpr int LPC = 2, RQ = kA / LPC;
        for (int j2 = tl / LPC; j2 < W2; j2 += 64 * NW / LPC) {
            const int h = tl % LPC;
            double k1[8];
            ld8d(KY1(j2), k1);
            const double sy = *SY1(j2);
            double v[RQ];
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int i1 = RQ * h + q;
                double a[8];
                ld8d(U1 + i1 * 8, a);
                double sm = a[0] * k1[0];
#pragma unroll
                for (int k = 1; k < 8; ++k) sm = fma(a[k], k1[k], sm);
                const bool row_has = ((xrow >> i1) & 1u) && sm > 0.0;
                v[q] = row_has ? ry[i1] + log_wide(sm) - sy : kNegD;
                Vc(j2)[i1] = v[q];
                // input of the pass over i1: V - psi (rows without mass drop out)
                v[q] = ((xrow >> i1) & 1u) ? v[q] - psi[i1] : kNegD;
            }
            double my = v[0];
#pragma unroll
            for (int q = 1; q < RQ; ++q) my = fmax(my, v[q]);
            if constexpr (LPC == 2)
                my = fmax(my, dppd<kDppXor1>(my));
            else
                my = max8(my);
#pragma unroll
            for (int q = 0; q < RQ; ++q) U2(j2)[RQ * h + q] = fexp((float)(v[q] - my));
            if (h == 0) {
                const int e = dx_block(j2, E2);
                *My(j2) = my;
                *Myx(j2) = my + (double)(e * e) * invk;
            }
        }
        Tm::sync();
    };

    // ---- fused Y-update (second part) and first X pass for the RC rows of one chunk:
    //      Zx = g + log nu_J - lnref - dx2(j2)^2 / kappa (float64), online row maximum over
    //      column blocks, acc(i2) = sum_j2 exp(Zx - max) KX1(j2, i2),
    //      R - dx1(j1)^2 / kappa = max + log acc - dx1(j1)^2 / kappa
    // log nu_J of block (ch, b) (RC rows by 4 column groups of one column block) from global
    // memory; `chunk` issues the next block's loads before it works on the current one, so
    // their latency hides behind a block of work
    using LnBlock = double[LNREG ? 1 : RC][4];
    auto load_ln = [&](int ch, int b, LnBlock& dst) {
        const double* lnb = p.lognu + bse;
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            const int jr = min(r + 8 * (w + NW * (RC * ch + t)), W1 - 1);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jc = min(c + 8 * u + 32 * b, W2 - 1);
                dst[t][u] = lnb[(unsigned)(jr * s1 + jc * s2)];
            }
        }
    };
    auto chunk = [&](int ch, LnBlock& lnq) {
        int j1[RC];
        bool rv[RC], tb[RC];  // tb: the wave's block of 8 rows reaches into the box (uniform)
        float ky[RC][8], acc[RC][8];
        double sy2[RC], m[RC];
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            tb[t] = 8 * (w + NW * (RC * ch + t)) < W1;
            j1[t] = r + 8 * (w + NW * (RC * ch + t));
            rv[t] = j1[t] < W1;
            const int jr = min(j1[t], W1 - 1);
            ld8(KY2(jr), ky[t]);
            sy2[t] = *SY2(jr);
            m[t] = kNegD;
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[t][k] = 0.f;
        }
        for (int b = 0; b < nb; ++b) {
            double Z[RC][4];
            unsigned badm = 0;  // entries whose Y-update sum underflowed
            // log nu_J of the block's entries (loaded during the previous block), and the
            // loads of the next block (this chunk's next column block, else the next chunk's
            // first) issued now
            double lnp[LNREG ? 1 : RC][4];
            if constexpr (!LNREG) {
#pragma unroll
                for (int t = 0; t < RC; ++t)
#pragma unroll
                    for (int u = 0; u < 4; ++u) lnp[t][u] = lnq[t][u];
                const int nch = b + 1 < nb ? ch : ch + 1, nbk = b + 1 < nb ? b + 1 : 0;
                if (RC * nch < ntw) load_ln(nch, nbk, lnq);  // wave-uniform
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j2 = c + 8 * u + 32 * b;
                if (8 * u + 32 * b >= W2) {  // the whole column block lies past the box
#pragma unroll
                    for (int t = 0; t < RC; ++t) Z[t][u] = kNegD;
                    continue;
                }
                const bool cv = j2 < W2;
                const int jc = min(j2, W2 - 1);
                float u2[8];
                ld8(U2(jc), u2);
                const double myv = *Myx(jc);
#pragma unroll
                for (int t = 0; t < RC; ++t) {
                    if (!tb[t]) {
                        Z[t][u] = kNegD;
                        continue;
                    }
                    float y = ky[t][0] * u2[0];
#pragma unroll
                    for (int k = 1; k < 8; ++k) y = fmaf(ky[t][k], u2[k], y);
                    double lnv;
                    if constexpr (LNREG) {
                        lnv = (double)lnr[RC * ch + t][u];
                    } else {
                        const double v = lnp[t][u];
                        lnv = v > kZeroMassLog ? v - lnref : kNegD;
                    }
                    const bool valid = rv[t] && cv && lnv > kZeroMassLog;
                    const bool under = !(y >= kFloorF);
                    badm |= (unsigned)(valid && under) << (t * 4 + u);
                    const double z = lnv - myv - (klog(y) - sy2[t]);
                    Z[t][u] = (valid && !under) ? z : kNegD;
                }
            }
            if (__builtin_expect(badm != 0, 0)) {
                // those entries exactly (log nu_J re-read from global memory)
#pragma unroll 1
                for (int q = 0; q < RC * 4; ++q) {
                    if (!((badm >> q) & 1u)) continue;
                    const int jq = r + 8 * (w + NW * (RC * ch + (q >> 2)));
                    const int kq = c + 8 * (q & 3) + 32 * b, e = dx_block(kq, E2);
                    const double ln = p.lognu[bse + (int64_t)jq * s1 + (int64_t)kq * s2];
                    const double z = ln - lnref - (double)(e * e) * invk -
                                     exact_y2(colp(kq), jq, E1, invk);
#pragma unroll
                    for (int pq = 0; pq < RC * 4; ++pq)
                        if (pq == q) Z[pq >> 2][pq & 3] = z;
                }
                if (c == 0 && r == 0) atomicAdd(&g.ctrl[15], 1);
            }
#pragma unroll
            for (int t = 0; t < RC; ++t) {
                if (!tb[t]) continue;
                double mb = fmax(fmax(Z[t][0], Z[t][1]), fmax(Z[t][2], Z[t][3]));
                mb = max8(mb);
                const double mn = fmax(m[t], mb);
                const float sc = fexp((float)(m[t] - mn));
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[t][k] *= sc;
                m[t] = mn;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (8 * u + 32 * b >= W2) continue;
                const int jc = min(c + 8 * u + 32 * b, W2 - 1);
                float kx[8];
                ld8(KX1(jc), kx);
#pragma unroll
                for (int t = 0; t < RC; ++t) {
                    if (!tb[t]) continue;
                    const float e0 = fexp((float)(Z[t][u] - m[t]));
                    const float e = Z[t][u] > kZeroMassLog ? e0 : 0.f;
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc[t][k] = fmaf(e, kx[k], acc[t][k]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            if (!tb[t]) continue;
            const float a = rs8(acc[t], c);
            const int e1 = dx_block(j1[t], E1);
            double R = m[t] + klog(a) - (double)(e1 * e1) * invk;
            const bool live = rv[t] && m[t] > kZeroMassLog;
            const bool unc = live && !(a >= kFloorF);
            if (__builtin_expect(unc, 0)) {
                // the sum is below the floor: keep an upper bound for now
                R = m[t] + klog(2.f * kFloorF) - (double)(e1 * e1) * invk;
                ired[1] = 1;
                if (c == 0) atomicAdd(&g.ctrl[12], 1);
            }
            if (rv[t]) {
                Rr(j1[t])[c] = live ? R : kNegD;
                UNC(j1[t])[c] = unc ? 1 : 0;
            }
        }
    };

    // ---- exact first X pass of the rows marked by `chunk`: the 8 lanes of a row split its
    //      columns, keep a running maximum and sum per output, then combine
    auto fix_rows = [&]() {
        for (int t = 0; t < ntw; ++t) {
            const int j1 = r + 8 * (w + NW * t), jr = min(j1, W1 - 1);
            const bool need = j1 < W1 && UNC(jr)[c] != 0;
            const unsigned long long bm = __ballot(need);
            if (!bm) continue;  // wave-uniform
            const bool rowneed = ((bm >> (8 * r)) & 0xFFull) != 0;
            float ky[8];
            ld8(KY2(jr), ky);
            const double sy2 = *SY2(jr);
            double mo[8], so[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                mo[k] = -1e300;
                so[k] = 0.0;
            }
            if (rowneed) {
                for (int j2 = c; j2 < W2; j2 += 8) {
                    const double ln = p.lognu[bse + (int64_t)jr * s1 + (int64_t)j2 * s2];
                    if (!(ln > kZeroMassLog)) continue;
                    float u2[8];
                    ld8(U2(j2), u2);
                    float y = ky[0] * u2[0];
#pragma unroll
                    for (int k = 1; k < 8; ++k) y = fmaf(ky[k], u2[k], y);
                    const double z = y >= kFloorF
                                         ? ln - lnref - *My(j2) - (klog(y) - sy2)
                                         : ln - lnref - exact_y2(colp(j2), jr, E1, invk);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const double d = j2 - k - E2;
                        const double v = z - d * d * invk;
                        if (v > mo[k]) {
                            so[k] = so[k] * (double)fexp((float)(mo[k] - v)) + 1.0;
                            mo[k] = v;
                        } else {
                            so[k] += (double)fexp((float)(v - mo[k]));
                        }
                    }
                }
            }
            // combine the 8 lanes of the row: common maximum, rescaled sums
            float sf[8];
            double M[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                M[k] = max8(mo[k]);
                sf[k] = (float)(so[k] * (double)fexp((float)(mo[k] - M[k])));
            }
            const float ssum = rs8(sf, c);
            double Mc = M[0];
#pragma unroll
            for (int k = 1; k < 8; ++k) Mc = c == k ? M[k] : Mc;
            const int e1 = dx_block(jr, E1);
            if (need) {
                Rr(jr)[c] = ssum > 0.f ? Mc + klog(ssum) - (double)(e1 * e1) * invk
                                       : kNegD;
                UNC(jr)[c] = 0;
            }
        }
        Tm::sync();
    };

    // ---- rest of one iteration from f = fc: returns s (first wave) and err ----------------
    auto iterate = [&](double fc, bool want_err, double& s_out, double& err_out) {
        LnBlock lnq;
        if constexpr (LNREG) {
#pragma unroll
            for (int ch = 0; ch < RPL / RC; ++ch)
                if (RC * ch < ntw) chunk(ch, lnq);
        } else {
            if (ntw > 0) load_ln(0, 0, lnq);
            for (int ch = 0; RC * ch < ntw; ++ch) chunk(ch, lnq);
        }
        Tm::sync();
        // second X pass (float64): Mx(i2) = max_j1 R, S(i1, i2) = sum_j1 KX2(j1, i1) exp(R - Mx),
        // once without the uncertain first-pass outputs (lo) and once with their upper bounds
        // (hi).  lo <= exact <= hi: when hi exceeds lo by at most 1e-9 everywhere, lo stands;
        // otherwise the uncertain outputs are computed exactly and the pass is repeated.
        for (;;) {
            double mx = kNegD;
            for (int t = 0; t < ntw; ++t) {
                const int j1 = r + 8 * (w + NW * t);
                const double v = Rr(min(j1, W1 - 1))[c];
                mx = j1 < W1 ? fmax(mx, v) : mx;
            }
            mx = maxr(mx);
            if constexpr (NW > 1) {
                if (r == 0) xd[w * 8 + c] = mx;
                Tm::sync();
                mx = xd[c];
#pragma unroll
                for (int q = 1; q < NW; ++q) mx = fmax(mx, xd[q * 8 + c]);
            }
            // (the upper sums only while some first-pass output is uncertain: team-uniform)
            const bool unc = __builtin_amdgcn_readfirstlane(ired[1]) != 0;
            double lo[8], hi[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) lo[k] = hi[k] = 0.0;
            if (unc) {
                for (int t = 0; t < ntw; ++t) {
                    const int j1 = r + 8 * (w + NW * t), jc = min(j1, W1 - 1);
                    const double Rv = Rr(jc)[c];
                    const double u4 = (j1 < W1 && Rv > kZeroMassLog) ? exp_wide(Rv - mx) : 0.0;
                    const double ul = UNC(jc)[c] ? 0.0 : u4;
                    double kx[8];
                    ld8d(KX2(jc), kx);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        hi[k] = fma(kx[k], u4, hi[k]);
                        lo[k] = fma(kx[k], ul, lo[k]);
                    }
                }
            } else {
                for (int t = 0; t < ntw; ++t) {
                    const int j1 = r + 8 * (w + NW * t), jc = min(j1, W1 - 1);
                    const double Rv = Rr(jc)[c];
                    const double u4 = (j1 < W1 && Rv > kZeroMassLog) ? exp_wide(Rv - mx) : 0.0;
                    double kx[8];
                    ld8d(KX2(jc), kx);
#pragma unroll
                    for (int k = 0; k < 8; ++k) lo[k] = fma(kx[k], u4, lo[k]);
                }
            }
            double Slo = rsrd(lo, r);
            double Shi = unc ? rsrd(hi, r) : Slo;
            if constexpr (NW > 1) {
                xs[w * 64 + lane] = Slo;
                if (unc) xs[(NW + w) * 64 + lane] = Shi;
                Tm::sync();
                if (w == 0) {
                    Slo = xs[lane];
#pragma unroll
                    for (int q = 1; q < NW; ++q) Slo += xs[q * 64 + lane];
                    Shi = Slo;
                    if (unc) {
                        Shi = xs[NW * 64 + lane];
#pragma unroll
                        for (int q = 1; q < NW; ++q) Shi += xs[(NW + q) * 64 + lane];
                    }
                }
            }
            bool redo = false;
            if (ired[1] != 0) {  // team-uniform: written before the last synchronisation
                const bool off = w == 0 && mu > 0.0 && !(Shi <= Slo * (1.0 + 1e-9));
                if constexpr (NW > 1) {
                    if (tl == 0) ired[4] = 0;
                    Tm::sync();
                    if (off) ired[4] = 1;
                    Tm::sync();
                    redo = ired[4] != 0;
                } else {
                    redo = __ballot(off) != 0;
                }
            }
            if (__builtin_expect(redo, 0)) {
                fix_rows();
                if (tl == 0) {
                    ired[1] = 0;
                    atomicAdd(&g.ctrl[14], 1);
                }
                Tm::sync();
                continue;
            }
            if (w == 0) {
                double sr = lnref + mx + log_wide(Slo);
                if (__builtin_expect(!(Slo > 0.0 && mx > kZeroMassLog), 0)) {
                    sr = lnref + exact_x2(rows, r, c, W1, E1, invk);
                    atomicAdd(&g.ctrl[13], 1);
                }
                s_out = sr;
                if (want_err) err_out = wsum(mu > 0.0 ? mu * fabs(expm1(fc + sr)) : 0.0);
            }
            break;
        }
    };

    // ---- g = -LSE_i [f + log mu - C] over the box, written to p.b -------------------------
    auto write_g = [&]() {
        for (int t = 0; t < ntw; ++t) {
            const int j1 = r + 8 * (w + NW * t);
            if (j1 >= W1) continue;
            float ky[8];
            ld8(KY2(j1), ky);
            const double sy2 = *SY2(j1);
            for (int j2 = c; j2 < W2; j2 += 8) {
                float u2[8];
                ld8(U2(j2), u2);
                float y = ky[0] * u2[0];
#pragma unroll
                for (int k = 1; k < 8; ++k) y = fmaf(ky[k], u2[k], y);
                double gv = -(*My(j2) + klog(y) - sy2);
                if (__builtin_expect(!(y >= kFloorF), 0)) gv = -exact_y2_call(colp(j2), j1, E1, invk);
                p.b[bse + (int64_t)j1 * s1 + (int64_t)j2 * s2] = gv;
            }
        }
    };

    // One loop for the three modes.  Every pass starts with the first part of the Y-update
    // from fc; it then either completes an iteration or, as the last pass, writes g.  At a
    // stop f stays at the start of the last iteration: (f, g) is the pair whose X-marginal
    // error was measured.
    double fc = f, err = 0.0, eref = 1e300, s = 0.0;
    double fprof = f;  // the f the absorbed profiles were built from (first wave)
    int it = 0;
    bool gpass = g.mode == kFinal;
    for (;;) {
        if (it > 0) {
            // The absorbed profiles follow f: a long solve refreshes them every 16 iterations,
            // and any solve as soon as f has moved by more than kProfileDrift anywhere since
            // they were built (e.g. the first iterations from a start far from the solution),
            // before the float64 factors of the first Y pass could underflow.
            double dv = (w == 0 && mu > 0.0) ? fabs(fc - fprof) : 0.0;
            if (w == 0) dv = wmax(dv);
            if constexpr (NW > 1) {
                if (tl == 0) red[2] = dv;
                Tm::sync();
                dv = red[2];
            }
            dv = uni(dv);
            if ((g.mode == kSolve && (it & 15) == 0) || dv > kProfileDrift) {
                build_y(fc);
                fprof = fc;
            }
        }
        y_first(fc);
        if (gpass) {
            write_g();
            break;
        }
        ++it;
        iterate(fc, g.mode == kSolve || it == K, s, err);
        if (g.mode == kBatch) {
            if (it >= K) {
                if (w == 0) g.f_keep[(int64_t)cell * 64 + xo] = fc;
                fc = -s;
                break;
            }
            fc = -s;
            continue;
        }
        // the first wave's error, known to every thread (same stop decision everywhere)
        if constexpr (NW > 1) {
            if (tl == 0) red[0] = err;
            Tm::sync();
            err = red[0];
        }
        err = uni(err);
        bool stop = it >= g.limit || (!g.fixed && err <= g.tol * mass_all);
        if (!g.fixed && g.stall > 0 && it % g.stall == 0) {
            if (err > 0.9995 * eref) stop = true;
            eref = err;
        }
        if (stop)
            gpass = true;
        else
            fc = -s;
    }
    if (w == 0) p.a[(int64_t)cell * 64 + xo] = fc;
    if (tl == 0) {
        if (g.mode == kFinal) {
            g.iters[cell] = g.ctrl[2];
        } else {
            if (g.mode == kSolve) g.iters[cell] = it;
            g.err[cell] = err;
            g.mass[cell] = mass_all;
        }
    }
    Tm::sync();
}

// batch rule: spacing of the tests in units of the least spacing (check_every), and the
// fraction of the predicted remaining iterations run before the next test
constexpr int kFirstRounds = 4, kMaxRounds = 32;
constexpr double kAheadFrac = 0.8;
constexpr int kSpecRounds = 4;  // rounds of a speculative solve (and between host reads)
// A tolerance solve's float32 phase aims below the tolerance, so that the float64 finish
// usually certifies it with its first error (float32 and float64 errors differ by a few
// percent, and every float64 iteration costs as much as ~15 float32 ones); it hands over
// early when its error stalls within kStallNear of that target.
constexpr double kF32Target = 0.85, kStallNear = 4.0, kStallRel = 1e-4;

// threads of a workgroup: four one-wave teams, or one team of NW waves
__host__ __device__ constexpr int team_block(int NW) { return NW == 1 ? kBlock : 64 * NW; }

template <int NW, int RPL, bool LNREG, int RC>
__global__ void __launch_bounds__(team_block(NW)) __attribute__((amdgpu_waves_per_eu(2)))
fast_kernel(FastArgs g) {
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_q, s_last;
    __shared__ double s_red[team_block(NW) / 64];
    int K = 0;
    if (g.mode == kBatch) {
        if (__atomic_load_n(&g.ctrl[2], __ATOMIC_RELAXED) != 0) return;
        // this round's length, set by the previous round's test (0: the first rounds)
        const int next = __atomic_load_n(&g.ctrl[5], __ATOMIC_RELAXED);
        K = min(next > 0 ? next : kFirstRounds * g.chunk,
                g.max_iter - __atomic_load_n(&g.ctrl[10], __ATOMIC_RELAXED));
    }
    int* queue = &g.ctrl[g.qidx];
    if constexpr (NW == 1) {
        const int lane = threadIdx.x & 63;
        const int slot = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const lds_p<char> base = (lds_p<char>)smem + slot * (int)slice_bytes(1, g.W1m, g.W2m);
        for (;;) {
            int q = 0;
            if (lane == 0) q = atomicAdd(queue, 1);
            q = __builtin_amdgcn_readfirstlane(__shfl(q, 0, 64));
            if (q >= g.n) break;
            run_cell<NW, RPL, LNREG, RC>(g, q, base, K);
        }
    } else {
        const lds_p<char> base = (lds_p<char>)smem;
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) s_q = atomicAdd(queue, 1);
            __syncthreads();
            const int q = s_q;
            if (q >= g.n) break;
            run_cell<NW, RPL, LNREG, RC>(g, q, base, K);
        }
    }
    if (g.mode != kBatch) return;
    // last workgroup of the round: reduce the per-cell errors in fixed cell order
    __syncthreads();
    __threadfence();
    if (threadIdx.x == 0) s_last = (atomicAdd(&g.ctrl[1], 1) == g.nblocks - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // by the first 256 threads in every class, so that the sum (and the stop) does not depend
    // on which class's workgroup comes last (the eight-wave class's other waves add zeros)
    double e = 0.0, m = 0.0;
    for (int c = threadIdx.x; threadIdx.x < 256 && c < g.p.ncells; c += 256) {
        e += g.err[c];
        m += g.mass[c];
    }
    e = block_sum(e, s_red);
    m = block_sum(m, s_red);
    if (threadIdx.x == 0) {
        const int it = g.ctrl[10] + K;
        g.dtot[0] = e;
        g.dtot[1] = m;
        const double lim = g.tol * m;
        const bool conv = e <= lim;
        if (conv) g.ctrl[4] = 1;
        g.ctrl[10] = it;
        const int it0 = g.ctrl[6];
        const double e0 = g.dtot[5];
        // an error near the target that no longer falls in float32 is left to the float64
        // finish that follows this phase
        const bool stalled = it0 > 0 && !conv && e <= kStallNear * lim && !(e < e0 * (1.0 - kStallRel));
        if (conv || stalled || it >= g.max_iter || !(e == e))
            __atomic_store_n(&g.ctrl[2], it, __ATOMIC_RELAXED);
        // length of the next round: the first two tests come kFirstRounds * chunk iterations
        // apart; later ones after a fraction of the iterations still needed if the error keeps
        // the geometric decay of the last two tests (never fewer than chunk, never more than
        // kMaxRounds * chunk)
        int next = it0 > 0 ? g.chunk : kFirstRounds * g.chunk;
        if (it0 > 0 && !conv && e < e0 && e > lim && lim > 0.0) {
            const double rate = log(e / e0) / (double)(it - it0);  // < 0
            const double left = log(lim / e) / rate;               // > 0
            next = (int)fmin(kAheadFrac * left, (double)(kMaxRounds * g.chunk));
            next = max(next, g.chunk);
        }
        g.ctrl[5] = next;
        g.ctrl[6] = it;
        g.dtot[5] = e;
        g.ctrl[0] = 0;
        g.ctrl[9] = 0;
        g.ctrl[11] = 0;
        g.ctrl[1] = 0;
    }
}

// the records of the queue slots: the cell, its box dims, shifts and base
__global__ void pack_recs_kernel(int n, const int32_t* __restrict__ order,
                                 const int32_t* __restrict__ dims, const int32_t* __restrict__ shift,
                                 const int64_t* __restrict__ base, int4* recs) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int c = order[q];
    const uint64_t b = (uint64_t)base[c];
    recs[2 * q] = make_int4(c, dims[2 * c], dims[2 * c + 1], 0);
    recs[2 * q + 1] = make_int4(shift[2 * c], shift[2 * c + 1], (int)(uint32_t)b,
                                (int)(uint32_t)(b >> 32));
}

__global__ void fill_ints(int* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// one wave per cell: box long side <= 32 (4 rows per lane, one column block)
#ifndef FAST_WAVE_RC
#define FAST_WAVE_RC 2
#endif
#ifndef FAST_GROUP_RC
#define FAST_GROUP_RC 2
#endif
constexpr int kWaveSide = 32;  // the most rows a one-wave team covers (4 per lane)
#define FAST_WAVE fast_kernel<1, 4, true, FAST_WAVE_RC>
#define FAST_GROUP fast_kernel<4, 16, false, FAST_GROUP_RC>
#define FAST_BIG fast_kernel<8, 8, false, FAST_GROUP_RC>
// Boxes of more entries than this take the longest per iteration (the time of smaller cells
// is bounded by their latency): they get teams of eight waves and are dispatched first.
constexpr int kBigEntries = 2048;

int cus() {
    static int n = 0;
    if (!n) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n < 1)
            n = 1;
    }
    return n;
}

// Workgroups per CU of a kernel at a block size and LDS size, asked of the runtime once per
// (kernel, block, LDS) on this device and then remembered.
template <typename Kern>
Status prep(Kern k, int block, size_t lds, int items, int& grid) {
    Status S;
    struct Key {
        const void* k;
        int block, dev;
        size_t lds;
        bool operator<(const Key& o) const {
            return std::tie(k, block, dev, lds) < std::tie(o.k, o.block, o.dev, o.lds);
        }
    };
    static std::mutex mu;
    static std::map<Key, int> per_cu;
    static std::map<std::pair<const void*, int>, size_t> lds_set;
    int dev = 0;
    DD_HIP(hipGetDevice(&dev), S);
    const Key key{(const void*)k, block, dev, lds};
    std::lock_guard<std::mutex> lock(mu);
    size_t& set = lds_set[{(const void*)k, dev}];
    if (lds > set) {
        DD_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds),
               S);
        set = lds;
    }
    auto it = per_cu.find(key);
    if (it == per_cu.end()) {
        int per = 0;
        DD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, block, lds), S);
        it = per_cu.emplace(key, std::max(per, 1)).first;
    }
    grid = std::max(1, std::min(items, it->second * cus()));
    return S;
}

}  // namespace

namespace {
// class of a box with long side a and short side b (kernel frame)
int cell_class(const FastClasses& k, int a, int b) {
    return a <= k.wave_side ? 0 : a * b > k.big_entries ? 2 : 1;
}
constexpr int kClassTeam[kClasses] = {1, 4, 8};
constexpr size_t kLdsPerCu = 160 * 1024;

// Candidate class thresholds, the measured default first (sweeps on the 512^2 mixtures).
constexpr FastClasses kCandidates[] = {{kWaveSide, kBigEntries}, {32, 1024}, {32, 4096},
                                       {24, 2048},                {24, 1024}, {24, 4096}};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);
static_assert(kWaveSide == 32, "one-wave teams cover 32 rows (4 per lane)");

class ClassTuner {
    static constexpr double kMargin = 0.97;

   public:
    int pick(const std::array<int, 3>& k) {
        std::lock_guard<std::mutex> g(mu_);
        Entry& e = tab_[k];
        for (int c = 0; c < kNumCandidates; ++c)
            if (e.n[c] == 0) return c;
        // the default stays unless another candidate is faster by more than run-to-run noise
        int best = 0;
        for (int c = 1; c < kNumCandidates; ++c)
            if (e.t[c] < kMargin * e.t[0] && e.t[c] < e.t[best]) best = c;
        return best;
    }
    void record(const std::array<int, 3>& k, int c, double t) {
        std::lock_guard<std::mutex> g(mu_);
        Entry& e = tab_[k];
        e.t[c] = e.n[c] ? std::min(e.t[c], t) : t;
        e.n[c] += 1;
    }
    // a pair to use from now on, or (0, 0): back to tuning, from scratch
    void force(int ws, int be) {
        std::lock_guard<std::mutex> g(mu_);
        forced_ = FastClasses{ws, be};
        has_forced_ = ws > 0;
        if (!has_forced_) tab_.clear();
    }
    bool forced(FastClasses* k) {
        std::lock_guard<std::mutex> g(mu_);
        if (has_forced_) *k = forced_;
        return has_forced_;
    }

   private:
    struct Entry {
        double t[kNumCandidates] = {};
        int n[kNumCandidates] = {};
    };
    std::mutex mu_;
    std::map<std::array<int, 3>, Entry> tab_;
    FastClasses forced_;
    bool has_forced_ = false;
};

ClassTuner& class_tuner() {
    static ClassTuner t;
    return t;
}

bool eligible_with(const SkBatch& p, const std::vector<int32_t>& hd, const FastClasses& cls) {
    int W1m[kClasses] = {1, 1, 1}, W2m[kClasses] = {1, 1, 1};
    for (int c = 0; c < p.ncells; ++c) {
        const int a = std::max(std::max(hd[2 * c], hd[2 * c + 1]), 1);
        const int b = std::max(std::min(hd[2 * c], hd[2 * c + 1]), 1);
        if (a > kFastMaxSide) return false;
        const int k = cell_class(cls, a, b);
        W1m[k] = std::max(W1m[k], a);
        W2m[k] = std::max(W2m[k], b);
    }
    for (int k = 0; k < kClasses; ++k) {
        const int t = kClassTeam[k];
        const size_t need = t == 1 ? kBlock / 64 * slice_bytes(1, W1m[k], W2m[k])
                                   : slice_bytes(t, W1m[k], W2m[k]);
        if (need > kLdsPerCu) return false;
    }
    return true;
}

bool fast_off() {
    static const bool off = [] {
        const char* e = std::getenv("DD_FAST");
        return e && e[0] == '0';
    }();
    return off;
}
}  // namespace

void fast_force(int wave_side, int big_entries) { class_tuner().force(wave_side, big_entries); }

void fast_record(const int key[3], int choice, double ms_per_term) {
    if (choice < 0 || choice >= kNumCandidates || !(ms_per_term > 0.0)) return;
    class_tuner().record({key[0], key[1], key[2]}, choice, ms_per_term);
}

bool fast_plan(const SkBatch& p, const std::vector<int32_t>& hd, const dd_sinkhorn_opts& o,
               FastClasses* cls, int* choice, int key[3]) {
    *choice = -1;
    if (fast_off() || p.prec != DD_PREC_F32 || p.xside != kA) return false;
    FastClasses f;
    if (class_tuner().forced(&f)) {
        *cls = f;
        return eligible_with(p, hd, f);
    }
    // the key: the mode and the cell count (a DD layer's partitions share it across the eps
    // stages, so the candidates are tried in the first solves of a layer); the mean box area
    // in powers of four
    double area = 0.0;
    for (int c = 0; c < p.ncells; ++c)
        area += (double)std::max(hd[2 * c], 1) * std::max(hd[2 * c + 1], 1);
    key[0] = o.fixed_iters > 0 ? 2 : o.stop_rule;
    key[1] = (int)std::log2(std::max(1.0, area / std::max(p.ncells, 1))) / 2;
    key[2] = (int)std::log2(std::max(1, p.ncells));
    const int c = class_tuner().pick({key[0], key[1], key[2]});
    if (eligible_with(p, hd, kCandidates[c])) {
        *cls = kCandidates[c];
        *choice = c;
        return true;
    }
    // a candidate whose classes do not fit the LDS: the default, untimed
    *cls = kCandidates[0];
    return eligible_with(p, hd, kCandidates[0]);
}

int fast_spec_max_iters(int chunk) {
    return kSpecRounds * std::max(kFirstRounds, kMaxRounds) * std::max(chunk, 1);
}

bool fast_eligible(const SkBatch& p, const std::vector<int32_t>& hd) {
    if (fast_off() || p.prec != DD_PREC_F32 || p.xside != kA) return false;
    return eligible_with(p, hd, FastClasses{});
}

Status fast_solve(const SkBatch& p, const dd_sinkhorn_opts& o, hipStream_t st, SkWork& w,
                  const std::vector<int32_t>& hd, const std::vector<int32_t>& order,
                  int32_t* iters, double* errs, FastInfo* info, bool final_pass,
                  int32_t* h_ord, FastClasses classes, int phase, int spec_rounds) {
    Status S;
    const int n = p.ncells;
    const bool resume = phase == kFastResume;
    // Cell classes by box shape (kernel frame), most work first within each:
    //   0: long side <= classes.wave_side (<= 32): one wave per cell (four per workgroup),
    //      log nu_J in registers;
    //   1: the rest up to classes.big_entries entries: a workgroup of four waves per cell;
    //   2: larger boxes: a workgroup of eight waves per cell.
    // Classes 1 and 2 read log nu_J from global memory.
    using KernFn = void (*)(FastArgs);
    const KernFn fns[kClasses] = {FAST_WAVE, FAST_GROUP, FAST_BIG};
    const int* team = kClassTeam;
    const int rpl[kClasses] = {4, 16, 8};  // rows per lane: a team covers 8 * team * rpl rows
    const int qidx[kClasses] = {9, 0, 11};
    // the eight-wave class goes on the caller's stream, which no event holds back, so that its
    // workgroups are dispatched first
    const hipStream_t streams[kClasses] = {w.stream2, w.stream3, st};
    std::vector<int32_t> cells[kClasses];
    int W1m[kClasses] = {1, 1, 1}, W2m[kClasses] = {1, 1, 1};
    for (int c : order) {  // most work first within each class
        const int a = std::max(std::max(hd[2 * c], hd[2 * c + 1]), 1);
        const int b = std::max(std::min(hd[2 * c], hd[2 * c + 1]), 1);
        const int k = cell_class(classes, a, b);
        cells[k].push_back(c);
        W1m[k] = std::max(W1m[k], a);
        W2m[k] = std::max(W2m[k], b);
    }
    std::vector<int32_t> ord;
    ord.reserve(n);
    int first[kClasses];
    for (int k = 0; k < kClasses; ++k) {
        first[k] = (int)ord.size();
        ord.insert(ord.end(), cells[k].begin(), cells[k].end());
    }
    const bool arena = w.arena != nullptr;  // no-allocation mode: caller's stream, no events
    if (arena) {
        if ((S = arena_take(w, w.order, (size_t)n)).code ||
            (S = arena_take(w, w.scr_off, (size_t)n)).code ||
            (S = arena_take(w, w.recs, 2 * (size_t)n)).code)
            return S;
        w.order_cap = n;
        w.recs_cap = n;
    } else if (n > w.order_cap) {
        w.mem.put(w.order);
        w.mem.put(w.scr_off);
        w.order = nullptr;
        w.scr_off = nullptr;
        w.order_cap = std::max(n, 1024);
        DD_HIP(w.mem.get(&w.order, w.order_cap * sizeof(int32_t)), S);
        DD_HIP(w.mem.get(&w.scr_off, w.order_cap * sizeof(int64_t)), S);
    }
    if (!arena && n > w.recs_cap) {
        w.mem.put(w.recs);
        w.recs = nullptr;
        w.recs_cap = std::max(n, 1024);
        DD_HIP(w.mem.get(&w.recs, 2 * (size_t)w.recs_cap * sizeof(int4)), S);
    }
    if (n > 0 && !resume) {  // (a resumed solve's order and records are on the device)
        if (h_ord) std::copy(ord.begin(), ord.end(), h_ord);
        DD_HIP(hipMemcpyAsync(w.order, h_ord ? h_ord : ord.data(), n * sizeof(int32_t),
                              hipMemcpyHostToDevice, st),
               S);
        pack_recs_kernel<<<(n + 255) / 256, 256, 0, st>>>(n, w.order, p.dims, p.shift, p.base,
                                                          w.recs);
        if (!h_ord) {
            DD_HIP(hipStreamSynchronize(st), S);
            ++w.waits;
        }  // `ord` goes out of scope here
    }
    FastArgs args[kClasses];
    size_t lds[kClasses];
    int grid[kClasses] = {0, 0, 0};
    int ncls = 0, nblocks = 0;
    for (int k = 0; k < kClasses; ++k) {
        const int nk = (int)cells[k].size();
        lds[k] = team[k] == 1 ? kBlock / 64 * slice_bytes(1, W1m[k], W2m[k])
                              : slice_bytes(team[k], W1m[k], W2m[k]);
        FastArgs& a = args[k];
        a = FastArgs{};
        a.p = p;
        a.cells = w.order + first[k];
        a.recs = w.recs + 2 * (size_t)first[k];
        a.n = nk;
        a.W1m = W1m[k];
        a.W2m = W2m[k];
        a.qidx = qidx[k];
        a.ctrl = w.ctrl;
        a.iters = iters;
        a.err = errs;
        a.mass = w.cell_mass;
        a.dtot = w.dtot;
        a.f_keep = w.a_alt;
        a.tol = o.fixed_iters > 0 ? o.tol : o.tol * kF32Target;
        a.max_iter = o.max_iter;
        if (info) {
            info->n[k] = nk;
            info->lds[k] = (int)lds[k];
        }
        if (!nk) continue;
        if (W1m[k] > 8 * team[k] * rpl[k]) {
            S.code = DD_EINVAL;
            S.msg = "sinkhorn: box side beyond the register-blocked teams";
            return S;
        }
        S = prep(fns[k], team_block(team[k]), lds[k], team[k] == 1 ? (nk + 3) / 4 : nk, grid[k]);
        if (S.code) return S;
        ++ncls;
        nblocks += grid[k];
    }
    // the classes run side by side on three streams, the other two forked from `st` and
    // joined back
    const bool multi = ncls > 1 && !arena;
    auto fork = [&]() {
        if (!multi) return;
        (void)hipEventRecord(w.evf, st);
        (void)hipStreamWaitEvent(w.stream2, w.evf, 0);
        (void)hipStreamWaitEvent(w.stream3, w.evf, 0);
    };
    auto join = [&]() {
        if (!multi) return;
        (void)hipEventRecord(w.evj2, w.stream2);
        (void)hipStreamWaitEvent(st, w.evj2, 0);
        (void)hipEventRecord(w.evj3, w.stream3);
        (void)hipStreamWaitEvent(st, w.evj3, 0);
    };
    // one launch of every class in `mode`, the largest cells first (they are the longest
    // solves of a round, so they start at once); with `ev` the launches are bracketed by
    // events (slot `slot`) on their own streams
    auto launch = [&](const FastArgs& a, int mode, bool ev, int slot) {
        for (int k = kClasses - 1; k >= 0; --k) {
            if (!args[k].n) continue;
            FastArgs x = args[k];
            x.mode = mode;
            x.limit = a.limit;
            x.fixed = a.fixed;
            x.stall = a.stall;
            x.chunk = a.chunk;
            x.nblocks = a.nblocks;
            const hipStream_t sk = multi ? streams[k] : st;
            if (ev) (void)hipEventRecord(w.kev[k][0][slot], sk);
            fns[k]<<<grid[k], team_block(team[k]), lds[k], sk>>>(x);
            if (ev) (void)hipEventRecord(w.kev[k][1][slot], sk);
        }
    };
    auto collect = [&](int slot) {
        for (int k = 0; k < kClasses; ++k) {
            if (!args[k].n || !info) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, w.kev[k][0][slot], w.kev[k][1][slot]) == hipSuccess) {
                info->ms[k] += ms;
                info->launches[k] += 1;
            }
        }
    };
    if (!resume) fill_ints<<<1, 64, 0, st>>>(w.ctrl, 16);
    const bool fixed = o.fixed_iters > 0;
    FastArgs a{};
    if (fixed || o.stop_rule == DD_STOP_CELL) {
        a.limit = fixed ? o.fixed_iters : o.max_iter;
        a.fixed = fixed ? 1 : 0;
        a.stall = fixed ? 0 : 32;  // a float64 finish follows
        fork();
        launch(a, kSolve, false, 0);
        join();
        DD_HIP(hipGetLastError(), S);
        return S;
    }
    a.chunk = std::max(1, o.check_every > 0 ? o.check_every : 8);
    a.nblocks = nblocks;
    // rounds whose lengths the device sets (see the end of fast_kernel), `reps` at a time
    // between reads of the device stop flag;
    // every launch is bracketed by events on its own stream (the per-class kernel time of the
    // statistics), the launches after the stop, which exit at once, included
    const int reps = kSpecRounds;
    if (!arena)
        for (auto& cls : w.kev)
            for (auto& se : cls)
                for (hipEvent_t& e : se)
                    if (!e) DD_HIP(hipEventCreate(&e), S);
    double terms_per_it[kClasses] = {0.0, 0.0, 0.0};
    for (int k = 0; k < kClasses; ++k)
        for (int c : cells[k]) terms_per_it[k] += sk_cell_terms(kA, hd[2 * c], hd[2 * c + 1]);
    if (info)
        for (int k = 0; k < kClasses; ++k) info->terms_per_it[k] = terms_per_it[k];
    int hctl[16] = {};
    if (phase == kFastSpec) {
        // `spec_rounds` (at most `reps`) rounds with no host wait: the caller reads the control
        // words after the whole half-iteration and resumes here if the rule had not stopped
        const int nspec = std::max(1, std::min(reps, spec_rounds));
        for (int r = 0; r < nspec; ++r) {
            fork();
            launch(a, kBatch, true, r);
            join();
        }
        launch_done_iters(n, iters, w.ctrl, st);
        if (info) {
            info->final_done = false;
            info->spec_slots = nspec;
        }
        DD_HIP(hipGetLastError(), S);
        return S;
    }
    if (resume) {
        // the speculative rounds' control words (read back after the caller's wait) and their
        // launch times
        std::copy(w.h_ctl32, w.h_ctl32 + 16, hctl);
        for (int r = 0; r < w.pend.spec_slots; ++r) collect(r);
    }
    // every round that starts before the stop runs at least one iteration
    for (int rounds = 0; rounds < o.max_iter && !hctl[2]; rounds += reps) {
        for (int r = 0; r < reps; ++r) {
            fork();
            launch(a, kBatch, !arena, r);
            join();
        }
        DD_HIP(hipMemcpyAsync(hctl, w.ctrl, sizeof hctl, hipMemcpyDeviceToHost, st), S);
        DD_HIP(hipStreamSynchronize(st), S);
        ++w.waits;
        if (!arena)
            for (int r = 0; r < reps; ++r) collect(r);
    }
    if (info)
        for (int k = 0; k < kClasses; ++k) info->terms[k] = terms_per_it[k] * hctl[10];
    if (info) info->stop_it = hctl[2];
    if (!final_pass && hctl[2] < o.max_iter) {
        // a float64 finish follows from the X potential the last round ended with
        launch_done_iters(n, iters, w.ctrl, st);
        if (info) info->final_done = false;
        DD_HIP(hipGetLastError(), S);
        return S;
    }
    // the final Y-update (g), timed the same way
    fork();
    launch(a, kFinal, !arena, 0);
    join();
    DD_HIP(hipStreamSynchronize(st), S);
    ++w.waits;
    if (!arena) collect(0);
    DD_HIP(hipGetLastError(), S);
    return S;
}

}  // namespace dd
