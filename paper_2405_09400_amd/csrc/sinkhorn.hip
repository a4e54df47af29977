// Batched separable log-domain cell Sinkhorn for gfx950.
//
// The cell problem and its Sinkhorn iteration are those of Alg. "DomDecIter",
// solved in the log domain with the cost evaluated online and split into one 1D
// log-sum-exp pass per axis (App. A.1 "Custom CUDA Sinkhorn").  Potentials are
// f = alpha/eps and g = beta/eps with reference measure mu_J (x) nu_J (equal to the
// paper's mu_J (x) nu up to a constant, Sec. 2.3): pi = mu nu_J exp(f + g - C).
//
// Precision: the log-sum-exp terms run in T (float32 for sinkhorn_batch, float64
// for sinkhorn_batch_f64).  Every 1D pass works on values shifted by a float64
// maximum of their input line, so each float32 term is O(1) no matter how large
// log mu, log nu_J or the potentials are; the line offsets, the potentials f and g,
// the marginal error and the masses are float64.  This is what lets float32 reach a
// marginal tolerance of 1e-5 (the paper saw plain float32 stall, App. A.2.1).
//
// Mapping to the hardware.  A workgroup is four wave64s.  Cells are split on the host by
// their LSE work per iteration: a "big" cell is solved by the whole workgroup, a "small"
// cell by one wave on its own, so a workgroup runs one big cell or four small ones.  Each
// cell keeps f, log mu, the Y box of log nu_J and g and the shifted per-axis intermediates
// in LDS (an LDS tile per class sized from the box-size quantiles; a box larger than its
// tile keeps its Y-box arrays in a per-cell global scratch read through L1/L2).  Each 1D
// pass gives one output per lane and walks its short reduction line from LDS (max pass,
// then exp-sum pass).  Row maxima and the float64 error / mass sums are wave shuffles;
// a wave working alone synchronises with wave-level barriers only.
//
// Two drivers:
//   * per-cell stopping or a fixed iteration count: a persistent kernel; workgroups first
//     pull big cells from one atomic queue, then each wave pulls small cells from a second
//     one, and every cell iterates to its own stop inside LDS -- no HBM traffic and no
//     grid-wide synchronisation between iterations;
//   * the paper's batch rule (App. A.2.1): one launch per iteration that reads f
//     from one buffer and writes the next f into the other, and ends with a
//     last-workgroup float64 reduction of the per-cell errors in fixed cell order
//     that sets a device-side stop flag; later launches exit at once.  The host
//     polls the flag every `check_every` launches, which changes only how many
//     no-op launches trail the stop, never the result.
#include "sinkhorn.hpp"

#include "fastcell.hpp"

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

namespace dd {

namespace {
thread_local std::string g_err;
}
void set_global_error(const std::string& m) { g_err = m; }
const char* global_error() { return g_err.c_str(); }

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

namespace {

// The team that works on one cell: the whole workgroup or one wave.
struct BlockTeam {
    __device__ int tid() const { return threadIdx.x; }
    __device__ int size() const { return blockDim.x; }
    __device__ int wid() const { return threadIdx.x >> 6; }
    __device__ int nw() const { return blockDim.x >> 6; }
    __device__ void sync() const { __syncthreads(); }
    template <typename P>
    __device__ double sum(double v, P scratch) const {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
        v = wave_sum(v);
        __syncthreads();
        if (lane == 0) scratch[w] = v;
        __syncthreads();
        double t = 0.0;
        for (int k = 0; k < nw; ++k) t += scratch[k];
        __syncthreads();
        return t;
    }
};

struct WaveTeam {
    __device__ int tid() const { return threadIdx.x & 63; }
    __device__ int size() const { return 64; }
    __device__ int wid() const { return 0; }
    __device__ int nw() const { return 1; }
    // a wave works from LDS only (small cells never use global scratch), and the LDS
    // operations of one wave are performed in order: keeping the compiler from moving memory
    // operations across this point is all a wave-level barrier needs
    __device__ void sync() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    template <typename P>
    __device__ double sum(double v, P) const { return wave_sum(v); }
};

// Order-preserving map of a double to an unsigned 64-bit key (and back), so that a maximum
// can be taken with an integer atomic.
__device__ __forceinline__ unsigned long long max_key(double d) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
    const unsigned long long u = (k >> 63) ? (k ^ 0x8000000000000000ull) : ~k;
    return __longlong_as_double((long long)u);
}

// Address-space-qualified pointers: LDS (ds_* instructions) and global (global_* ones), so
// that no access in the hot loops goes through flat addressing.
template <typename T>
using lds_p = __attribute__((address_space(3))) T*;
template <typename T>
using glb_p = __attribute__((address_space(1))) T*;

// A cell's working set.  The X arrays always live in LDS; the Y-box arrays live in the LDS
// tile (G = false) or, for a box larger than the tile, in the cell's global scratch (G = true).
//
// Each 1D log-sum-exp pass, LSE_k [in(k) - (k - q + e)^2 / kappa] for the outputs q of one
// line, is evaluated as a stabilised kernel product: with in(k) shifted by the line maximum,
// u(k) = exp(in(k) - max), and the cost split at the input c(q) nearest to q - e,
//   (k - q + e)^2 = (c(q) - q + e)^2 + [(k - q + e)^2 - (c(q) - q + e)^2],
// the pass is  max - s(q) + log sum_k u(k) Kt[k][q],  s(q) = (c(q) - q + e)^2 / kappa,
// Kt[k][q] = exp(-[(k - q + e)^2 - (c(q) - q + e)^2] / kappa) in (0, 1], Kt = 1 at k = c(q).
// Kt and s depend only on the box shape and kappa, so a cell builds its four tables once,
// and the exponentials per iteration drop from one per term to one per input and output.
// A sum that underflows (every input near q is negligible against the line maximum) is
// recomputed for that output by the exact two-pass log-sum-exp.
template <typename T, bool G>
struct Lds {
    using YT = std::conditional_t<G, glb_p<T>, lds_p<T>>;
    using YD = std::conditional_t<G, glb_p<double>, lds_p<double>>;
    // X arrays
    lds_p<double> f;    // [N2]        X potential f
    lds_p<double> lm;   // [N2]        log mu
    lds_p<double> mu;   // [N2]        mu (0 where log mu is the sentinel)
    lds_p<double> s;    // [N2]        LSE_j (g + log nu_J - C)
    lds_p<double> ry;   // [AS]        row maxima of f + log mu
    lds_p<double> Mx;   // [AS]        column maxima of the X-half intermediate
    lds_p<double> red;  // [16]        reductions
    lds_p<T> wq;        // [N2]        f + log mu - ry(row)
    lds_p<T> u1;        // [N2]        exp(wq)
    lds_p<T> sX1;       // [AS]        nearest-point shifts of the X-half passes
    lds_p<T> sX2;       // [AS]
    glb_p<double> gout;  // [W1][W2]   the output g (row stride W2), written by each Y-update
    // Y-box arrays (LDS tile, or global scratch for a box beyond the tile)
    YD qx;              // [W1]        row maxima of g + log nu_J
    YD My;              // [W2]        column maxima of the Y-half intermediate
    YD ln;              // [W1][ys]    log nu_J
    YD v;               // [W1][ys]    g + log nu_J
    YT u3;              // [W1][ys]    exp(v - qx(row))
    YT KY1;             // [AS][W2p]   kernel table, Y-half pass over i2
    YT t1;              // [AS][W2p]   Y-half intermediate, relative to ry
    YT u2;              // [AS][W2p]   exp(t1 + ry - My)
    YT KY2;             // [AS][W1p]   kernel table, Y-half pass over i1
    YT KX1;             // [W2][ASp]   kernel table, X-half pass over j2
    YT r;               // [W1][ASp]   X-half intermediate, relative to qx
    YT u4;              // [W1][ASp]   exp(r + qx - Mx)
    YT KX2;             // [W1][ASp]   kernel table, X-half pass over j1
    YT sY1;             // [W2]
    YT sY2;             // [W1]
    int ys, W2p, W1p, ASp;
};

// Bytes of the X arrays and of the Y-box arrays of a (w1 x w2) box (strides included).
__host__ __device__ inline size_t x_bytes(int AS, size_t elem) {
    const size_t N2 = (size_t)AS * AS;
    return 8 * (4 * N2 + 2 * (size_t)AS + 16) + elem * (2 * N2 + 2 * (size_t)AS);
}
__host__ __device__ inline size_t box_bytes(int AS, int w1, int w2, size_t elem) {
    const size_t ys = (size_t)w2 + 1, W2p = ys, W1p = (size_t)w1 + 1, ASp = (size_t)AS + 1;
    const size_t nd = 2 * (size_t)w1 * ys + w1 + w2;
    const size_t nt = (size_t)w1 * ys + 3 * (size_t)AS * W2p + (size_t)AS * W1p +
                      (size_t)w2 * ASp + 3 * (size_t)w1 * ASp + w2 + w1;
    return 8 * nd + elem * nt + 64;
}

// LDS bytes of one cell slice: the X arrays plus the Y-box arrays for the tile (lw1 x lw2);
// cells beyond the tile keep their Y-box arrays in global scratch (read through L1/L2).
__host__ __device__ inline size_t lds_layout_bytes(int AS, int lw1, int lw2, size_t elem) {
    return (x_bytes(AS, elem) + box_bytes(AS, lw1, lw2, elem) + 15) & ~size_t(15);
}

// Global scratch (in doubles) of a cell whose box exceeds the tile.
__host__ __device__ inline int64_t cell_scratch_doubles(int AS, int W1, int W2, size_t elem) {
    return (int64_t)((box_bytes(AS, W1, W2, elem) + 15) / 16) * 2;
}

// Bind the Y-box arrays of a (W1 x W2) box with strides for (w1s x w2s) starting at `base`.
template <typename T, typename PD, typename PT>
__device__ __forceinline__ void bind_box(PD& ln, PD& vv, PD& qx, PD& My, PT& u3, PT& KY1, PT& t1,
                                         PT& u2,
                                         PT& KY2, PT& KX1, PT& r, PT& u4, PT& KX2, PT& sY1,
                                         PT& sY2, PD base, int AS, int w1s, int w2s) {
    const int ys = w2s + 1, W2p = ys, W1p = w1s + 1, ASp = AS + 1;
    PD d = base;
    ln = d;
    d += (size_t)w1s * ys;
    vv = d;
    d += (size_t)w1s * ys;
    qx = d;
    d += w1s;
    My = d;
    d += w2s;
    PT t = (PT)d;
    u3 = t;
    t += (size_t)w1s * ys;
    KY1 = t;
    t += (size_t)AS * W2p;
    t1 = t;
    t += (size_t)AS * W2p;
    u2 = t;
    t += (size_t)AS * W2p;
    KY2 = t;
    t += (size_t)AS * W1p;
    KX1 = t;
    t += (size_t)w2s * ASp;
    r = t;
    t += (size_t)w1s * ASp;
    u4 = t;
    t += (size_t)w1s * ASp;
    KX2 = t;
    t += (size_t)w1s * ASp;
    sY1 = t;
    t += w2s;
    sY2 = t;
}

// The row-maximum keys share the storage of qx (same address space).
template <typename T, bool G>
__device__ __forceinline__ auto qx_key(const Lds<T, G>& L, int j1) {
    using P = std::conditional_t<G, glb_p<unsigned long long>, lds_p<unsigned long long>>;
    return (P)(L.qx + j1);
}

// Carve the X arrays (and, for G = false, the tile) out of an LDS slice; for G = true bind
// the Y-box arrays to the cell's global scratch.  g and log nu_J point into the packed
// float64 arrays at the cell's offset.
template <typename T, bool G>
__device__ __forceinline__ Lds<T, G> carve(lds_p<char> base, const SkBatch& p, int lw1, int lw2,
                                           int c, int W1, int W2, int64_t ybase,
                                           double* big_scratch) {
    Lds<T, G> L;
    const int AS = p.xside, N2 = AS * AS;
    lds_p<double> d = (lds_p<double>)base;
    L.red = d;
    d += 16;
    L.f = d;
    d += N2;
    L.lm = d;
    d += N2;
    L.mu = d;
    d += N2;
    L.s = d;
    d += N2;
    L.ry = d;
    d += AS;
    L.Mx = d;
    d += AS;
    lds_p<T> t = (lds_p<T>)d;
    L.wq = t;
    t += N2;
    L.u1 = t;
    t += N2;
    L.sX1 = t;
    t += AS;
    L.sX2 = t;
    L.ASp = AS + 1;
    L.gout = (glb_p<double>)(p.b + ybase);
    if constexpr (!G) {
        lds_p<double> bb = (lds_p<double>)(base + ((x_bytes(AS, sizeof(T)) + 15) & ~size_t(15)));
        bind_box<T>(L.ln, L.v, L.qx, L.My, L.u3, L.KY1, L.t1, L.u2, L.KY2, L.KX1, L.r, L.u4, L.KX2, L.sY1,
                    L.sY2, bb, AS, lw1, lw2);
        L.ys = lw2 + 1;
        L.W2p = lw2 + 1;
        L.W1p = lw1 + 1;
    } else {
        glb_p<double> bb = (glb_p<double>)(big_scratch + p.scr_off[c]);
        bind_box<T>(L.ln, L.v, L.qx, L.My, L.u3, L.KY1, L.t1, L.u2, L.KY2, L.KX1, L.r, L.u4, L.KX2, L.sY1,
                    L.sY2, bb, AS, W1, W2);
        L.ys = W2 + 1;
        L.W2p = W2 + 1;
        L.W1p = W1 + 1;
    }
    return L;
}

// Kernel table of one pass: inputs k in [0, K), outputs q in [0, Q), d = k - q + e;
// Kt[k * ks + q * qs] and the shifts sh[q] (see above).
template <typename Tm, typename T, typename P, typename PS>
__device__ __forceinline__ void build_table(const Tm& tm, P Kt, PS sh, int K, int Q, int e,
                                            int ks, int qs, T invk) {
    for (int o = tm.tid(); o < K * Q; o += tm.size()) {
        const int k = o / Q, q = o - k * Q;
        const int c = min(max(q - e, 0), K - 1);
        const int d = k - q + e, dn = c - q + e;
        Kt[k * ks + q * qs] = fexp(-T(d * d - dn * dn) * invk);
        if (k == 0) sh[q] = T(dn * dn) * invk;
    }
}

// Exact LSE_k [in(k) - (k - q + e)^2 / kappa] of one output, in(k) = base[k * stride] + add[k]
// (the fallback of an underflowed kernel-product sum).
template <typename T, typename F>
__device__ __forceinline__ T lse_exact(F in, int K, int q, int e, T invk) {
    T m = T(-3.0e38);
    for (int k = 0; k < K; ++k) {
        const T d = T(k - q + e);
        m = fmax(m, in(k) - d * d * invk);
    }
    T sum = T(0);
    for (int k = 0; k < K; ++k) {
        const T d = T(k - q + e);
        sum += fexp(in(k) - d * d * invk - m);
    }
    return m + flog(sum);
}

// smallest kernel-product sum trusted without the exact fallback
template <typename T>
__device__ __forceinline__ T sum_floor();
template <>
__device__ __forceinline__ float sum_floor<float>() { return 1e-30f; }
template <>
__device__ __forceinline__ double sum_floor<double>() { return 1e-290; }

// Lanes per output for a line of K inputs.  It depends on K only, so a wave and a workgroup
// compute every sum with the same terms in the same order.
__device__ __forceinline__ int lanes_for(int K) {
    return K >= 96 ? 8 : K >= 40 ? 4 : K >= 16 ? 2 : 1;
}

// For every output o in [0, Q): sum_k u[k * su] * kt[k * sk] with (u, su, kt, sk) = line(o),
// by LN lanes per output (strided over k, two accumulators each, combined by a fixed xor
// tree); fin(o, sum) runs on the group's first lane.  Groups of LN consecutive lanes sit in
// one wave and are active together.
template <int LN, typename T, typename Tm, typename FL, typename Fin>
__device__ __forceinline__ void pass_lanes(const Tm& tm, int Q, int K, FL&& line, Fin&& fin) {
    const int tid = tm.tid(), nt = tm.size();
    for (int v = tid; v < Q * LN; v += nt) {
        const int o = v / LN, sub = v - o * LN;
        const auto ln = line(o);
        const auto u = ln.u + sub * ln.su;
        const auto kt = ln.kt + sub * ln.sk;
        const int su = LN * ln.su, sk = LN * ln.sk;
        const int n = (K - sub + LN - 1) / LN;  // terms of this lane
        T a0 = T(0), a1 = T(0);
        int k = 0;
        for (; k + 1 < n; k += 2) {
            a0 += u[k * su] * kt[k * sk];
            a1 += u[(k + 1) * su] * kt[(k + 1) * sk];
        }
        if (k < n) a0 += u[k * su] * kt[k * sk];
        T sum = a0 + a1;
        if constexpr (LN > 1) {
#pragma unroll
            for (int off = 1; off < LN; off <<= 1) sum += __shfl_xor(sum, off, 64);
        }
        if (sub == 0) fin(o, sum);
    }
}

template <typename PU, typename PK>
struct Line {
    PU u;
    int su;
    PK kt;
    int sk;
};

template <typename T, typename Tm, typename FL, typename Fin>
__device__ __forceinline__ void kernel_pass(const Tm& tm, int Q, int K, FL&& line, Fin&& fin) {
    switch (lanes_for(K)) {
        case 8: pass_lanes<8, T>(tm, Q, K, line, fin); break;
        case 4: pass_lanes<4, T>(tm, Q, K, line, fin); break;
        case 2: pass_lanes<2, T>(tm, Q, K, line, fin); break;
        default: pass_lanes<1, T>(tm, Q, K, line, fin); break;
    }
}

// Load one cell: f and log mu into LDS, log nu_J into the tile (G = false), kernel tables.
template <typename Tm, typename T, bool G>
__device__ __forceinline__ void load_cell(const Tm& tm, const SkBatch& p, const Lds<T, G>& L,
                                          const double* f_src, int c, int W1, int W2,
                                          int64_t base) {
    const int AS = p.xside, N2 = AS * AS, tid = tm.tid(), nt = tm.size();
    const int E1 = p.shift[2 * c], E2 = p.shift[2 * c + 1];
    const T invk = T(1.0 / p.kappa);
    // zero-mass points carry the log-domain sentinel in log mu / log nu_J, which removes
    // them from every sum whatever their potential
    for (int i = tid; i < N2; i += nt) {
        const double lm = p.logmu[(int64_t)c * N2 + i];
        L.lm[i] = lm;
        L.mu[i] = lm > kZeroMassLog ? exp(lm) : 0.0;
        L.f[i] = f_src[(int64_t)c * N2 + i];
    }
    for (int o = tid; o < W1 * W2; o += nt) {
        const int j1 = o / W2, j2 = o - j1 * W2;
        L.ln[j1 * L.ys + j2] = p.lognu[base + o];
    }
    // Y-half: over i2 (d = i2 - j2 + E2), over i1 (d = i1 - j1 + E1);
    // X-half: over j2 (d = j2 - i2 - E2), over j1 (d = j1 - i1 - E1)
    build_table(tm, L.KY1, L.sY1, AS, W2, E2, L.W2p, 1, invk);
    build_table(tm, L.KY2, L.sY2, AS, W1, E1, L.W1p, 1, invk);
    build_table(tm, L.KX1, L.sX1, W2, AS, -E2, L.ASp, 1, invk);
    build_table(tm, L.KX2, L.sX2, W1, AS, -E1, L.ASp, 1, invk);
    tm.sync();
}

// Y-update g(j) = -LSE_i [f(i) + log mu(i) - C(i,j)]: pass over i2, then over i1.
// Writes g (float64) to the output array.
template <typename Tm, typename T, bool G>
__device__ __forceinline__ void y_half(const Tm& tm, const Lds<T, G>& L, int AS, int W1, int W2,
                                       int E1, int E2, T invk) {
    const int N2 = AS * AS, tid = tm.tid(), nt = tm.size();
    if (tid < AS) {
        const int i1 = tid;
        double r = L.f[i1 * AS] + L.lm[i1 * AS];
        for (int i2 = 1; i2 < AS; ++i2) r = fmax(r, L.f[i1 * AS + i2] + L.lm[i1 * AS + i2]);
        L.ry[i1] = r;
    }
    tm.sync();
    for (int i = tid; i < N2; i += nt) {
        const T w = (T)(L.f[i] + L.lm[i] - L.ry[i / AS]);
        L.wq[i] = w;
        L.u1[i] = fexp(w);
    }
    tm.sync();
    // pass over i2: t1(i1, j2) = LSE_i2 [wq(i1, i2) - (i2 - j2 + E2)^2 / kappa]
    using YT = typename Lds<T, G>::YT;
    kernel_pass<T>(
        tm, AS * W2, AS,
        [&](int o) {
            const int i1 = o / W2, j2 = o - i1 * W2;
            return Line<lds_p<T>, YT>{L.u1 + i1 * AS, 1, L.KY1 + j2, L.W2p};
        },
        [&](int o, T sum) {
            const int i1 = o / W2, j2 = o - i1 * W2;
            T v;
            if (sum >= sum_floor<T>())
                v = flog(sum) - L.sY1[j2];
            else
                v = lse_exact<T>([&](int k) { return L.wq[i1 * AS + k]; }, AS, j2, E2, invk);
            L.t1[i1 * L.W2p + j2] = v;
        });
    tm.sync();
    // row-maximum keys of the X-half start at the smallest key
    for (int j1 = tid; j1 < W1; j1 += nt)
        *qx_key(L, j1) = 0ull;
    // column maxima over i1 of t1 + ry, and the scaled inputs of the second pass
    for (int j2 = tid; j2 < W2; j2 += nt) {
        double m = (double)L.t1[j2] + L.ry[0];
        for (int i1 = 1; i1 < AS; ++i1) m = fmax(m, (double)L.t1[i1 * L.W2p + j2] + L.ry[i1]);
        L.My[j2] = m;
    }
    tm.sync();
    for (int o = tid; o < AS * W2; o += nt) {
        const int i1 = o / W2, j2 = o - i1 * W2;
        L.u2[i1 * L.W2p + j2] = fexp((T)((double)L.t1[i1 * L.W2p + j2] + L.ry[i1] - L.My[j2]));
    }
    tm.sync();
    // pass over i1: g(j1, j2) = -LSE_i1 [t1(i1, j2) + ry(i1) - (i1 - j1 + E1)^2 / kappa];
    // each output also folds g + log nu_J into its row's maximum (the X-half's row shift),
    // kept as an order-preserving integer key in qx
    kernel_pass<T>(
        tm, W1 * W2, AS,
        [&](int o) {
            const int j1 = o / W2, j2 = o - j1 * W2;
            return Line<YT, YT>{L.u2 + j2, L.W2p, L.KY2 + j1, L.W1p};
        },
        [&](int o, T sum) {
            const int j1 = o / W2, j2 = o - j1 * W2;
            const double Mj = L.My[j2];
            T v;
            if (sum >= sum_floor<T>()) {
                v = flog(sum) - L.sY2[j1];
            } else {
                v = lse_exact<T>(
                    [&](int k) { return L.t1[k * L.W2p + j2] + (T)(L.ry[k] - Mj); }, AS, j1,
                    E1, invk);
            }
            const double g = -(Mj + (double)v);
            L.gout[o] = g;
            const double z = g + L.ln[j1 * L.ys + j2];
            L.v[j1 * L.ys + j2] = z;
            if (z > kZeroMassLog)
                __hip_atomic_fetch_max(qx_key(L, j1), max_key(z), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        });
    tm.sync();
}

// s(i) = LSE_j [g(j) + log nu_J(j) - C(i,j)] (float64 result): pass over j2, then over j1
// (cost (i - j + E)^2 = (j - i - E)^2).
template <typename Tm, typename T, bool G>
__device__ __forceinline__ void x_half(const Tm& tm, const Lds<T, G>& L, int AS, int W1, int W2,
                                       int E1, int E2, T invk) {
    const int tid = tm.tid(), nt = tm.size();
    // row maxima of g + log nu_J (keys left by the Y-update; a row with no mass gets the
    // zero-mass sentinel), then the scaled inputs, all entries in flight at once
    for (int j1 = tid; j1 < W1; j1 += nt) {
        const unsigned long long k = *qx_key(L, j1);
        L.qx[j1] = k ? key_value(k) : kNegD;
    }
    tm.sync();
    for (int o = tid; o < W1 * W2; o += nt) {
        const int j1 = o / W2, j2 = o - j1 * W2;
        const double q = L.qx[j1];
        // a row without mass carries the sentinel in qx and drops out of the second pass
        // whatever its first-pass values; 0 (u = 1) keeps those finite
        L.u3[j1 * L.ys + j2] = q > kZeroMassLog ? fexp((T)(L.v[j1 * L.ys + j2] - q)) : T(1);
    }
    tm.sync();
    // pass over j2: r(j1, i2) = LSE_j2 [g + log nu_J - qx(j1) - (j2 - i2 - E2)^2 / kappa]
    using YT = typename Lds<T, G>::YT;
    kernel_pass<T>(
        tm, W1 * AS, W2,
        [&](int o) {
            const int j1 = o / AS, i2 = o - j1 * AS;
            return Line<YT, YT>{L.u3 + j1 * L.ys, 1, L.KX1 + i2, L.ASp};
        },
        [&](int o, T sum) {
            const int j1 = o / AS, i2 = o - j1 * AS;
            T v;
            if (sum >= sum_floor<T>()) {
                v = flog(sum) - L.sX1[i2];
            } else {
                const double q = L.qx[j1];
                v = lse_exact<T>([&](int k) { return (T)(L.v[j1 * L.ys + k] - q); }, W2, i2, -E2,
                                 invk);
            }
            L.r[j1 * L.ASp + i2] = v;
        });
    tm.sync();
    // column maxima over j1 of r + qx, and the scaled inputs of the second pass
    for (int i2 = tid; i2 < AS; i2 += nt) {
        double m = (double)L.r[i2] + L.qx[0];
        for (int j1 = 1; j1 < W1; ++j1) m = fmax(m, (double)L.r[j1 * L.ASp + i2] + L.qx[j1]);
        L.Mx[i2] = m;
    }
    tm.sync();
    for (int o = tid; o < W1 * AS; o += nt) {
        const int j1 = o / AS, i2 = o - j1 * AS;
        L.u4[j1 * L.ASp + i2] = fexp((T)((double)L.r[j1 * L.ASp + i2] + L.qx[j1] - L.Mx[i2]));
    }
    tm.sync();
    // pass over j1: s(i1, i2) = LSE_j1 [r(j1, i2) + qx(j1) - (j1 - i1 - E1)^2 / kappa]
    kernel_pass<T>(
        tm, AS * AS, W1,
        [&](int o) {
            const int i1 = o / AS, i2 = o - i1 * AS;
            return Line<YT, YT>{L.u4 + i2, L.ASp, L.KX2 + i1, L.ASp};
        },
        [&](int o, T sum) {
            const int i1 = o / AS, i2 = o - i1 * AS;
            const double Mi = L.Mx[i2];
            T v;
            if (sum >= sum_floor<T>()) {
                v = flog(sum) - L.sX2[i1];
            } else {
                v = lse_exact<T>(
                    [&](int k) { return L.r[k * L.ASp + i2] + (T)(L.qx[k] - Mi); }, W1, i1,
                    -E1, invk);
            }
            L.s[o] = Mi + (double)v;
        });
    tm.sync();
}

// X-marginal L1 error sum_i mu |exp(f + s) - 1| and mass sum_i mu, float64, summed by the
// first wave in a fixed order whatever the team (so a cell's stop decision does not depend
// on whether a wave or a workgroup solves it).
template <typename Tm, typename T, bool G>
__device__ __forceinline__ void err_mass(const Tm& tm, const Lds<T, G>& L, int AS, double& err,
                                         double& mass) {
    if (tm.wid() == 0) {
        double e = 0.0, m = 0.0;
        for (int i = threadIdx.x & 63; i < AS * AS; i += 64) {
            const double mu = L.mu[i];
            if (mu > 0.0) {
                e += mu * fabs(expm1(L.f[i] + L.s[i]));
                m += mu;
            }
        }
        e = wave_sum(e);
        m = wave_sum(m);
        if ((threadIdx.x & 63) == 0) {
            L.red[0] = e;
            L.red[1] = m;
        }
    }
    tm.sync();
    err = L.red[0];
    mass = L.red[1];
    tm.sync();
}

// g is written to the output by every Y-update (it lives in p.b), nothing to store.
template <typename Tm, typename T, bool G>
__device__ __forceinline__ void store_g(const Tm&, const SkBatch&, const Lds<T, G>&, int, int,
                                        int64_t) {}

// ctrl words: [0] big-cell queue, [1] ticket, [2] done iteration, [3] bad-dims flag,
// [4] converged, [9] small-cell queue; [5..8] batch statistics
__global__ void zero_ints(int* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Bind cell c to an LDS slice -- its Y-box arrays in the slice's tile when the box fits,
// else (AllowG) in its global scratch -- and run `body` on the view.  A box that fits
// neither sets the bad-dims flag and is skipped.
template <typename T, bool AllowG, typename Tm, typename F>
__device__ __forceinline__ void with_cell(const Tm& tm, const SkBatch& p, lds_p<char> slice,
                                          int lw1, int lw2, int c, double* big_scratch,
                                          int* ctrl, F&& body) {
    const int W1 = p.dims[2 * c], W2 = p.dims[2 * c + 1];
    const bool bad = W1 < 1 || W2 < 1 || W1 > p.max_w1 || W2 > p.max_w2;
    const bool fits = W1 <= lw1 && W2 <= lw2;
    if (bad || (!AllowG && !fits)) {
        if (tm.tid() == 0) atomicOr(&ctrl[3], 1);
        body.skip(c);
        return;
    }
    const int64_t base = p.base[c];
    if (fits) {
        const Lds<T, false> L = carve<T, false>(slice, p, lw1, lw2, c, W1, W2, base, big_scratch);
        body(L, c, W1, W2, base);
    } else if constexpr (AllowG) {
        const Lds<T, true> L = carve<T, true>(slice, p, lw1, lw2, c, W1, W2, base, big_scratch);
        body(L, c, W1, W2, base);
    }
}

// Per-cell rule / fixed count: iterate the cell to its own stop, then store f and g.
template <typename Tm, typename T>
struct SolveCell {
    const Tm& tm;
    const SkBatch& p;
    double tol;
    int limit, fixed, stall_window;
    int32_t* iters_out;
    double* err_out;
    double* mass_out;
    __device__ void skip(int c) const {
        if (tm.tid() == 0) {
            iters_out[c] = 0;
            err_out[c] = 0.0;
            mass_out[c] = 0.0;
        }
    }
    template <bool G>
    __device__ void operator()(const Lds<T, G>& L, int c, int W1, int W2, int64_t base) const {
        const int AS = p.xside, N2 = AS * AS, tid = tm.tid(), nt = tm.size();
        const T invk = T(1.0 / p.kappa);
        const int E1 = p.shift[2 * c], E2 = p.shift[2 * c + 1];
        load_cell(tm, p, L, p.a, c, W1, W2, base);
        double err = 0.0, mass = 0.0, err_ref = 1e300;
        int it = 1;
        for (;; ++it) {
            y_half(tm, L, AS, W1, W2, E1, E2, invk);
            x_half(tm, L, AS, W1, W2, E1, E2, invk);
            err_mass(tm, L, AS, err, mass);
            bool stop = (it >= limit) || (!fixed && err <= tol * mass);
            // a float32 solve whose error has stopped falling (rounding floor) hands the
            // cell to the float64 finish, which certifies the tolerance
            if (!fixed && stall_window > 0 && it % stall_window == 0) {
                if (err > 0.9995 * err_ref) stop = true;
                err_ref = err;
            }
            if (stop) break;
            for (int i = tid; i < N2; i += nt) L.f[i] = -L.s[i];
            tm.sync();
        }
        for (int i = tid; i < N2; i += nt) p.a[(int64_t)c * N2 + i] = L.f[i];
        store_g(tm, p, L, W1, W2, base);
        if (tid == 0) {
            iters_out[c] = it;
            err_out[c] = err;
            mass_out[c] = mass;
        }
        tm.sync();
    }
};

// The cell classes run as separate launches (each with its own LDS size and tile), side by
// side on separate streams.  A launch covers order[q_lo, q_hi) with its tile (lw1, lw2):
// MODE 0 = one cell per workgroup, MODE 1 = one cell per wave.
constexpr int kBig = 0, kSmall = 1;
// A workgroup of up to kBigThreads threads per cell (MODE 0): every sum has the same terms in
// the same order for any workgroup size (a pass's outputs are spread over the threads, each
// output's sum over a fixed group of lanes of one wave; a cell's error over its first wave),
// so the size changes the speed of a class and not its results.
constexpr int kBigThreads = 512;

template <typename T, int MODE>
__global__ void __launch_bounds__(MODE == kBig ? kBigThreads : kThreads)
    sk_cell_kernel(SkBatch p, double tol, int limit, int fixed, int stall_window, int* queue,
                   int* ctrl, int32_t* iters_out, double* err_out, double* mass_out,
                   double* big_scratch) {
    extern __shared__ __align__(16) char smem[];
    const lds_p<char> base = (lds_p<char>)smem;
    if constexpr (MODE == kBig) {
        __shared__ int s_cell;
        const BlockTeam tm;
        const SolveCell<BlockTeam, T> body{tm, p, tol, limit, fixed, stall_window,
                                           iters_out, err_out, mass_out};
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) s_cell = p.q_lo + atomicAdd(queue, 1);
            __syncthreads();
            const int q = s_cell;
            if (q >= p.q_hi) break;
            with_cell<T, true>(tm, p, base, p.lw1, p.lw2, p.order[q], big_scratch, ctrl, body);
        }
    } else {
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
        const lds_p<char> slice = base + w * lds_layout_bytes(p.xside, p.lw1, p.lw2, sizeof(T));
        const WaveTeam tm;
        const SolveCell<WaveTeam, T> body{tm, p, tol, limit, fixed, stall_window,
                                          iters_out, err_out, mass_out};
        for (;;) {
            int q = 0;
            if (lane == 0) q = p.q_lo + atomicAdd(queue, 1);
            q = __builtin_amdgcn_readfirstlane(__shfl(q, 0, 64));
            if (q >= p.q_hi) break;
            // small cells fit the small tile by construction (the host's split)
            with_cell<T, false>(tm, p, slice, p.lw1, p.lw2, p.order[q], big_scratch, ctrl,
                                body);
        }
    }
}

// One batch-rule iteration of a cell: f_in -> f_out, per-cell error and mass.
template <typename Tm, typename T>
struct IterCell {
    const Tm& tm;
    const SkBatch& p;
    const double* f_in;
    double* f_out;
    double* cell_err;
    double* cell_mass;
    __device__ void skip(int c) const {
        if (tm.tid() == 0) {
            cell_err[c] = 0.0;
            cell_mass[c] = 0.0;
        }
    }
    template <bool G>
    __device__ void operator()(const Lds<T, G>& L, int c, int W1, int W2, int64_t base) const {
        const int AS = p.xside, N2 = AS * AS, tid = tm.tid(), nt = tm.size();
        const T invk = T(1.0 / p.kappa);
        const int E1 = p.shift[2 * c], E2 = p.shift[2 * c + 1];
        load_cell(tm, p, L, f_in, c, W1, W2, base);
        y_half(tm, L, AS, W1, W2, E1, E2, invk);
        x_half(tm, L, AS, W1, W2, E1, E2, invk);
        double err, mass;
        err_mass(tm, L, AS, err, mass);
        if (tid == 0) {
            cell_err[c] = err;
            cell_mass[c] = mass;
        }
        for (int i = tid; i < N2; i += nt) f_out[(int64_t)c * N2 + i] = -L.s[i];
        tm.sync();
    }
};

// g from the final f (one Y-update) of a cell, for the batch-rule driver.
template <typename Tm, typename T>
struct FinalCell {
    const Tm& tm;
    const SkBatch& p;
    int done;
    int32_t* iters_out;
    __device__ void skip(int) const {}
    template <bool G>
    __device__ void operator()(const Lds<T, G>& L, int c, int W1, int W2, int64_t base) const {
        const T invk = T(1.0 / p.kappa);
        load_cell(tm, p, L, p.a, c, W1, W2, base);
        y_half(tm, L, p.xside, W1, W2, p.shift[2 * c], p.shift[2 * c + 1], invk);
        store_g(tm, p, L, W1, W2, base);
        if (tm.tid() == 0) iters_out[c] = done;
        tm.sync();
    }
};

// Work items of a launch: one cell per item (MODE 0) or four (MODE 1, one per wave).
__host__ __device__ inline int class_items(int mode, int ncells) {
    return mode == kBig ? ncells : (ncells + kWaves - 1) / kWaves;
}

// Run `make(team)` over the batch-rule items of this launch assigned to this workgroup.
template <typename T, int MODE, typename Make>
__device__ __forceinline__ void for_items(const SkBatch& p, lds_p<char> base, double* big_scratch,
                                          int* ctrl, Make&& make) {
    const int nitems = class_items(MODE, p.q_hi - p.q_lo);
    for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
        if constexpr (MODE == kBig) {
            const BlockTeam tm;
            with_cell<T, true>(tm, p, base, p.lw1, p.lw2, p.order[p.q_lo + q], big_scratch, ctrl,
                               make(tm));
        } else {
            const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
            const lds_p<char> slice =
                base + w * lds_layout_bytes(p.xside, p.lw1, p.lw2, sizeof(T));
            const int k = p.q_lo + q * kWaves + w;
            if (k < p.q_hi) {
                const WaveTeam tm;
                with_cell<T, false>(tm, p, slice, p.lw1, p.lw2, p.order[k], big_scratch, ctrl,
                                    make(tm));
            }
        }
        __syncthreads();
    }
}

// One batch-rule iteration of one launch.  The workgroups of all the launches of an iteration
// take one ticket each; the last of all (`nblocks` in total) reduces the per-cell errors in
// fixed cell order and sets the stop flag.
template <typename T, int MODE>
__global__ void __launch_bounds__(MODE == kBig ? kBigThreads : kThreads)
    sk_iter_kernel(SkBatch p, double* fa, double* fb, int limit, double tol, int nblocks,
                   int* ctrl, double* cell_err, double* cell_mass, double* dtot,
                   double* big_scratch) {
    if (__atomic_load_n(&ctrl[2], __ATOMIC_RELAXED) != 0) return;
    // the iteration number lives on the device (every launch is identical, so a chunk of
    // launches can be captured once and replayed); odd iterations read fa and write fb
    const int it = __atomic_load_n(&ctrl[10], __ATOMIC_RELAXED) + 1;
    const double* f_in = (it & 1) ? fa : fb;
    double* f_out = (it & 1) ? fb : fa;
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_last;
    __shared__ double s_red[16];
    for_items<T, MODE>(p, (lds_p<char>)smem, big_scratch, ctrl, [&](const auto& tm) {
        using Tm = std::decay_t<decltype(tm)>;
        return IterCell<Tm, T>{tm, p, f_in, f_out, cell_err, cell_mass};
    });
    __threadfence();
    if (threadIdx.x == 0) s_last = (atomicAdd(&ctrl[1], 1) == nblocks - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // by the first kThreads threads whatever the workgroup size, so that the sum (and the
    // stop) does not depend on which class's workgroup comes last (the others add zeros)
    double e = 0.0, m = 0.0;
    for (int c = threadIdx.x; threadIdx.x < kThreads && c < p.ncells; c += kThreads) {
        e += cell_err[c];
        m += cell_mass[c];
    }
    e = block_sum(e, s_red);
    m = block_sum(m, s_red);
    if (threadIdx.x == 0) {
        dtot[0] = e;
        dtot[1] = m;
        const bool conv = e <= tol * m;
        if (conv) ctrl[4] = 1;
        if (conv || it >= limit || !(e == e)) __atomic_store_n(&ctrl[2], it, __ATOMIC_RELAXED);
        ctrl[10] = it;
        ctrl[1] = 0;
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(MODE == kBig ? kBigThreads : kThreads) sk_final_kernel(SkBatch p, int* ctrl,
                                                           int32_t* iters_out,
                                                           double* big_scratch) {
    extern __shared__ __align__(16) char smem[];
    const int done = ctrl[2];
    for_items<T, MODE>(p, (lds_p<char>)smem, big_scratch, ctrl, [&](const auto& tm) {
        using Tm = std::decay_t<decltype(tm)>;
        return FinalCell<Tm, T>{tm, p, done, iters_out};
    });
}

// Batch statistics: sums of err, mass, iterations, terms and algorithmic bytes; min/max
// iterations; whether every cell met its per-cell tolerance.  One workgroup.
__global__ void __launch_bounds__(kThreads)
    sk_stats_kernel(int ncells, const int32_t* iters, const int32_t* iters64, const double* err,
                    const double* mass, double tol, const int32_t* dims, int xside, double* dtot,
                    int* ictl) {
    __shared__ double red[8];
    __shared__ int smin[kWaves], smax[kWaves], sconv[kWaves], spol[kWaves];
    double e = 0.0, m = 0.0, work = 0.0, bytes = 0.0, terms = 0.0;
    int imin = 0x7fffffff, imax = 0, allconv = 1, pmax = 0;
    for (int c = threadIdx.x; c < ncells; c += blockDim.x) {
        const int it = iters[c];
        if (iters64) pmax = max(pmax, iters64[c]);
        e += err[c];
        m += mass[c];
        work += it;
        const double W1 = dims[2 * c], W2 = dims[2 * c + 1];
        const double A = xside;
        terms += it * (A * W2 * (A + W1) + A * W1 * (W2 + A));
        bytes += it * 12.0 * (A * A + W1 * W2);
        imin = min(imin, it);
        imax = max(imax, it);
        if (!(err[c] <= tol * mass[c])) allconv = 0;
    }
    e = block_sum(e, red);
    m = block_sum(m, red);
    work = block_sum(work, red);
    terms = block_sum(terms, red);
    bytes = block_sum(bytes, red);
    const int w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
    imin = wave_min_i(imin);
    imax = wave_max_i(imax);
    allconv = wave_min_i(allconv);
    pmax = wave_max_i(pmax);
    if ((threadIdx.x & 63) == 0) {
        smin[w] = imin;
        smax[w] = imax;
        sconv[w] = allconv;
        spol[w] = pmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < nw; ++k) {
            imin = min(imin, smin[k]);
            imax = max(imax, smax[k]);
            allconv = min(allconv, sconv[k]);
            pmax = max(pmax, spol[k]);
        }
        ictl[8] = pmax;
        dtot[0] = e;
        dtot[1] = m;
        dtot[2] = work;
        dtot[3] = terms;
        dtot[4] = bytes;
        ictl[5] = ncells > 0 ? imin : 0;
        ictl[6] = imax;
        ictl[7] = allconv;
    }
}

// After a float64 finish, per-cell iterations count both phases.  When the finish starts with
// a Y-update of the X potential the float32 phase stopped at (`shared`), it repeats that
// phase's last Y-update in float64 and the two phases share one iteration; from the X-update
// that followed (the register-blocked path) the finish's iterations come on top.
__global__ void merge_iters_kernel(int ncells, int32_t* iters, const int32_t* iters64, int shared) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncells && iters64[c] > 0) iters[c] += iters64[c] - shared;
}

__global__ void done_iters_kernel(int ncells, int32_t* iters, const int* ctrl) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncells) iters[c] = ctrl[2];
}

}  // namespace

void launch_done_iters(int ncells, int32_t* iters, const int* ctrl, hipStream_t st) {
    if (ncells > 0)
        done_iters_kernel<<<(ncells + kThreads - 1) / kThreads, kThreads, 0, st>>>(ncells, iters,
                                                                                  ctrl);
}

size_t sk_lds_bytes(int xside, int prec) {
    if (xside < 2 || xside > 16) return 0;
    const size_t e = prec == DD_PREC_F64 ? sizeof(double) : sizeof(float);
    return lds_layout_bytes(xside, 0, 0, e);
}

Status sk_work_reserve(SkWork& w, int ncells, size_t a_n) {
    Status st;
    if (w.arena) {
        // no-allocation mode: carve the per-solve buffers from the start of the arena
        w.arena_used = 0;
        if ((st = arena_take(w, w.ctrl, 16)).code || (st = arena_take(w, w.dtot, 8)).code ||
            (st = arena_take(w, w.cell_err, (size_t)ncells)).code ||
            (st = arena_take(w, w.cell_mass, (size_t)ncells)).code ||
            (st = arena_take(w, w.cell_iters, (size_t)ncells)).code ||
            (st = arena_take(w, w.iters64, (size_t)ncells)).code ||
            (st = arena_take(w, w.a_alt, a_n)).code)
            return st;
        w.cap = ncells;
        w.a_alt_n = a_n;
        return st;
    }
    if (!w.ctrl) {
        DD_HIP(w.mem.get(&w.ctrl, 16 * sizeof(int)), st);
        DD_HIP(w.mem.get(&w.ctrl64, 16 * sizeof(int)), st);
        DD_HIP(hipHostMalloc((void**)&w.h_ctl32, 16 * sizeof(int)), st);
        DD_HIP(w.mem.get(&w.dtot, 8 * sizeof(double)), st);
        DD_HIP(hipEventCreate(&w.ev0), st);
        DD_HIP(hipEventCreate(&w.ev1), st);
        DD_HIP(hipEventCreate(&w.ev2), st);
        DD_HIP(hipEventCreateWithFlags(&w.evj, hipEventDisableTiming), st);
        DD_HIP(hipEventCreateWithFlags(&w.evf, hipEventDisableTiming), st);
        DD_HIP(hipEventCreateWithFlags(&w.evj2, hipEventDisableTiming), st);
        DD_HIP(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking), st);
        DD_HIP(hipStreamCreateWithFlags(&w.stream2, hipStreamNonBlocking), st);
        DD_HIP(hipStreamCreateWithFlags(&w.stream3, hipStreamNonBlocking), st);
        DD_HIP(hipEventCreateWithFlags(&w.evj3, hipEventDisableTiming), st);
    }
    if (ncells > w.cap) {
        w.mem.put(w.cell_err);
        w.mem.put(w.cell_mass);
        w.mem.put(w.cell_iters);
        w.cell_err = nullptr;
        w.cell_mass = nullptr;
        w.cell_iters = nullptr;
        const int cap = std::max(ncells, 1024);
        DD_HIP(w.mem.get(&w.cell_err, cap * sizeof(double)), st);
        DD_HIP(w.mem.get(&w.cell_mass, cap * sizeof(double)), st);
        DD_HIP(w.mem.get(&w.cell_iters, cap * sizeof(int32_t)), st);
        w.mem.put(w.iters64);
        w.iters64 = nullptr;
        DD_HIP(w.mem.get(&w.iters64, cap * sizeof(int32_t)), st);
        w.cap = cap;
    }
    if (a_n > w.a_alt_n) {
        w.mem.put(w.a_alt);
        w.a_alt = nullptr;
        DD_HIP(w.mem.get(&w.a_alt, a_n * sizeof(double)), st);
        w.a_alt_n = a_n;
    }
    return st;
}

void sk_work_release(SkWork& w) {
    if (w.arena) return;  // no-allocation mode: nothing of its own to release
    w.mem.put(w.order);
    w.mem.put(w.scr_off);
    w.mem.put(w.recs);
    if (w.h_stage) (void)hipHostFree(w.h_stage);
    if (w.h_ctl) (void)hipHostFree(w.h_ctl);
    if (w.h_ctl32) (void)hipHostFree(w.h_ctl32);
    w.mem.put(w.ctrl64);
    if (w.h_tot) (void)hipHostFree(w.h_tot);
    w.mem.put(w.order64);
    w.mem.put(w.scr_off64);
    w.mem.put(w.big);
    w.mem.put(w.iters64);
    w.mem.put(w.a_alt);
    w.mem.put(w.cell_err);
    w.mem.put(w.cell_mass);
    w.mem.put(w.cell_iters);
    w.mem.put(w.ctrl);
    w.mem.put(w.dtot);
    if (w.ev0) (void)hipEventDestroy(w.ev0);
    if (w.ev1) (void)hipEventDestroy(w.ev1);
    if (w.ev2) (void)hipEventDestroy(w.ev2);
    if (w.evj) (void)hipEventDestroy(w.evj);
    if (w.evf) (void)hipEventDestroy(w.evf);
    if (w.evj2) (void)hipEventDestroy(w.evj2);
    if (w.evj3) (void)hipEventDestroy(w.evj3);
    for (auto& a : w.kev)
        for (auto& b : a)
            for (hipEvent_t& e : b)
                if (e) (void)hipEventDestroy(e);
    for (hipStream_t* sp : {&w.stream, &w.stream2, &w.stream3})
        if (*sp) {
            (void)hipStreamSynchronize(*sp);
            (void)hipStreamDestroy(*sp);
        }
    const Mem m = w.mem;
    w = SkWork{};
    w.mem = m;
}

namespace {
int g_num_cus = 0;
int num_cus() {
    if (!g_num_cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&g_num_cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess)
            g_num_cus = 256;
    }
    return g_num_cus;
}

template <typename K>
Status set_lds_attr(K kernel, size_t bytes, Status& st) {
    DD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
           st);
    return st;
}

template <typename K>
int grid_for(K kernel, size_t lds, int items, int threads = kThreads) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel),
                                                     threads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const long g = (long)per_cu * num_cus();
    return (int)std::max(1L, std::min<long>(g, items));
}

// A class of cells for one launch: order[lo, hi), solved one per workgroup (kBig) or one per
// wave (kSmall), with LDS tiles for float32 and float64 terms.
struct CellClass {
    int mode = kBig;
    int lo = 0, hi = 0;
    int t[2] = {0, 0};  // LDS tile (W1, W2)
    size_t budget = 0;
    int threads = kThreads;  // workgroup size (MODE kBig: up to kBigThreads)
};

// first_chunk: iterations launched before the first read of the stop flag (batch rule; 0: a
// whole chunk of check_every).  Batch rule only: `ctl` is the control block (default w.ctrl);
// phase kRunSpec launches the first iterations without reading the stop flag (the caller has
// cleared `ctl`, or marked it done so that they exit at once), then picks the output buffer
// and the per-cell counts on the device; kRunResume continues such a run from the stop-flag
// read (the state on the device is that of a run at the same point).
constexpr int kRunAll = 0, kRunSpec = 1, kRunResume = 2;

__global__ void pick_final_kernel(int64_t n, double* a, const double* alt, const int* ctrl) {
    // the last X-update of a batch-rule run that stopped at iteration `done` is in `alt`
    // when done is even (odd iterations read a and write alt)
    const int done = __atomic_load_n(&ctrl[2], __ATOMIC_RELAXED);
    if (done <= 0 || ((done - 1) & 1) == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = alt[i];
}

template <typename T>
Status run_solver(const SkBatch& p0, const std::vector<CellClass>& cls, const dd_sinkhorn_opts& o,
                  hipStream_t st, SkWork& w, int32_t* iters, double* errs, int first_chunk = 0,
                  int* done_out = nullptr, int* ctl = nullptr, int phase = kRunAll) {
    Status S;
    if (!ctl) ctl = w.ctrl;
    double* big = reinterpret_cast<double*>(w.big);
    // the small and giant classes run on `st`, the big class on the second stream, side by side
    const bool one_stream = w.arena != nullptr;  // no-allocation mode: the caller's stream only
    const hipStream_t streams[3] = {st, one_stream ? st : w.stream2, st};
    hipEvent_t joins[3] = {nullptr, w.evj2, nullptr};
    const int qidx[3] = {0, 9, 11};
    const int ncls = (int)cls.size();
    std::vector<SkBatch> pk(ncls, p0);
    std::vector<size_t> lds(ncls);
    for (int k = 0; k < ncls; ++k) {
        pk[k].q_lo = cls[k].lo;
        pk[k].q_hi = cls[k].hi;
        pk[k].lw1 = cls[k].t[0];
        pk[k].lw2 = cls[k].t[1];
        const size_t one = lds_layout_bytes(p0.xside, pk[k].lw1, pk[k].lw2, sizeof(T));
        lds[k] = cls[k].mode == kBig ? one : kWaves * one;
    }
    // classes on the second stream are forked from `st` and joined back
    auto fork = [&]() {
        if (ncls < 2 || one_stream) return;
        (void)hipEventRecord(w.evf, st);
        (void)hipStreamWaitEvent(streams[1], w.evf, 0);
    };
    auto join = [&]() {
        if (ncls < 2 || one_stream) return;
        (void)hipEventRecord(joins[1], streams[1]);
        (void)hipStreamWaitEvent(st, joins[1], 0);
    };
    const bool fixed = o.fixed_iters > 0;
    if (phase == kRunAll) zero_ints<<<1, 64, 0, st>>>(ctl, 12);
    if (fixed || o.stop_rule == DD_STOP_CELL) {
        const int limit = fixed ? o.fixed_iters : o.max_iter;
        // stall detection only where a float64 finish follows
        const int stall = sizeof(T) == sizeof(float) ? 32 : 0;
        fork();
        for (int k = 0; k < ncls; ++k) {
            const int n = cls[k].hi - cls[k].lo;
            auto kern = cls[k].mode == kBig ? sk_cell_kernel<T, kBig> : sk_cell_kernel<T, kSmall>;
            if (set_lds_attr(kern, lds[k], S).code) return S;
            kern<<<grid_for(kern, lds[k], class_items(cls[k].mode, n), cls[k].threads),
                   cls[k].threads, lds[k], streams[k]>>>(pk[k], o.tol, limit, fixed ? 1 : 0, stall, ctl + qidx[k],
                                 ctl, iters, errs, w.cell_mass, big);
        }
        join();
        DD_HIP(hipGetLastError(), S);
        return S;
    }
    std::vector<int> grid(ncls);
    int nblocks = 0;
    for (int k = 0; k < ncls; ++k) {
        const int n = cls[k].hi - cls[k].lo;
        auto ik = cls[k].mode == kBig ? sk_iter_kernel<T, kBig> : sk_iter_kernel<T, kSmall>;
        auto fk = cls[k].mode == kBig ? sk_final_kernel<T, kBig> : sk_final_kernel<T, kSmall>;
        if (set_lds_attr(ik, lds[k], S).code || set_lds_attr(fk, lds[k], S).code) return S;
        grid[k] = grid_for(ik, lds[k], class_items(cls[k].mode, n), cls[k].threads);
        nblocks += grid[k];
    }
    double* bufs[2] = {p0.a, w.a_alt};
    const size_t a_bytes = (size_t)p0.ncells * p0.xside * p0.xside * sizeof(double);
    const int chunk = o.check_every > 0 ? o.check_every : 8;
    // a chunk of identical iterations (every class's launch, forked and joined) is captured
    // into a HIP graph once and replayed; the host reads the device stop flag between replays
    // (in no-allocation mode the chunk is launched directly, no graph is built)
    auto chunk_launches = [&]() {
        for (int r = 0; r < chunk; ++r) {
            fork();
            for (int k = 0; k < ncls; ++k) {
                auto ik = cls[k].mode == kBig ? sk_iter_kernel<T, kBig> : sk_iter_kernel<T, kSmall>;
                ik<<<grid[k], cls[k].threads, lds[k], streams[k]>>>(pk[k], bufs[0], bufs[1], o.max_iter,
                                                              o.tol, nblocks, ctl, errs,
                                                              w.cell_mass, w.dtot, big);
            }
            join();
        }
    };
    // The first `first_chunk` launches go out directly (a float64 finish usually stops in its
    // first iteration, so it pays for no capture); if the rule has not stopped by then, a chunk
    // of `chunk` launches is captured once and replayed.
    int done = 0, launched = 0;
    auto read_done = [&]() {
        ++w.waits;
        return hipMemcpyAsync(&done, ctl + 2, sizeof(int), hipMemcpyDeviceToHost, st) ==
                   hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    // (a speculative run and its resumption take first_chunk as it is, 0 included)
    const int first = phase != kRunAll
                          ? std::max(0, std::min(first_chunk, o.max_iter))
                          : std::max(1, std::min(first_chunk > 0 ? first_chunk : chunk, o.max_iter));
    for (int r = 0; phase != kRunResume && r < first; ++r) {
        fork();
        for (int k = 0; k < ncls; ++k) {
            auto ik = cls[k].mode == kBig ? sk_iter_kernel<T, kBig> : sk_iter_kernel<T, kSmall>;
            ik<<<grid[k], cls[k].threads, lds[k], streams[k]>>>(pk[k], bufs[0], bufs[1], o.max_iter,
                                                          o.tol, nblocks, ctl, errs,
                                                          w.cell_mass, w.dtot, big);
        }
        join();
    }
    launched = first;
    if (phase == kRunSpec) {
        const int64_t na = (int64_t)p0.ncells * p0.xside * p0.xside;
        pick_final_kernel<<<(int)std::min<int64_t>((na + 255) / 256, 1024), 256, 0, st>>>(
            na, p0.a, bufs[1], ctl);
        launch_done_iters(p0.ncells, iters, ctl, st);
        DD_HIP(hipGetLastError(), S);
        return S;
    }
    if (!read_done()) {
        S.code = DD_EDEVICE;
        S.msg = "sinkhorn: reading the stop flag failed";
        return S;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (!done && launched < o.max_iter && !one_stream) {
        DD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), S);
        chunk_launches();
        const hipError_t ce = hipStreamEndCapture(st, &graph);
        if (ce != hipSuccess ||
            hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            S.code = DD_EDEVICE;
            S.msg = "sinkhorn: HIP graph capture of the iteration failed";
            return S;
        }
    }
    for (; launched < o.max_iter && !done; launched += chunk) {
        if (one_stream)
            chunk_launches();
        if ((!one_stream && hipGraphLaunch(exec, st) != hipSuccess) || !read_done()) {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            S.code = DD_EDEVICE;
            S.msg = "sinkhorn: graph replay failed";
            return S;
        }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (done < 1) done = o.max_iter;  // unreachable: the kernel sets done at max_iter
    if (((done - 1) & 1) == 1)
        DD_HIP(hipMemcpyAsync(p0.a, bufs[1], a_bytes, hipMemcpyDeviceToDevice, st), S);
    // g of the stopping iteration is already in p.b (every Y-update writes it, and no
    // iteration runs after the stop); each cell's count is the stop iteration
    launch_done_iters(p0.ncells, iters, ctl, st);
    if (done_out) *done_out = done;
    DD_HIP(hipGetLastError(), S);
    return S;
}

// LDS tile for the Y-box arrays of one class of cells: the largest bounds within the byte
// budget, taken from per-axis quantiles of the class's box dims so that most of its cells
// stay LDS-resident.
void plan_tile(const std::vector<int32_t>& hd, const std::vector<int32_t>& cells, int xside,
               size_t elem, size_t budget, int& lw1, int& lw2) {
    lw1 = lw2 = 0;
    const int n = (int)cells.size();
    if (n == 0) return;
    auto fits = [&](int a, int b) { return lds_layout_bytes(xside, a, b, elem) <= budget; };
    // per-axis order statistics of the box dims from histograms (dims are small integers)
    int m1 = 1, m2 = 1;
    for (int c : cells) {
        m1 = std::max(m1, hd[2 * c]);
        m2 = std::max(m2, hd[2 * c + 1]);
    }
    std::vector<int> h1(m1 + 1, 0), h2(m2 + 1, 0);
    for (int c : cells) {
        ++h1[std::max(hd[2 * c], 0)];
        ++h2[std::max(hd[2 * c + 1], 0)];
    }
    auto kth = [](const std::vector<int>& h, int k) {  // the k-th smallest (0-based)
        int acc = 0;
        for (int v = 0; v < (int)h.size(); ++v)
            if ((acc += h[v]) > k) return v;
        return (int)h.size() - 1;
    };
    if (fits(kth(h1, n - 1), kth(h2, n - 1))) {
        lw1 = kth(h1, n - 1);
        lw2 = kth(h2, n - 1);
        return;
    }
    for (double q : {0.99, 0.97, 0.95, 0.9, 0.85, 0.8, 0.7, 0.6, 0.5, 0.3, 0.1}) {
        const int k = std::min(n - 1, (int)(q * n));
        const int a = kth(h1, k), b = kth(h2, k);
        if (fits(a, b)) {
            lw1 = a;
            lw2 = b;
            return;
        }
    }
}

constexpr size_t kBudgets[] = {52 * 1024, 78 * 1024};  // small and big launches
constexpr size_t kBigBudget = 156 * 1024;

// The launch plan of one precision: processing order (giant, big, small classes, most work
// first within each), the classes with their LDS tiles, and the global scratch offsets of the
// boxes beyond the giant tile.
//   small: LSE work per iteration below 64K terms and a box within the small tile (per-wave
//          budget), one cell per wave;
//   big:   the rest within the big tile, one cell per workgroup;
//   giant: boxes beyond the big tile, one per workgroup with the whole LDS of a CU.
struct Plan {
    std::vector<int32_t> ord;
    std::vector<CellClass> classes;
    std::vector<int64_t> off;
    int64_t scr = 0;
    int n_big = 0, n_giant = 0;
    int small_tile[2] = {0, 0}, big_tile[2] = {0, 0};
};

// `ord`: the cells in order of decreasing LSE work per iteration (ties by index).
Plan plan_classes(const std::vector<int32_t>& hd, const std::vector<int32_t>& ord, int ncells,
                  int AS, size_t elem, size_t small_budget, size_t big_budget) {
    Plan P;
    auto work = [&](int c) {
        return sk_cell_terms(AS, std::max(hd[2 * c], 0), std::max(hd[2 * c + 1], 0));
    };
    auto fits = [&](int c, const int* t) { return hd[2 * c] <= t[0] && hd[2 * c + 1] <= t[1]; };
    const double small_terms = 64.0 * 1024.0;
    std::vector<int32_t> cand, rest, small_cells, big_cells, giant_cells;
    std::vector<uint8_t> to_rest(ncells, 0);
    for (int c : ord) {
        if (work(c) < small_terms)
            cand.push_back(c);
        else
            to_rest[c] = 1;
    }
    CellClass sc, bc, gc;
    sc.mode = kSmall;
    sc.budget = small_budget;
    plan_tile(hd, cand, AS, elem, small_budget / kWaves, sc.t[0], sc.t[1]);
    for (int c : cand) {
        if (fits(c, sc.t))
            small_cells.push_back(c);
        else
            to_rest[c] = 1;
    }
    // the rest in the same order (most work first)
    for (int c : ord)
        if (to_rest[c]) rest.push_back(c);
    bc.budget = big_budget;
    plan_tile(hd, rest, AS, elem, big_budget, bc.t[0], bc.t[1]);
    for (int c : rest) (fits(c, bc.t) ? big_cells : giant_cells).push_back(c);
    gc.budget = kBigBudget;
    // the largest boxes, one workgroup per CU by their LDS: twice the threads per cell (the
    // same results, see kBig)
    gc.threads = kBigThreads;
    plan_tile(hd, giant_cells, AS, elem, kBigBudget, gc.t[0], gc.t[1]);
    P.ord = giant_cells;
    P.ord.insert(P.ord.end(), big_cells.begin(), big_cells.end());
    P.ord.insert(P.ord.end(), small_cells.begin(), small_cells.end());
    gc.lo = 0;
    gc.hi = (int)giant_cells.size();
    bc.lo = gc.hi;
    bc.hi = bc.lo + (int)big_cells.size();
    sc.lo = bc.hi;
    sc.hi = ncells;
    if (sc.hi > sc.lo) P.classes.push_back(sc);
    if (bc.hi > bc.lo) P.classes.push_back(bc);
    if (gc.hi > gc.lo) P.classes.push_back(gc);
    P.off.assign(ncells, 0);
    for (int c : giant_cells) {
        const int W1 = hd[2 * c], W2 = hd[2 * c + 1];
        if (W1 < 1 || W2 < 1 || fits(c, gc.t)) continue;
        P.off[c] = P.scr;
        P.scr += cell_scratch_doubles(AS, W1, W2, elem);
    }
    P.n_big = (int)(big_cells.size() + giant_cells.size());
    P.n_giant = (int)giant_cells.size();
    P.small_tile[0] = sc.t[0];
    P.small_tile[1] = sc.t[1];
    P.big_tile[0] = bc.t[0];
    P.big_tile[1] = bc.t[1];
    return P;
}

// Online tuner of the LDS budget per workgroup of the small-cell launch (occupancy against
// LDS-resident boxes):
// each key (block side, precision, stop rule, box-size class) tries every candidate once on
// consecutive solves, then keeps the one with the least Sinkhorn time per LSE term.
constexpr int kNumBudgets = sizeof(kBudgets) / sizeof(kBudgets[0]);

struct TuneKey {
    int as, prec, rule, bucket;
    bool operator<(const TuneKey& o) const {
        if (as != o.as) return as < o.as;
        if (prec != o.prec) return prec < o.prec;
        if (rule != o.rule) return rule < o.rule;
        return bucket < o.bucket;
    }
};

// A choice is (small budget, big budget): choice % kNumBudgets, choice / kNumBudgets.
constexpr int kNumChoices = kNumBudgets * kNumBudgets;

class Tuner {
   public:
    int pick(const TuneKey& k) {
        std::lock_guard<std::mutex> g(mu_);
        Entry& e = tab_[k];
        if (forced_ >= 0) return forced_;
        for (int c = 0; c < kNumChoices; ++c)
            if (e.n[c] == 0) return c;
        int best = 0;
        for (int c = 1; c < kNumChoices; ++c)
            if (e.t[c] < e.t[best]) best = c;
        return best;
    }
    void record(const TuneKey& k, int c, double t) {
        std::lock_guard<std::mutex> g(mu_);
        Entry& e = tab_[k];
        e.t[c] = e.n[c] ? std::min(e.t[c], t) : t;
        e.n[c] += 1;
    }
    void force(int c) { forced_ = c; }

   private:
    struct Entry {
        double t[kNumChoices] = {};
        int n[kNumChoices] = {};
    };
    std::mutex mu_;
    std::map<TuneKey, Entry> tab_;
    int forced_ = -1;
};

Tuner& tuner() {
    static Tuner t;
    return t;
}
}  // namespace

namespace {
// Runs the solve on the library's own stream, ordered after the caller's stream on entry
// and before it on exit (a stream of our own can be captured into graphs whatever stream
// the caller uses).
struct StreamJoin {
    hipStream_t caller, own;
    hipEvent_t ev;
    StreamJoin(hipStream_t c, hipStream_t o, hipEvent_t e) : caller(c), own(o), ev(e) {
        if (!ev) return;  // no-allocation mode: the caller's stream is used directly
        (void)hipEventRecord(ev, caller);
        (void)hipStreamWaitEvent(own, ev, 0);
    }
    ~StreamJoin() {
        if (!ev) return;
        (void)hipEventRecord(ev, own);
        (void)hipStreamWaitEvent(caller, ev, 0);
    }
};
}  // namespace

Status finish_stats(SkWork& w, const int* hctl, const double* htot, dd_batch_stats* stats);

template <typename Work>
std::vector<int32_t> work_order(int n, Work&& work) {
    std::vector<uint32_t> key(n), key2(n);
    std::vector<int32_t> ord(n), ord2(n);
    for (int c = 0; c < n; ++c) {
        key[c] = 4294967295u - (uint32_t)std::min(work(c), 4294967295.0);
        ord[c] = c;
    }
    for (int shift = 0; shift < 32; shift += 8) {
        int cnt[257] = {};
        for (int k = 0; k < n; ++k) ++cnt[((key[k] >> shift) & 255u) + 1];
        if (cnt[((key[0] >> shift) & 255u) + 1] == n) continue;  // one digit: nothing moves
        for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
        for (int k = 0; k < n; ++k) {
            const int d = cnt[(key[k] >> shift) & 255u]++;
            key2[d] = key[k];
            ord2[d] = ord[k];
        }
        key.swap(key2);
        ord.swap(ord2);
    }
    return ord;
}

// the register-blocked path's part of the pending statistics
void set_fast_pend(SkWork::Pend& pd, const FastInfo& fi) {
    pd.terms32 = 0.0;
    for (int k = 0; k < kClasses; ++k) {
        pd.n[k] = fi.n[k];
        pd.lds[k] = fi.lds[k];
        pd.launches[k] = fi.launches[k];
        pd.ms[k] = fi.ms[k];
        pd.terms[k] = fi.terms[k];
        pd.terms32 += fi.terms[k];
    }
}

// Speculative solves (DD_SPEC=0 in the environment switches them off, for A/B timing and
// the tests that compare both; read on every solve).
bool spec_enabled() {
    const char* e = std::getenv("DD_SPEC");
    return !(e && e[0] == '0');
}

// float32 rounds a speculative solve of a batch of n cells enqueues: one more than the last
// such solve needed (from its iteration count: the first two rounds run 4 check_every
// iterations each), between 2 and the kSpecRounds the bound assumes; 4 for an unseen size
int spec_rounds_for(const SkWork& w, int n) {
    for (int k = 0; k < 4; ++k)
        if (w.spec_n[k] == n) return w.spec_r[k];
    return 4;
}

void spec_rounds_learn(SkWork& w, int n, int it32, int chunk, bool resumed) {
    const int used = resumed ? 4 : it32 <= 4 * chunk ? 1 : it32 <= 8 * chunk ? 2 : 4;
    const int r = std::min(4, std::max(2, used + 1));
    int slot = 0;
    for (int k = 0; k < 4; ++k)
        if (w.spec_n[k] == n || w.spec_n[k] == 0) {
            slot = k;
            break;
        } else if (k == 3) {
            slot = (w.spec_next++) & 3;
        }
    w.spec_n[slot] = n;
    w.spec_r[slot] = r;
}

// float64-finish iterations launched speculatively: 2, or DD_SPEC_FINISH in [0, 8] (0 makes
// every speculative solve resume its finish: the tests' way to reach that path)
int spec_finish_launches() {
    const char* e = std::getenv("DD_SPEC_FINISH");
    if (!e || !*e) return 2;
    return std::max(0, std::min(8, std::atoi(e)));
}

// Between the speculative float32 rounds and the float64 finish: the finish's control block
// is cleared when the rounds stopped short of the cap, else marked done (-1), so that the
// finish's launches exit at once and the caller resumes the rounds.
__global__ void spec_gate_kernel(const int* c32, int* c64, int max_iter) {
    const int stop = __atomic_load_n(&c32[2], __ATOMIC_RELAXED);
    const int t = threadIdx.x;
    if (t < 16) c64[t] = (t == 2 && !(stop > 0 && stop < max_iter)) ? -1 : 0;
}

Status sk_solve(const SkBatch& p, const dd_sinkhorn_opts& o, hipStream_t caller_st, SkWork& w,
                dd_batch_stats* stats, int32_t* cell_iters_out, double* cell_err_out,
                const int32_t* host_dims, bool defer, bool spec) {
    Status S;
    w.pend.active = false;
    if (p.ncells < 0 || p.xside < 2 || p.xside > 16 || !(p.kappa > 0.0) || p.max_w1 < 1 ||
        p.max_w2 < 1 || (p.prec != DD_PREC_F32 && p.prec != DD_PREC_F64)) {
        S.code = DD_EINVAL;
        S.msg = "sinkhorn: bad batch (ncells, xside in [2,16], kappa > 0, max_w >= 1)";
        return S;
    }
    if (o.max_iter < 1 || o.fixed_iters < 0 ||
        (o.stop_rule != DD_STOP_BATCH && o.stop_rule != DD_STOP_CELL) || !(o.tol >= 0.0) ||
        o.check_every < 0) {
        S.code = DD_EINVAL;
        S.msg = "sinkhorn: bad options (max_iter >= 1, fixed_iters >= 0, stop_rule, tol >= 0)";
        return S;
    }
    S = sk_work_reserve(w, p.ncells, (size_t)p.ncells * p.xside * p.xside);
    if (S.code) return S;
    const bool arena = w.arena != nullptr;
    const StreamJoin join(caller_st, arena ? caller_st : w.stream, arena ? nullptr : w.evj);
    const hipStream_t st = arena ? caller_st : w.stream;
    int32_t* iters = cell_iters_out ? cell_iters_out : w.cell_iters;
    double* errs = cell_err_out ? cell_err_out : w.cell_err;
    if (p.ncells == 0) {
        if (stats) {
            *stats = dd_batch_stats{};
            stats->converged = 1;
        }
        return S;
    }
    // plan on the host from the box dims: processing order (most LSE work first), the split
    // into big (workgroup) and small (wave) cells, an LDS tile per class, and global scratch
    // for the boxes beyond their tile
    std::vector<int32_t> hd(2 * (size_t)p.ncells);
    if (host_dims) {
        std::copy(host_dims, host_dims + hd.size(), hd.begin());
    } else {
        DD_HIP(hipMemcpyAsync(hd.data(), p.dims, hd.size() * 4, hipMemcpyDeviceToHost, st), S);
        DD_HIP(hipStreamSynchronize(st), S);
        ++w.waits;
    }
    // pinned staging of the launch plans and the statistics (outside no-allocation mode):
    // [order64 | off64 | order | off | fast order], 8-byte aligned
    const bool pinned = !arena;
    if (defer && !pinned) {
        S.code = DD_EINVAL;
        S.msg = "sinkhorn: deferred statistics need the allocating entry points";
        return S;
    }
    const size_t nn = (size_t)p.ncells, o4 = (nn * 4 + 7) & ~(size_t)7;
    const size_t stage_need = 3 * o4 + 2 * nn * 8;
    if (pinned) {
        if (!w.h_ctl) DD_HIP(hipHostMalloc((void**)&w.h_ctl, 16 * sizeof(int)), S);
        if (!w.h_tot) DD_HIP(hipHostMalloc((void**)&w.h_tot, 8 * sizeof(double)), S);
        if (stage_need > w.h_stage_cap) {
            if (w.h_stage) (void)hipHostFree(w.h_stage);
            w.h_stage = nullptr;
            w.h_stage_cap = 0;
            const size_t cap = std::max<size_t>(stage_need + stage_need / 4, 1 << 16);
            DD_HIP(hipHostMalloc((void**)&w.h_stage, cap), S);
            w.h_stage_cap = cap;
        }
    }
    auto region = [&](size_t off) { return pinned ? w.h_stage + off : nullptr; };
    int32_t* h_ord64 = (int32_t*)region(0);
    int64_t* h_off64 = (int64_t*)region(o4);
    int32_t* h_ordg = (int32_t*)region(o4 + nn * 8);
    int64_t* h_offg = (int64_t*)region(2 * o4 + nn * 8);
    int32_t* h_ordf = (int32_t*)region(2 * o4 + 2 * nn * 8);
    const int AS = p.xside;
    // a box outside [1, max_w] is rejected before any launch (a and b untouched)
    for (int c = 0; c < p.ncells; ++c)
        if (hd[2 * c] < 1 || hd[2 * c + 1] < 1 || hd[2 * c] > p.max_w1 ||
            hd[2 * c + 1] > p.max_w2) {
            S.code = DD_EINVAL;
            S.msg = "sinkhorn: a cell's Y box is empty or exceeds max_w1/max_w2";
            return S;
        }
    auto work = [&](int c) {
        return sk_cell_terms(AS, std::max(hd[2 * c], 0), std::max(hd[2 * c + 1], 0));
    };
    // cells in order of decreasing LSE work per iteration, ties by index (the work of a cell
    // is an integer below 2^32): a stable least-significant-digit radix sort of the inverted
    // work in four byte passes, from the index order (linear in the cells; a comparison sort
    // of the four thousand cells of a 512^2 partition was most of the host's planning time)
    std::vector<int32_t> ord = work_order(p.ncells, work);
    const size_t elem = p.prec == DD_PREC_F64 ? sizeof(double) : sizeof(float);
    // Launch plans, one per precision (the float64 finish has its own tiles).  The two LDS
    // budgets come from the tuner, keyed by block side, precision, stop rule and the size
    // class of the boxes.  Neither the budgets nor the split change the arithmetic (every
    // output has its own fixed-order sum, and the error reduction is the same for a wave and
    // a workgroup), so every choice gives the same result.
    double area = 0.0;
    for (int c = 0; c < p.ncells; ++c)
        area += (double)std::max(hd[2 * c], 1) * std::max(hd[2 * c + 1], 1);
    const int bucket = (int)std::log2(std::max(1.0, area / p.ncells));
    const TuneKey key{AS, p.prec, o.fixed_iters > 0 ? 2 : o.stop_rule, bucket};
    const int choice = tuner().pick(key);
    const size_t small_budget = kBudgets[choice % kNumBudgets];
    const size_t big_budget = kBudgets[choice / kNumBudgets];
    const bool finish = p.prec == DD_PREC_F32 && o.fixed_iters == 0;
    FastClasses fcls;
    int fchoice = -1, fkey[3] = {0, 0, 0};
    const bool fast = fast_plan(p, hd, o, &fcls, &fchoice, fkey);
    // the general path's plan (not needed when the register-blocked path takes the batch), and
    // the float64 finish's
    const Plan P = fast ? Plan{} : plan_classes(hd, ord, p.ncells, AS, elem, small_budget, big_budget);
    Plan P64;
    auto put = [&](int32_t*& dev_ord, int64_t*& dev_off, int& cap, const Plan& pl,
                   int32_t* h_o, int64_t* h_f) -> Status {
        Status E;
        if (arena) {
            if ((E = arena_take(w, dev_ord, (size_t)p.ncells)).code ||
                (E = arena_take(w, dev_off, (size_t)p.ncells)).code)
                return E;
            cap = p.ncells;
        } else if (p.ncells > cap) {
            w.mem.put(dev_ord);
            w.mem.put(dev_off);
            dev_ord = nullptr;
            dev_off = nullptr;
            cap = std::max(p.ncells, 1024);
            DD_HIP(w.mem.get(&dev_ord, cap * sizeof(int32_t)), E);
            DD_HIP(w.mem.get(&dev_off, cap * sizeof(int64_t)), E);
        }
        const void* so = pl.ord.data();
        const void* sf = pl.off.data();
        if (h_o) {
            std::copy(pl.ord.begin(), pl.ord.end(), h_o);
            std::copy(pl.off.begin(), pl.off.end(), h_f);
            so = h_o;
            sf = h_f;
        }
        DD_HIP(hipMemcpyAsync(dev_ord, so, pl.ord.size() * 4, hipMemcpyHostToDevice, st), E);
        DD_HIP(hipMemcpyAsync(dev_off, sf, pl.off.size() * 8, hipMemcpyHostToDevice, st), E);
        return E;
    };
    // 8 x 8 blocks in float32 take the register-blocked path (same iteration and rules)
    if (!fast) {
        S = put(w.order, w.scr_off, w.order_cap, P, h_ordg, h_offg);
        if (S.code) return S;
    }
    SkBatch q = p;
    q.order = w.order;
    q.scr_off = w.scr_off;
    SkBatch q64 = p;
    // the float64 finish's plan, its upload and the global scratch of both plans; a
    // speculative solve does this after its float32 rounds are enqueued (the device is busy
    // with them meanwhile)
    auto plan_finish = [&]() -> Status {
        Status E;
        if (finish) {
            P64 = plan_classes(hd, ord, p.ncells, AS, sizeof(double), kBudgets[1], kBudgets[1]);
            E = put(w.order64, w.scr_off64, w.order64_cap, P64, h_ord64, h_off64);
            if (E.code) return E;
            q64.order = w.order64;
            q64.scr_off = w.scr_off64;
        }
        const int64_t scr = std::max(P.scr, P64.scr);
        if (arena) {
            double* bigp = nullptr;
            E = arena_take(w, bigp, (size_t)std::max<int64_t>(scr, 0) + 8);
            if (E.code) return E;
            w.big = bigp;
            w.big_bytes = ((size_t)std::max<int64_t>(scr, 0) + 8) * sizeof(double);
        } else if (scr > 0) {
            const size_t need = (size_t)scr * sizeof(double) + 64;
            if (need > w.big_bytes) {
                w.mem.put(w.big);
                w.big = nullptr;
                DD_HIP(w.mem.get(&w.big, need), E);
                w.big_bytes = need;
            }
        }
        return E;
    };
    const int spec_chunk = std::max(1, o.check_every > 0 ? o.check_every : 8);
    const int spec_first64 = spec_finish_launches();
    const bool use_spec = spec && defer && pinned && fast && finish &&
                          o.stop_rule == DD_STOP_BATCH &&
                          o.max_iter >= fast_spec_max_iters(spec_chunk) + spec_first64 + 2 &&
                          spec_enabled();
    if (!use_spec) {
        S = plan_finish();
        if (S.code) return S;
    }
    // without the pinned staging the copies read the plans' own vectors: wait for them
    if (!pinned) {
        DD_HIP(hipStreamSynchronize(st), S);
        ++w.waits;
    }
    if (!arena) DD_HIP(hipEventRecord(w.ev0, st), S);
    zero_ints<<<1, 64, 0, st>>>(w.ctrl, 16);
    FastInfo fi;
    int k32 = 0;  // batch rule: the float32 phase's stop iteration
    // the whole solve enqueued with no host wait (see sk_solve in the header); the float64
    // finish's first two iterations are then launched with the full max_iter as their limit,
    // which stops neither of them when the float32 phase has stopped at least two iterations
    // short of the cap -- what the bound on the speculative rounds' iterations guarantees.
    // The rounds enqueued: one more than the last solve of a batch of this size needed (the
    // rounds after the stop cost a launch each), at most four
    const int spec_rounds = use_spec ? spec_rounds_for(w, p.ncells) : 0;
    if (fast)
        S = fast_solve(p, o, st, w, hd, ord, iters, errs, &fi, !finish, h_ordf, fcls,
                       use_spec ? kFastSpec : kFastAll, spec_rounds);
    else
        S = p.prec == DD_PREC_F32 ? run_solver<float>(q, P.classes, o, st, w, iters, errs, 0, &k32)
                                  : run_solver<double>(q, P.classes, o, st, w, iters, errs);
    if (S.code) return S;
    if (fast) k32 = fi.stop_it;
    if (!arena) DD_HIP(hipEventRecord(w.ev2, st), S);
    // float64 finish: continue the same stopping rule in float64 from the float32 state; the
    // tolerance is then certified by a float64 error (usually after one Y-update).  It starts
    // from the float32 phase's last (f, g) -- its first Y-update repeats that iteration -- or,
    // on the register-blocked path, from the X-update after it (one more iteration); under
    // the batch rule both phases together stay within max_iter.
    const bool shared = !(fast && !fi.final_done);
    dd_sinkhorn_opts o64 = o;
    if (o.stop_rule == DD_STOP_BATCH) o64.max_iter = o.max_iter - k32 + (shared ? 1 : 0);
    const bool run64 = finish && o64.max_iter >= 1;
    if (use_spec) {
        S = plan_finish();
        if (S.code) return S;
        spec_gate_kernel<<<1, 64, 0, st>>>(w.ctrl, w.ctrl64, o.max_iter);
        S = run_solver<double>(q64, P64.classes, o64, st, w, w.iters64, errs, spec_first64,
                               nullptr, w.ctrl64, kRunSpec);
        if (S.code) return S;
    } else if (run64) {
        S = run_solver<double>(q64, P64.classes, o64, st, w, w.iters64, errs, 2);
        if (S.code) return S;
    }
    int* const ctl_stats = use_spec ? w.ctrl64 : w.ctrl;
    // per-cell iterations of both phases, then the statistics over them
    if (run64)
        merge_iters_kernel<<<(p.ncells + kThreads - 1) / kThreads, kThreads, 0, st>>>(
            p.ncells, iters, w.iters64, shared ? 1 : 0);
    sk_stats_kernel<<<1, kThreads, 0, st>>>(p.ncells, iters, run64 ? w.iters64 : nullptr, errs,
                                            w.cell_mass, o.tol, p.dims, p.xside, w.dtot,
                                            ctl_stats);
    if (!arena) DD_HIP(hipEventRecord(w.ev1, st), S);
    auto& pd = w.pend;
    pd = SkWork::Pend{};
    pd.active = true;
    pd.fast = fast;
    pd.run64 = run64;
    pd.ncells = p.ncells;
    pd.fixed_iters = o.fixed_iters;
    pd.stop_rule = o.stop_rule;
    pd.tune = !fast && !arena;
    pd.choice = choice;
    pd.key[0] = key.as;
    pd.key[1] = key.prec;
    pd.key[2] = key.rule;
    pd.key[3] = key.bucket;
    set_fast_pend(pd, fi);
    pd.n_big = P.n_big;
    pd.n_giant = P.n_giant;
    pd.small_tile[0] = P.small_tile[0];
    pd.small_tile[1] = P.small_tile[1];
    pd.big_tile[0] = P.big_tile[0];
    pd.big_tile[1] = P.big_tile[1];
    pd.small_budget = small_budget;
    pd.big_budget = big_budget;
    if (fast) {
        pd.fchoice = arena ? -1 : fchoice;
        for (int k = 0; k < 3; ++k) pd.fkey[k] = fkey[k];
        pd.wave_side = fcls.wave_side;
        pd.big_entries = fcls.big_entries;
    }
    if (use_spec) {
        pd.spec = true;
        pd.spec_slots = fi.spec_slots;
        for (int k = 0; k < kClasses; ++k) pd.tpi[k] = fi.terms_per_it[k];
        // what a resumption needs
        auto& sp = w.spec;
        sp.need_resume = false;
        sp.p = p;
        sp.q64 = q64;
        sp.o = o;
        sp.hd = std::move(hd);
        sp.ord = std::move(ord);
        sp.cls64.clear();
        for (const CellClass& c : P64.classes) {
            const int64_t v[7] = {c.mode, c.lo, c.hi, c.t[0], c.t[1], (int64_t)c.budget,
                                  c.threads};
            sp.cls64.insert(sp.cls64.end(), v, v + 7);
        }
        sp.wave_side = fcls.wave_side;
        sp.big_entries = fcls.big_entries;
        sp.iters = iters;
        sp.errs = errs;
        sp.caller = caller_st;
        sp.first64 = spec_first64;
    }
    if (pinned) {
        DD_HIP(hipMemcpyAsync(w.h_ctl, ctl_stats, 16 * sizeof(int), hipMemcpyDeviceToHost, st), S);
        if (use_spec)
            DD_HIP(hipMemcpyAsync(w.h_ctl32, w.ctrl, 16 * sizeof(int), hipMemcpyDeviceToHost, st),
                   S);
        DD_HIP(hipMemcpyAsync(w.h_tot, w.dtot, 8 * sizeof(double), hipMemcpyDeviceToHost, st), S);
        if (defer) return S;  // the caller synchronises, then sk_finish
        DD_HIP(hipStreamSynchronize(st), S);
        ++w.waits;
        return sk_finish(w, stats);
    }
    int hctl[16];
    double htot[8];
    DD_HIP(hipMemcpyAsync(hctl, w.ctrl, sizeof hctl, hipMemcpyDeviceToHost, st), S);
    DD_HIP(hipMemcpyAsync(htot, w.dtot, sizeof htot, hipMemcpyDeviceToHost, st), S);
    DD_HIP(hipStreamSynchronize(st), S);
    ++w.waits;
    return finish_stats(w, hctl, htot, stats);
}

Status sk_resume(SkWork& w) {
    Status S;
    SkWork::Spec& sp = w.spec;
    SkWork::Pend& pd = w.pend;
    if (!sp.need_resume || !pd.active || !pd.spec) {
        S.code = DD_ESTATE;
        S.msg = "sinkhorn: no speculative solve to resume";
        return S;
    }
    sp.need_resume = false;
    const StreamJoin join(sp.caller, w.stream, w.evj);
    const hipStream_t st = w.stream;
    const dd_sinkhorn_opts& o = sp.o;
    std::vector<CellClass> cls64(sp.cls64.size() / 7);
    for (size_t k = 0; k < cls64.size(); ++k) {
        const int64_t* v = &sp.cls64[7 * k];
        cls64[k].threads = (int)v[6];
        cls64[k].mode = (int)v[0];
        cls64[k].lo = (int)v[1];
        cls64[k].hi = (int)v[2];
        cls64[k].t[0] = (int)v[3];
        cls64[k].t[1] = (int)v[4];
        cls64[k].budget = (size_t)v[5];
    }
    const int stop32 = w.h_ctl32[2];
    dd_sinkhorn_opts o64 = o;
    int* ctl_stats = w.ctrl;
    bool shared = false, run64 = true;
    if (!(stop32 > 0 && stop32 < o.max_iter)) {
        // the float32 rounds had not stopped (or stopped at the cap): continue them, then the
        // float64 finish as a solve without speculation runs it
        FastInfo fi;
        FastClasses fcls;
        fcls.wave_side = sp.wave_side;
        fcls.big_entries = sp.big_entries;
        S = fast_solve(sp.p, o, st, w, sp.hd, sp.ord, sp.iters, sp.errs, &fi, false, nullptr,
                       fcls, kFastResume);
        if (S.code) return S;
        DD_HIP(hipEventRecord(w.ev2, st), S);
        shared = fi.final_done;
        o64.max_iter = o.max_iter - fi.stop_it + (shared ? 1 : 0);
        run64 = o64.max_iter >= 1;
        if (run64) {
            S = run_solver<double>(sp.q64, cls64, o64, st, w, w.iters64, sp.errs, 2);
            if (S.code) return S;
        }
        set_fast_pend(pd, fi);
        pd.spec = false;
    } else {
        // the float32 phase stopped; the float64 finish had not within its first iterations
        o64.max_iter = o.max_iter - stop32;
        S = run_solver<double>(sp.q64, cls64, o64, st, w, w.iters64, sp.errs, sp.first64,
                               nullptr, w.ctrl64, kRunResume);
        if (S.code) return S;
        ctl_stats = w.ctrl64;
    }
    pd.run64 = run64;
    if (run64)
        merge_iters_kernel<<<(sp.p.ncells + kThreads - 1) / kThreads, kThreads, 0, st>>>(
            sp.p.ncells, sp.iters, w.iters64, shared ? 1 : 0);
    sk_stats_kernel<<<1, kThreads, 0, st>>>(sp.p.ncells, sp.iters, run64 ? w.iters64 : nullptr,
                                            sp.errs, w.cell_mass, o.tol, sp.p.dims, sp.p.xside,
                                            w.dtot, ctl_stats);
    DD_HIP(hipEventRecord(w.ev1, st), S);
    DD_HIP(hipMemcpyAsync(w.h_ctl, ctl_stats, 16 * sizeof(int), hipMemcpyDeviceToHost, st), S);
    if (pd.spec)
        DD_HIP(hipMemcpyAsync(w.h_ctl32, w.ctrl, 16 * sizeof(int), hipMemcpyDeviceToHost, st), S);
    DD_HIP(hipMemcpyAsync(w.h_tot, w.dtot, 8 * sizeof(double), hipMemcpyDeviceToHost, st), S);
    DD_HIP(hipGetLastError(), S);
    return S;  // the caller synchronises, then sk_finish
}

Status finish_stats(SkWork& w, const int* hctl, const double* htot, dd_batch_stats* stats) {
    Status S;
    const SkWork::Pend& pd = w.pend;
    w.pend.active = false;
    const bool arena = w.arena != nullptr;
    float ms = 0.f, ms_main = 0.f;
    if (!arena) {
        DD_HIP(hipEventElapsedTime(&ms, w.ev0, w.ev1), S);
        DD_HIP(hipEventElapsedTime(&ms_main, w.ev0, w.ev2), S);
    }
    if (hctl[3]) {
        S.code = DD_EINVAL;
        S.msg = "sinkhorn: a cell's Y box is empty or exceeds max_w1/max_w2";
        return S;
    }
    dd_batch_stats bs{};
    bs.ncells = pd.ncells;
    bs.iters_min = hctl[5];
    bs.iters_max = hctl[6];
    bs.err = htot[0];
    bs.mass = htot[1];
    bs.cell_iters = (int64_t)htot[2];
    bs.lse_terms = htot[3];
    bs.alg_bytes = htot[4];
    bs.time_ms = ms;
    bs.main_ms = ms_main;
    bs.finish_iters_max = pd.run64 ? hctl[8] : 0;
    if (pd.fast) {
        bs.path = 1;
        // fallbacks: first-X-pass outputs kept as upper bounds, exact second-X-pass outputs,
        // repeats of the second X pass after exact first-pass outputs, exact Y-update entries
        bs.tile_small[0] = hctl[12];
        bs.tile_small[1] = hctl[13];
        bs.tile_big[0] = hctl[14];
        bs.tile_big[1] = hctl[15];
        bs.n_big = pd.n[1] + pd.n[2];
        bs.n_giant = pd.n[2];
        bs.lds_kb[0] = (pd.lds[0] + 1023) / 1024;
        bs.lds_kb[1] = (std::max(pd.lds[1], pd.lds[2]) + 1023) / 1024;
        for (int k = 0; k < kClasses; ++k) {
            bs.kernel_launches[k] = pd.launches[k];
            bs.kernel_ms[k] = pd.ms[k];
            bs.kernel_terms[k] = pd.terms[k];
        }
        bs.wave_side = pd.wave_side;
        bs.big_entries = pd.big_entries;
        // the tuner learns from the float32 phase's device time per LSE term
        if (pd.fchoice >= 0 && pd.terms32 > 0.0) fast_record(pd.fkey, pd.fchoice, ms_main / pd.terms32);
    } else {
        bs.n_big = pd.n_big;
        bs.n_giant = pd.n_giant;
        bs.lds_kb[0] = (int32_t)(pd.small_budget / 1024);
        bs.lds_kb[1] = (int32_t)(pd.big_budget / 1024);
        bs.tile_small[0] = pd.small_tile[0];
        bs.tile_small[1] = pd.small_tile[1];
        bs.tile_big[0] = pd.big_tile[0];
        bs.tile_big[1] = pd.big_tile[1];
    }
    if (pd.fixed_iters > 0)
        bs.converged = 1;
    else if (pd.stop_rule == DD_STOP_CELL)
        bs.converged = hctl[7];
    else
        bs.converged = hctl[4];
    if (pd.tune && bs.lse_terms > 0.0)
        tuner().record(TuneKey{pd.key[0], pd.key[1], pd.key[2], pd.key[3]}, pd.choice,
                       ms_main / bs.lse_terms);
    if (stats) *stats = bs;
    if (!std::isfinite(bs.err)) {
        S.code = DD_ENUMERIC;
        S.msg = "sinkhorn: non-finite marginal error";
        return S;
    }
    if (!bs.converged) {
        S.code = DD_NOTCONV;
        S.msg = "sinkhorn: iteration limit reached before the tolerance";
    }
    return S;
}

Status sk_finish(SkWork& w, dd_batch_stats* stats) {
    // (an empty batch has already reported its statistics)
    if (!w.pend.active) return Status{};
    SkWork::Pend& pd = w.pend;
    if (!pd.spec) return finish_stats(w, w.h_ctl, w.h_tot, stats);
    // a speculative solve: done if the float32 rounds stopped short of the cap and the float64
    // finish stopped within its first iterations; otherwise the caller resumes it
    const int* c32 = w.h_ctl32;
    const int chunk = std::max(1, w.spec.o.check_every > 0 ? w.spec.o.check_every : 8);
    if (!(c32[2] > 0 && c32[2] < w.spec.o.max_iter && w.h_ctl[2] > 0)) {
        // (a finish that needs more iterations says nothing about the rounds)
        if (!(c32[2] > 0 && c32[2] < w.spec.o.max_iter))
            spec_rounds_learn(w, pd.ncells, c32[10], chunk, true);
        w.spec.need_resume = true;
        return Status{};
    }
    spec_rounds_learn(w, pd.ncells, c32[10], chunk, false);
    for (int r = 0; r < pd.spec_slots; ++r)
        for (int k = 0; k < kClasses; ++k) {
            float ms = 0.f;
            if (pd.n[k] && hipEventElapsedTime(&ms, w.kev[k][0][r], w.kev[k][1][r]) == hipSuccess) {
                pd.ms[k] += ms;
                pd.launches[k] += 1;
            }
        }
    pd.spec_slots = 0;
    pd.terms32 = 0.0;
    for (int k = 0; k < kClasses; ++k) {
        pd.terms[k] = pd.tpi[k] * c32[10];
        pd.terms32 += pd.terms[k];
    }
    // the statistics and the finish's words from its own block, the float32 phase's fallback
    // counters and bad-box flag from the rounds' block
    int hctl[16];
    std::copy(w.h_ctl, w.h_ctl + 16, hctl);
    hctl[3] |= c32[3];
    for (int k = 12; k < 16; ++k) hctl[k] = c32[k];
    return finish_stats(w, hctl, w.h_tot, stats);
}

}  // namespace dd

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {
dd_status batch_entry(int prec, int32_t ncells, int32_t xside, const int32_t* dims,
                      const int64_t* base, const int32_t* shift, const double* logmu,
                      const double* lognu, double* a, double* b, double kappa, int32_t max_w1,
                      int32_t max_w2, const dd_sinkhorn_opts* opts, int32_t* cell_iters,
                      double* cell_err, void* stream, dd_batch_stats* stats) {
    if (!opts || (ncells > 0 && (!dims || !base || !shift || !logmu || !lognu || !a || !b))) {
        dd::set_global_error("sinkhorn_batch: null argument");
        return DD_EINVAL;
    }
    dd::SkBatch p;
    p.ncells = ncells;
    p.xside = xside;
    p.dims = dims;
    p.base = base;
    p.shift = shift;
    p.logmu = logmu;
    p.lognu = lognu;
    p.a = a;
    p.b = b;
    p.kappa = kappa;
    p.max_w1 = max_w1;
    p.max_w2 = max_w2;
    p.prec = prec;
    dd::SkWork w;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    dd::Status s = dd::sk_solve(p, *opts, st, w, stats, cell_iters, cell_err);
    (void)hipStreamSynchronize(st);
    dd::sk_work_release(w);
    if (s.code != DD_OK) dd::set_global_error(s.msg);
    return s.code;
}
}  // namespace

extern "C" dd_status sinkhorn_set_classes(int32_t wave_side, int32_t big_entries) {
    if (wave_side == 0 && big_entries == 0) {
        dd::fast_force(0, 0);
        return DD_OK;
    }
    if (wave_side < 8 || wave_side > 32 || big_entries < 64 || big_entries > 65536) {
        dd::set_global_error("sinkhorn_set_classes: wave_side in [8, 32], big_entries in "
                             "[64, 65536], or both 0");
        return DD_EINVAL;
    }
    dd::fast_force(wave_side, big_entries);
    return DD_OK;
}

extern "C" dd_status sinkhorn_batch(int32_t ncells, int32_t xside, const int32_t* dims,
                                    const int64_t* base, const int32_t* shift, const double* logmu,
                                    const double* lognu, double* a, double* b, double kappa,
                                    int32_t max_w1, int32_t max_w2, const dd_sinkhorn_opts* opts,
                                    int32_t* cell_iters, double* cell_err, void* stream,
                                    dd_batch_stats* stats) {
    return batch_entry(DD_PREC_F32, ncells, xside, dims, base, shift, logmu, lognu, a, b, kappa,
                       max_w1, max_w2, opts, cell_iters, cell_err, stream, stats);
}

extern "C" dd_status sinkhorn_batch_f64(int32_t ncells, int32_t xside, const int32_t* dims,
                                        const int64_t* base, const int32_t* shift,
                                        const double* logmu, const double* lognu, double* a,
                                        double* b, double kappa, int32_t max_w1, int32_t max_w2,
                                        const dd_sinkhorn_opts* opts, int32_t* cell_iters,
                                        double* cell_err, void* stream, dd_batch_stats* stats) {
    return batch_entry(DD_PREC_F64, ncells, xside, dims, base, shift, logmu, lognu, a, b, kappa,
                       max_w1, max_w2, opts, cell_iters, cell_err, stream, stats);
}

// ---------------------------------------------------------------------------
// No-allocation entry point
// ---------------------------------------------------------------------------
namespace {
// The fixed device buffer every workspace of sinkhorn_batch_noalloc is carved from (control
// words, per-cell errors, masses and iteration counts, the second X-potential buffer, the
// processing orders and the global scratch of boxes beyond the LDS tiles).  Each device holds
// its own copy for the life of the process.  Host code never passes `scratch` itself to a
// kernel (in host code the name is not a device address): it uses the per-device address
// from hipGetSymbolAddress.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's `scratch`, looked up once per device with the device
// current.
dd::Status scratch_address(char*& out) {
    dd::Status st;
    int dev = -1;
    DD_HIP(hipGetDevice(&dev), st);
    if (dev < 0 || dev >= kMaxDevices) {
        st.code = DD_EDEVICE;
        st.msg = "sinkhorn_batch_noalloc: device index beyond the supported range";
        return st;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        DD_HIP(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)), st);
        if (!ptr) {
            st.code = DD_EDEVICE;
            st.msg = "sinkhorn_batch_noalloc: no device address for the scratch buffer";
            return st;
        }
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    out = g_scratch_ptr[dev];
    return st;
}
}  // namespace

extern "C" dd_status sinkhorn_batch_noalloc(int32_t ncells, int32_t xside, const int32_t* dims,
                                            const int64_t* base, const int32_t* shift,
                                            const double* logmu, const double* lognu, double* a,
                                            double* b, double kappa, int32_t max_w1,
                                            int32_t max_w2, const dd_sinkhorn_opts* opts,
                                            int32_t* cell_iters, double* cell_err, void* stream,
                                            dd_batch_stats* stats) {
    if (!opts || (ncells > 0 && (!dims || !base || !shift || !logmu || !lognu || !a || !b))) {
        dd::set_global_error("sinkhorn_batch_noalloc: null argument");
        return DD_EINVAL;
    }
    char* arena = nullptr;
    dd::Status s = scratch_address(arena);
    if (s.code != DD_OK) {
        dd::set_global_error(s.msg);
        return s.code;
    }
    dd::SkBatch p;
    p.ncells = ncells;
    p.xside = xside;
    p.dims = dims;
    p.base = base;
    p.shift = shift;
    p.logmu = logmu;
    p.lognu = lognu;
    p.a = a;
    p.b = b;
    p.kappa = kappa;
    p.max_w1 = max_w1;
    p.max_w2 = max_w2;
    p.prec = DD_PREC_F32;
    dd::SkWork w;
    w.arena = arena;
    w.arena_bytes = kNoAllocBytes;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s = dd::sk_solve(p, *opts, st, w, stats, cell_iters, cell_err);
    (void)hipStreamSynchronize(st);
    if (s.code != DD_OK) dd::set_global_error(s.msg);
    return s.code;
}
