// Flow update with product gluing candidates (Sec. 3.2 Def. "Flow update", Def. "Gluing edge
// candidate", Remark "eps-gamma"; implementation steps of Sec. 5.1).
//
//   1. edge costs (device, float64):
//        cbar_ij = <c, mu_j/m_j (x) nu_i/m_i> - <c, pi_i>/m_i          (i != j), cbar_ii = 0
//      from cell moments.  With x, y in [0,1]^2 and c = |x - y|^2,
//        <c, mu_j/m_j (x) nu_i/m_i> = (E_j|x|^2 S0_i - 2 <xbar_j, S1_i> + S2_i) / m_i
//      where S0, S1, S2 are the zeroth, first and second moments of the stored nu_i, and
//        <c, pi_i> = sum_{x in X_i} |x|^2 pi(x,.) - 2 sum <x, y> pi + sum_y |y|^2 nu_i^pi(y)
//      with pi_i the restriction of the preceding B solve's composite plan to X_i x Y (its
//      X-moments from a float64 weighted separable LSE, its Y-marginal from CompositeToBasic
//      before balancing);
//   2. min-cost flow (host): masses b_i by largest remainder with sum 2^40, costs
//      round(cbar 2^30 / max|cbar|), network simplex; w_ij = flow_ij m_i / b_i;
//   3. assembly (device): nu_hat_j = sum_{i in N(j)} w_ij nu_i / m_i on the union of the
//      in-neighbours' boxes (eq. flow-update-cell-marginals), summed over i in ascending
//      order, then truncated below the threshold and repacked.
// The neighbourhood is the 4-neighbourhood plus self loops on the basic-cell grid; arcs are
// listed per tail in ascending head order.
//
// Gluing edge candidates from entropic plans (Def. "Gluing edge candidate", Remark "eps-gamma";
// the candidate choice of Sec. 5.1 step 1): gamma_ij is the entropic optimal transport plan
// between mu_i/m_i and mu_j/m_j (cost |x - x'|^2, regularisation eps_gamma), computed once per
// eps_gamma (mu does not change); the candidate
//     pihat_ij(x', y) = (1/m_i) sum_{x in X_i} (gamma_ij)_x(x') pi_i(x, y)
// (with (gamma_ij)_x the row of gamma_ij at x, normalised) has the edge cost
//     cbar_ij = (1/m_i) sum_{x in X_i} [(a(x) - |x|^2) P0(x) - 2 <b(x) - x, P1(x)>]
// where a(x), b(x) are the conditional second and first moments of x' under (gamma_ij)_x and
// P0(x), P1(x) = sum_y pi_i(x, y) (1, y) the per-pixel moments of the plan (the P2 terms of
// the candidate and of pi_i cancel).  With gamma_ij the product plan this is the product
// candidate's cost above.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "cells.hpp"
#include "ctx.hpp"
#include "eval.hpp"
#include "mcf.hpp"

using namespace dd;

struct FlowState {
    int narcs = 0;
    std::vector<int32_t> tail, head;
    int32_t* d_tail = nullptr;
    int32_t* d_head = nullptr;
    int32_t* d_in_start = nullptr;  // [nI+1] in-arcs of each head, tails ascending
    int32_t* d_in_arc = nullptr;
    double* d_xstat = nullptr;      // [nI][3] E|x|^2, xbar1, xbar2 of mu_j / m_j
    double* d_ystat = nullptr;      // [nI][3] S0, S1.1, S1.2 of nu_i
    double* d_ys2 = nullptr;        // [nI]    S2 of nu_i
    double* d_cbar = nullptr;       // [narcs]
    double* d_w = nullptr;          // [narcs]
    int32_t* d_nbox = nullptr;      // [nI][4]
    int64_t* d_nsize = nullptr;
    int32_t* d_flags = nullptr;
    double* d_tmp = nullptr;
    size_t tmp_cap = 0;
    McfWarm* mcf_warm = nullptr;  // the last min-cost flow's optimal basis (same graph, supplies)
    // gluing candidates: per arc and pixel x of X_tail, a(x) - |x|^2, b1(x) - x1, b2(x) - x2
    double* d_cand = nullptr;     // [narcs][s*s][3]
    double cand_eps = -1.0;       // eps_gamma d_cand was computed for
    double* d_pix = nullptr;      // [N*N][3] per-pixel moments of the last B plans
};

namespace {

constexpr int kT = 256;

__global__ void ystat_kernel(int nI, const int32_t* __restrict__ box, const int64_t* __restrict__ base,
                             const double* __restrict__ data, double h, double* ystat, double* ys2) {
    __shared__ double red[8];
    for (int i = blockIdx.x; i < nI; i += gridDim.x) {
        const int o1 = box[4 * i], o2 = box[4 * i + 1], w2 = box[4 * i + 3];
        const int64_t b = base[i], n = base[i + 1] - base[i];
        double s0 = 0, s1 = 0, s2 = 0, sq = 0;
        for (int64_t o = threadIdx.x; o < n; o += blockDim.x) {
            const double v = data[b + o];
            const double y1 = (o1 + (double)(o / w2) + 0.5) * h, y2 = (o2 + (double)(o % w2) + 0.5) * h;
            s0 += v;
            s1 += v * y1;
            s2 += v * y2;
            sq += v * (y1 * y1 + y2 * y2);
        }
        s0 = block_sum(s0, red);
        s1 = block_sum(s1, red);
        s2 = block_sum(s2, red);
        sq = block_sum(sq, red);
        if (threadIdx.x == 0) {
            ystat[3 * i] = s0;
            ystat[3 * i + 1] = s1;
            ystat[3 * i + 2] = s2;
            ys2[i] = sq;
        }
    }
}

__global__ void cbar_kernel(int narcs, const int32_t* __restrict__ tail, const int32_t* __restrict__ head,
                            const double* __restrict__ m, const double* __restrict__ xstat,
                            const double* __restrict__ ystat, const double* __restrict__ ys2,
                            const double* __restrict__ pstat /*[nI][3] pixel units*/,
                            const double* __restrict__ py2, double h, double* cbar) {
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < narcs; a += gridDim.x * blockDim.x) {
        const int i = tail[a], j = head[a];
        if (i == j) {
            cbar[a] = 0.0;
            continue;
        }
        const double mi = m[i];
        const double cand = xstat[3 * j] * ystat[3 * i] -
                            2.0 * (xstat[3 * j + 1] * ystat[3 * i + 1] +
                                   xstat[3 * j + 2] * ystat[3 * i + 2]) +
                            ys2[i];
        const double self = h * h * (pstat[3 * i + 1] - 2.0 * pstat[3 * i + 2]) + py2[i];
        cbar[a] = (cand - self) / mi;
    }
}

// gamma_ij for arc (i, j), i != j, by log-domain Sinkhorn on the s^2 x s^2 problem (one thread
// per arc, float64), then the conditional moments of its rows.  Rows x: the pixels of X_i with
// weights mu/m_i; columns x': those of X_j.  Only the column potential enters the normalised
// rows, so the iteration stops once it no longer moves (or after kGammaIters).
constexpr int kMaxS2 = 64, kGammaIters = 20000;
__global__ void gamma_kernel(int narcs, const int32_t* __restrict__ tail,
                             const int32_t* __restrict__ head, int n, int s, int N,
                             const double* __restrict__ mu, double h, double eps_g,
                             double* __restrict__ cand) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= narcs) return;
    const int i = tail[a], j = head[a], S2 = s * s;
    double* out = cand + (int64_t)a * S2 * 3;
    if (i == j) {
        for (int k = 0; k < 3 * S2; ++k) out[k] = 0.0;
        return;
    }
    const int ri = (i / n) * s, ci = (i % n) * s, rj = (j / n) * s, cj = (j % n) * s;
    double lmi[kMaxS2], lmj[kMaxS2], f[kMaxS2], g[kMaxS2];
    for (int u = 0; u < S2; ++u) {
        const double vi = mu[(int64_t)(ri + u / s) * N + ci + u % s];
        const double vj = mu[(int64_t)(rj + u / s) * N + cj + u % s];
        lmi[u] = vi > 0.0 ? log(vi) : kNegD;
        lmj[u] = vj > 0.0 ? log(vj) : kNegD;
        f[u] = 0.0;
        g[u] = 0.0;
    }
    // cost in units of eps_gamma: h^2 |p - p'|^2 / eps_g in pixel offsets
    const double ck = h * h / eps_g;
    auto cost = [&](int u, int v) {
        const double d1 = (ri + u / s) - (rj + v / s), d2 = (ci + u % s) - (cj + v % s);
        return ck * (d1 * d1 + d2 * d2);
    };
    for (int it = 0; it < kGammaIters; ++it) {
        // g(x') = -LSE_x [f(x) + log mu_i(x) - c(x, x')]  (the mass normalisations are constants)
        double moved = 0.0;
        for (int v = 0; v < S2; ++v) {
            double m = -1e300;
            for (int u = 0; u < S2; ++u)
                if (lmi[u] > kZeroMassLog) m = fmax(m, f[u] + lmi[u] - cost(u, v));
            double t = 0.0;
            for (int u = 0; u < S2; ++u)
                if (lmi[u] > kZeroMassLog) t += exp(f[u] + lmi[u] - cost(u, v) - m);
            const double gv = -(m + log(t));
            moved = fmax(moved, fabs(gv - g[v]));
            g[v] = gv;
        }
        if (it > 0 && moved <= 1e-13) break;
        // f(x) = -LSE_x' [g(x') + log mu_j(x') - c(x, x')]
        for (int u = 0; u < S2; ++u) {
            double m = -1e300;
            for (int v = 0; v < S2; ++v)
                if (lmj[v] > kZeroMassLog) m = fmax(m, g[v] + lmj[v] - cost(u, v));
            double t = 0.0;
            for (int v = 0; v < S2; ++v)
                if (lmj[v] > kZeroMassLog) t += exp(g[v] + lmj[v] - cost(u, v) - m);
            f[u] = -(m + log(t));
        }
    }
    // conditional moments of the normalised rows, in [0, 1] coordinates
    for (int u = 0; u < S2; ++u) {
        double m = -1e300;
        for (int v = 0; v < S2; ++v)
            if (lmj[v] > kZeroMassLog) m = fmax(m, g[v] + lmj[v] - cost(u, v));
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, wq = 0.0;
        for (int v = 0; v < S2; ++v) {
            if (!(lmj[v] > kZeroMassLog)) continue;
            const double r = exp(g[v] + lmj[v] - cost(u, v) - m);
            const double y1 = (rj + v / s + 0.5) * h, y2 = (cj + v % s + 0.5) * h;
            w0 += r;
            w1 += r * y1;
            w2 += r * y2;
            wq += r * (y1 * y1 + y2 * y2);
        }
        const double x1 = (ri + u / s + 0.5) * h, x2 = (ci + u % s + 0.5) * h;
        out[3 * u] = wq / w0 - (x1 * x1 + x2 * x2);
        out[3 * u + 1] = w1 / w0 - x1;
        out[3 * u + 2] = w2 / w0 - x2;
    }
}

__global__ void cbar_glued_kernel(int narcs, const int32_t* __restrict__ tail,
                                  const int32_t* __restrict__ head, int n, int s, int N,
                                  const double* __restrict__ m, const double* __restrict__ cand,
                                  const double* __restrict__ pix, double h, double* cbar) {
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < narcs; a += gridDim.x * blockDim.x) {
        const int i = tail[a], j = head[a];
        if (i == j) {
            cbar[a] = 0.0;
            continue;
        }
        const int ri = (i / n) * s, ci = (i % n) * s, S2 = s * s;
        const double* cd = cand + (int64_t)a * S2 * 3;
        double t = 0.0;
        for (int u = 0; u < S2; ++u) {
            const double* p = pix + 3 * ((int64_t)(ri + u / s) * N + ci + u % s);
            // P1 = h (sum_y (y_pix + 1/2) pi) in [0, 1] coordinates
            t += cd[3 * u] * p[0] - 2.0 * h * (cd[3 * u + 1] * p[1] + cd[3 * u + 2] * p[2]);
        }
        cbar[a] = t / m[i];
    }
}

// union box of the in-neighbours with w > 0
__global__ void fbox_kernel(int nI, const int32_t* __restrict__ in_start, const int32_t* __restrict__ in_arc,
                            const int32_t* __restrict__ tail, const double* __restrict__ w,
                            const int32_t* __restrict__ box, int32_t* nbox, int64_t* nsize) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nI) return;
    int lo1 = 0x7fffffff, lo2 = 0x7fffffff, hi1 = -0x7fffffff, hi2 = -0x7fffffff;
    for (int k = in_start[j]; k < in_start[j + 1]; ++k) {
        const int a = in_arc[k];
        if (!(w[a] > 0.0)) continue;
        const int i = tail[a];
        lo1 = min(lo1, box[4 * i]);
        lo2 = min(lo2, box[4 * i + 1]);
        hi1 = max(hi1, box[4 * i] + box[4 * i + 2]);
        hi2 = max(hi2, box[4 * i + 1] + box[4 * i + 3]);
    }
    if (hi1 < lo1) {  // no inflow: cannot happen for a feasible flow (m_j > 0)
        lo1 = box[4 * j];
        lo2 = box[4 * j + 1];
        hi1 = lo1 + 1;
        hi2 = lo2 + 1;
    }
    nbox[4 * j] = lo1;
    nbox[4 * j + 1] = lo2;
    nbox[4 * j + 2] = hi1 - lo1;
    nbox[4 * j + 3] = hi2 - lo2;
    nsize[j] = (int64_t)(hi1 - lo1) * (hi2 - lo2);
}

// nu_hat_j on its union box (before truncation)
__global__ void __launch_bounds__(kT)
    fassemble_kernel(int nI, const int32_t* __restrict__ in_start, const int32_t* __restrict__ in_arc,
                     const int32_t* __restrict__ tail, const double* __restrict__ w,
                     const double* __restrict__ m, const int32_t* __restrict__ box,
                     const int64_t* __restrict__ base, const double* __restrict__ data,
                     const int32_t* __restrict__ ubox, const int64_t* __restrict__ ubase, double* out) {
    for (int j = blockIdx.x; j < nI; j += gridDim.x) {
        const int u1 = ubox[4 * j], u2 = ubox[4 * j + 1], uw2 = ubox[4 * j + 3];
        const int64_t n = (int64_t)ubox[4 * j + 2] * uw2, ob = ubase[j];
        const int k0 = in_start[j], k1 = in_start[j + 1];
        for (int64_t o = threadIdx.x; o < n; o += blockDim.x) {
            const int y1 = u1 + (int)(o / uw2), y2 = u2 + (int)(o % uw2);
            double v = 0.0;
            for (int k = k0; k < k1; ++k) {
                const int a = in_arc[k];
                const double wa = w[a];
                if (!(wa > 0.0)) continue;
                const int i = tail[a];
                const int r = y1 - box[4 * i], c = y2 - box[4 * i + 1];
                if (r >= 0 && r < box[4 * i + 2] && c >= 0 && c < box[4 * i + 3])
                    v += (wa / m[i]) * data[base[i] + (int64_t)r * box[4 * i + 3] + c];
            }
            out[ob + o] = v;
        }
    }
}

__global__ void __launch_bounds__(kT)
    ftrunc_kernel(int nI, const int32_t* __restrict__ ubox, const int64_t* __restrict__ ubase,
                  const double* __restrict__ vals, double trunc, int32_t* nbox, int64_t* nsize,
                  int32_t* flags) {
    __shared__ int r[4][kT / 64];
    for (int j = blockIdx.x; j < nI; j += gridDim.x) {
        const int W2 = ubox[4 * j + 3];
        const int64_t n = (int64_t)ubox[4 * j + 2] * W2, b = ubase[j];
        int mn1 = 0x7fffffff, mn2 = 0x7fffffff, mx1 = -1, mx2 = -1;
        for (int64_t o = threadIdx.x; o < n; o += blockDim.x) {
            if (vals[b + o] >= trunc) {
                const int j1 = (int)(o / W2), j2 = (int)(o % W2);
                mn1 = min(mn1, j1);
                mn2 = min(mn2, j2);
                mx1 = max(mx1, j1);
                mx2 = max(mx2, j2);
            }
        }
        mn1 = wave_min_i(mn1);
        mn2 = wave_min_i(mn2);
        mx1 = wave_max_i(mx1);
        mx2 = wave_max_i(mx2);
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            r[0][w] = mn1;
            r[1][w] = mn2;
            r[2][w] = mx1;
            r[3][w] = mx2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
                mn1 = min(mn1, r[0][q]);
                mn2 = min(mn2, r[1][q]);
                mx1 = max(mx1, r[2][q]);
                mx2 = max(mx2, r[3][q]);
            }
            int keep_all = 0;
            if (mx1 < 0) {
                mn1 = mn2 = 0;
                mx1 = ubox[4 * j + 2] - 1;
                mx2 = W2 - 1;
                keep_all = 1;
            }
            flags[j] = keep_all;
            nbox[4 * j] = ubox[4 * j] + mn1;
            nbox[4 * j + 1] = ubox[4 * j + 1] + mn2;
            nbox[4 * j + 2] = mx1 - mn1 + 1;
            nbox[4 * j + 3] = mx2 - mn2 + 1;
            nsize[j] = (int64_t)(mx1 - mn1 + 1) * (mx2 - mn2 + 1);
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kT)
    fcompact_kernel(int nI, const int32_t* __restrict__ ubox, const int64_t* __restrict__ ubase,
                    const double* __restrict__ vals, double trunc, const int32_t* __restrict__ nbox,
                    const int64_t* __restrict__ nbase, const int32_t* __restrict__ flags, double* out) {
    for (int j = blockIdx.x; j < nI; j += gridDim.x) {
        const int r0 = nbox[4 * j] - ubox[4 * j], c0 = nbox[4 * j + 1] - ubox[4 * j + 1];
        const int w2 = nbox[4 * j + 3], W2 = ubox[4 * j + 3];
        const int64_t n = (int64_t)nbox[4 * j + 2] * w2;
        const double thr = flags[j] ? 0.0 : trunc;
        for (int64_t o = threadIdx.x; o < n; o += blockDim.x) {
            const int rr = (int)(o / w2), cc = (int)(o % w2);
            const double v = vals[ubase[j] + (int64_t)(r0 + rr) * W2 + (c0 + cc)];
            out[nbase[j] + o] = v >= thr ? v : 0.0;
        }
    }
}

dd_status ffail(dd_ctx* c, dd_status code, const std::string& m) {
    if (c) c->err = m;
    set_global_error(m);
    return code;
}

template <typename P>
bool dalloc(const dd::Mem& M, P*& p, size_t n) {
    return M.get(&p, std::max<size_t>(n, 1) * sizeof(P)) == hipSuccess;
}

// Build the static flow structures on first use.
dd_status flow_prepare(dd_ctx* c) {
    if (c->flow) return DD_OK;
    FlowState* F = new FlowState();
    const int n = c->n, nI = c->nI;
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) {
            const int i = r * n + q;
            const int nb[5][2] = {{r - 1, q}, {r, q - 1}, {r, q}, {r, q + 1}, {r + 1, q}};
            for (auto& d : nb)
                if (d[0] >= 0 && d[0] < n && d[1] >= 0 && d[1] < n) {
                    F->tail.push_back(i);
                    F->head.push_back(d[0] * n + d[1]);
                }
        }
    F->narcs = (int)F->tail.size();
    std::vector<int32_t> in_start(nI + 1, 0), in_arc(F->narcs);
    for (int a = 0; a < F->narcs; ++a) in_start[F->head[a] + 1]++;
    for (int j = 0; j < nI; ++j) in_start[j + 1] += in_start[j];
    {
        std::vector<int32_t> fill(in_start.begin(), in_start.end() - 1);
        for (int a = 0; a < F->narcs; ++a) in_arc[fill[F->head[a]]++] = a;  // tails ascending
    }
    // X statistics of mu_j / m_j in [0,1] coordinates (host copy of mu is not kept: read back)
    std::vector<double> mu((size_t)c->N * c->N);
    if (hipMemcpy(mu.data(), c->d_mu, mu.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        delete F;
        return ffail(c, DD_EDEVICE, "flow_update: reading mu failed");
    }
    std::vector<double> xstat(3 * (size_t)nI);
    const int s = c->s, N = c->N;
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) {
            const int j = r * n + q;
            double e2 = 0, x1 = 0, x2 = 0;
            for (int a = 0; a < s; ++a)
                for (int b = 0; b < s; ++b) {
                    const double v = mu[(size_t)(r * s + a) * N + (q * s + b)];
                    const double p1 = (r * s + a + 0.5) * c->h, p2 = (q * s + b + 0.5) * c->h;
                    e2 += v * (p1 * p1 + p2 * p2);
                    x1 += v * p1;
                    x2 += v * p2;
                }
            xstat[3 * j] = e2 / c->m[j];
            xstat[3 * j + 1] = x1 / c->m[j];
            xstat[3 * j + 2] = x2 / c->m[j];
        }
    bool ok = dalloc(c->mem, F->d_tail, F->narcs) && dalloc(c->mem, F->d_head, F->narcs) &&
              dalloc(c->mem, F->d_in_start, nI + 1) && dalloc(c->mem, F->d_in_arc, F->narcs) &&
              dalloc(c->mem, F->d_xstat, 3 * (size_t)nI) && dalloc(c->mem, F->d_ystat, 3 * (size_t)nI) &&
              dalloc(c->mem, F->d_ys2, nI) && dalloc(c->mem, F->d_cbar, F->narcs) && dalloc(c->mem, F->d_w, F->narcs) &&
              dalloc(c->mem, F->d_nbox, 4 * (size_t)nI) && dalloc(c->mem, F->d_nsize, nI) &&
              dalloc(c->mem, F->d_flags, nI + 1);
    ok = ok &&
         hipMemcpy(F->d_tail, F->tail.data(), F->narcs * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(F->d_head, F->head.data(), F->narcs * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(F->d_in_start, in_start.data(), (nI + 1) * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(F->d_in_arc, in_arc.data(), F->narcs * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(F->d_xstat, xstat.data(), xstat.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    c->flow = F;
    if (!ok) return ffail(c, DD_ENOMEM, "flow_update: allocating flow structures failed");
    return DD_OK;
}

}  // namespace

void flow_release(dd_ctx* c) {
    FlowState* F = c->flow;
    if (!F) return;
    auto Fr = [c](auto& p) {
        c->mem.put(p);
        p = nullptr;
    };
    Fr(F->d_tail);
    Fr(F->d_head);
    Fr(F->d_in_start);
    Fr(F->d_in_arc);
    Fr(F->d_xstat);
    Fr(F->d_ystat);
    Fr(F->d_ys2);
    Fr(F->d_cbar);
    Fr(F->d_w);
    Fr(F->d_nbox);
    Fr(F->d_nsize);
    Fr(F->d_flags);
    Fr(F->d_tmp);
    Fr(F->d_cand);
    Fr(F->d_pix);
    mcf_warm_free(F->mcf_warm);
    delete F;
    c->flow = nullptr;
}

extern "C" dd_status flow_costs(dd_ctx* c, int32_t candidate, double eps_gamma, double* cbar,
                                int32_t* n_arcs) {
    if (!c) return ffail(c, DD_EINVAL, "flow_costs: null context");
    dd_forget_pred(c);
    if (candidate != DD_CAND_PRODUCT && candidate != DD_CAND_GLUED)
        return ffail(c, DD_EINVAL, "flow_costs: candidate must be DD_CAND_PRODUCT or DD_CAND_GLUED");
    if (candidate == DD_CAND_GLUED && (!(eps_gamma > 0.0) || !std::isfinite(eps_gamma) || c->s > 8))
        return ffail(c, DD_EINVAL, "flow_costs: glued candidates need 0 < eps_gamma < inf, s <= 8");
    if (c->last_part != DD_PART_B)
        return ffail(c, DD_ESTATE, "flow_costs: the last iteration must be on partition B");
    dd_status st = flow_prepare(c);
    if (st != DD_OK) return st;
    FlowState* F = c->flow;
    if (n_arcs) *n_arcs = F->narcs;
    const hipStream_t hs = c->st;
    const int ab = std::max(1, (F->narcs + kT - 1) / kT);
    if (candidate == DD_CAND_PRODUCT) {
        dd_eval_cells(c);  // X moments of pi_i from the last B solve -> d_basic_out
        const int nb = std::max(1, std::min(c->nI, 4096));
        ystat_kernel<<<nb, kT, 0, hs>>>(c->nI, c->S.box, c->S.base, c->S.data, c->h, F->d_ystat,
                                        F->d_ys2);
        cbar_kernel<<<ab, kT, 0, hs>>>(F->narcs, F->d_tail, F->d_head, c->d_m, F->d_xstat,
                                       F->d_ystat, F->d_ys2, c->d_basic_out, c->d_py2, c->h,
                                       F->d_cbar);
    } else {
        const int S2 = c->s * c->s;
        if (!F->d_cand && !dalloc(c->mem, F->d_cand, (size_t)F->narcs * S2 * 3))
            return ffail(c, DD_ENOMEM, "flow_costs: allocating the candidates failed");
        if (!F->d_pix && !dalloc(c->mem, F->d_pix, (size_t)c->N * c->N * 3))
            return ffail(c, DD_ENOMEM, "flow_costs: allocating the pixel moments failed");
        if (F->cand_eps != eps_gamma) {
            gamma_kernel<<<ab, kT, 0, hs>>>(F->narcs, F->d_tail, F->d_head, c->n, c->s, c->N,
                                            c->d_mu, c->h, eps_gamma, F->d_cand);
            F->cand_eps = eps_gamma;
        }
        dd_eval_cells(c, F->d_pix);  // per-pixel X moments of pi_i from the last B solve
        cbar_glued_kernel<<<ab, kT, 0, hs>>>(F->narcs, F->d_tail, F->d_head, c->n, c->s, c->N,
                                             c->d_m, F->d_cand, F->d_pix, c->h, F->d_cbar);
    }
    if (cbar && hipMemcpyAsync(cbar, F->d_cbar, F->narcs * sizeof(double), hipMemcpyDeviceToHost, hs) !=
                    hipSuccess)
        return ffail(c, DD_EDEVICE, "flow_costs: copy failed");
    if (hipStreamSynchronize(hs) != hipSuccess || hipGetLastError() != hipSuccess)
        return ffail(c, DD_EDEVICE, "flow_costs: a kernel failed");
    return DD_OK;
}

extern "C" dd_status flow_apply(dd_ctx* c, const double* w) {
    if (!c || !w) return ffail(c, DD_EINVAL, "flow_apply: null argument");
    dd_forget_pred(c);
    dd_status st = flow_prepare(c);
    if (st != DD_OK) return st;
    FlowState* F = c->flow;
    const hipStream_t hs = c->st;
    const int nI = c->nI;
    if (hipMemcpyAsync(F->d_w, w, F->narcs * sizeof(double), hipMemcpyHostToDevice, hs) != hipSuccess)
        return ffail(c, DD_EDEVICE, "flow_apply: copy failed");
    // union boxes -> S2 (temporarily), sizes, bases
    fbox_kernel<<<std::max(1, (nI + 255) / 256), 256, 0, hs>>>(nI, F->d_in_start, F->d_in_arc, F->d_tail,
                                                                F->d_w, c->S.box, F->d_nbox, F->d_nsize);
    launch_scan(F->d_nsize, c->S2.base, nI, hs);
    int64_t utot = 0;
    if (hipMemcpyAsync(&utot, c->S2.base + nI, sizeof utot, hipMemcpyDeviceToHost, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return ffail(c, DD_EDEVICE, "flow_apply: reading sizes failed");
    if ((size_t)utot > F->tmp_cap) {
        c->mem.put(F->d_tmp);
        F->d_tmp = nullptr;
        F->tmp_cap = (size_t)(utot * 1.25) + 64;
        if (c->mem.get(&F->d_tmp, F->tmp_cap * sizeof(double)) != hipSuccess)
            return ffail(c, DD_ENOMEM, "flow_apply: out of memory");
    }
    // keep the union bases: copy into a scratch int64 array (reuse d_nsize after the scan)
    int64_t* ubase = nullptr;
    if (c->mem.get(&ubase, (nI + 1) * sizeof(int64_t)) != hipSuccess)
        return ffail(c, DD_ENOMEM, "flow_apply: out of memory");
    (void)hipMemcpyAsync(ubase, c->S2.base, (nI + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, hs);
    const int nb = std::max(1, std::min(nI, 4096));
    fassemble_kernel<<<nb, kT, 0, hs>>>(nI, F->d_in_start, F->d_in_arc, F->d_tail, F->d_w, c->d_m, c->S.box,
                                        c->S.base, c->S.data, F->d_nbox, ubase, F->d_tmp);
    launch_fill_i32(F->d_flags, nI + 1, 0, hs);
    ftrunc_kernel<<<nb, kT, 0, hs>>>(nI, F->d_nbox, ubase, F->d_tmp, c->trunc, c->S2.box, F->d_nsize,
                                     F->d_flags);
    launch_scan(F->d_nsize, c->S2.base, nI, hs);
    int64_t ntot = 0;
    if (hipMemcpyAsync(&ntot, c->S2.base + nI, sizeof ntot, hipMemcpyDeviceToHost, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess) {
        c->mem.put(ubase);
        return ffail(c, DD_EDEVICE, "flow_apply: reading sizes failed");
    }
    if ((size_t)ntot > c->S2.cap) {
        c->mem.put(c->S2.data);
        c->S2.data = nullptr;
        c->S2.cap = (size_t)(ntot * 1.25) + 64;
        if (c->mem.get(&c->S2.data, c->S2.cap * sizeof(double)) != hipSuccess) {
            c->mem.put(ubase);
            return ffail(c, DD_ENOMEM, "flow_apply: out of memory");
        }
    }
    fcompact_kernel<<<nb, kT, 0, hs>>>(nI, F->d_nbox, ubase, F->d_tmp, c->trunc, c->S2.box, c->S2.base,
                                       F->d_flags, c->S2.data);
    if (hipStreamSynchronize(hs) != hipSuccess || hipGetLastError() != hipSuccess) {
        c->mem.put(ubase);
        return ffail(c, DD_EDEVICE, "flow_apply: a kernel failed");
    }
    c->mem.put(ubase);
    std::swap(c->S, c->S2);
    // the composite plans no longer describe the state: X-marginal / primal need a new iteration
    c->last_part = -1;
    return DD_OK;
}

extern "C" dd_status dd_mcf_solve(int32_t n, int32_t m, const int32_t* tail, const int32_t* head,
                                  const int64_t* cost, const int64_t* supply, int64_t* flow,
                                  int64_t* potential) {
    if (n < 0 || m < 0 || (m > 0 && (!tail || !head || !cost || !flow)) || (n > 0 && !supply)) {
        set_global_error("dd_mcf_solve: bad arguments");
        return DD_EINVAL;
    }
    const int r = mcf_network_simplex(n, m, tail, head, cost, supply, flow, potential);
    if (r == 0) return DD_OK;
    set_global_error(r == -1 ? "dd_mcf_solve: infeasible" : r == -2 ? "dd_mcf_solve: bad input"
                     : r == -3 ? "dd_mcf_solve: pivot limit reached" : "dd_mcf_solve: unbounded");
    return r == -2 ? DD_EINVAL : DD_ENUMERIC;
}

extern "C" dd_status flow_update(dd_ctx* c, int32_t candidate, double eps_gamma,
                                 dd_flow_stats* out) {
    if (!c) return ffail(c, DD_EINVAL, "flow_update: null context");
    dd_forget_pred(c);
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    int32_t na = 0;
    dd_status st = flow_prepare(c);
    if (st != DD_OK) return st;
    FlowState* F = c->flow;
    std::vector<double> cbar(F->narcs);
    st = flow_costs(c, candidate, eps_gamma, cbar.data(), &na);
    if (st != DD_OK) return st;
    const auto t1 = clk::now();
    // integerise: masses by largest remainder to 2^40, costs to 2^30 / max|cbar|
    const int nI = c->nI;
    const int64_t T = (int64_t)1 << 40;
    double msum = 0.0;
    for (double v : c->m) msum += v;
    std::vector<int64_t> b(nI), cost(na), flow(na);
    std::vector<double> frac(nI);
    int64_t bs = 0;
    for (int i = 0; i < nI; ++i) {
        const double q = c->m[i] / msum * (double)T;
        b[i] = (int64_t)std::floor(q);
        frac[i] = q - (double)b[i];
        bs += b[i];
    }
    {
        std::vector<int> order(nI);
        for (int i = 0; i < nI; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return frac[x] > frac[y]; });
        for (int64_t k = 0; k < T - bs; ++k) b[order[k]] += 1;
    }
    double cmax = 0.0;
    for (double v : cbar) cmax = std::max(cmax, std::fabs(v));
    const double scale = cmax > 0 ? (double)((int64_t)1 << 30) / cmax : 0.0;
    for (int a = 0; a < na; ++a) cost[a] = (int64_t)std::nearbyint(cbar[a] * scale);
    // successive updates share the graph and the supplies (the masses of mu): the last
    // update's optimal basis starts this one
    if (!F->mcf_warm) F->mcf_warm = mcf_warm_create();
    const int r = mcf_network_simplex_warm(nI, na, F->tail.data(), F->head.data(), cost.data(),
                                           b.data(), flow.data(), nullptr, F->mcf_warm);
    if (r != 0) return ffail(c, DD_ENUMERIC, "flow_update: min-cost flow failed");
    const auto t2 = clk::now();
    std::vector<double> w(na);
    double value = 0.0, moved = 0.0;
    long double ival = 0.0L;
    int active = 0;
    for (int a = 0; a < na; ++a) {
        const int i = F->tail[a];
        w[a] = (double)flow[a] * (c->m[i] / (double)b[i]);
        value += w[a] * cbar[a];
        ival += (long double)flow[a] * (long double)cost[a];
        if (F->tail[a] != F->head[a] && flow[a] > 0) {
            moved += w[a];
            ++active;
        }
    }
    st = flow_apply(c, w.data());
    if (st != DD_OK) return st;
    const auto t3 = clk::now();
    if (out) {
        dd_flow_stats s{};
        s.n_nodes = nI;
        s.n_arcs = na;
        s.int_value = (double)ival;
        s.value = value;
        s.moved_mass = moved;
        s.n_active_arcs = active;
        s.t_costs_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        s.t_mcf_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
        s.t_assemble_ms = std::chrono::duration<double, std::milli>(t3 - t2).count();
        *out = s;
    }
    return DD_OK;
}
