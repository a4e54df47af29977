// Basic/composite cell-marginal kernels of one domain-decomposition iteration on gfx950.
//
//   comp_boxes  composite Y box = union of the member boxes; gauge shift E and G
//   b2c         BasicToComposite (App. A.1 eq. get-composite-cell-marginal): nu_J = sum of
//               the member nu_i on the composite box (float64), plus log nu_J for the solver
//   warm_start  X-potential initialisation: alpha = 0, or the previous visit's
//               potential re-gauged and rescaled to the new eps (alpha kept in energy units)
//   c2b         CompositeToBasic (App. A.1 "Online reduction for basic cell marginals"):
//               partial separable LSE of f + log mu over each member's X sub-block,
//               normalised shares in float64, nu_i = nu_J * share_i
//   balance     restore sum_y nu_i = m_i inside each composite cell (App. A Alg.
//               "DomDecIterGPU", BalanceGPU), pointwise proportional transfers
//   trunc_boxes / compact   TruncateGPU: zero entries below the threshold, shrink each box
//               to the entries that remain, repack with prefix-sum bases
//   scan        exclusive int64 prefix sum (one workgroup, fixed order)
//
// Everything that sums mass runs in float64 in a fixed order.  One workgroup per
// composite cell; box rows are read with consecutive lanes on consecutive pixels.
#include <algorithm>

#include "cells.hpp"

namespace dd {

namespace {

constexpr int kT = 256;

__global__ void comp_boxes_kernel(int ncell, const int32_t* __restrict__ members,
                                  const int32_t* __restrict__ xorig, const int32_t* __restrict__ box,
                                  int xside, int32_t* dims, int32_t* orig, int32_t* shift,
                                  int32_t* gofs, int64_t* size) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= ncell) return;
    int lo1 = 0x7fffffff, lo2 = 0x7fffffff, hi1 = -0x7fffffff, hi2 = -0x7fffffff;
    for (int k = 0; k < 4; ++k) {
        const int i = members[4 * J + k];
        if (i < 0) continue;
        const int o1 = box[4 * i], o2 = box[4 * i + 1], w1 = box[4 * i + 2], w2 = box[4 * i + 3];
        lo1 = min(lo1, o1);
        lo2 = min(lo2, o2);
        hi1 = max(hi1, o1 + w1);
        hi2 = max(hi2, o2 + w2);
    }
    const int W1 = hi1 - lo1, W2 = hi2 - lo2;
    // E centres the X block on the Y box: jl ~ il + E carries the bulk of the plan
    const int E1 = (W1 - xside) >> 1, E2 = (W2 - xside) >> 1;
    dims[2 * J] = W1;
    dims[2 * J + 1] = W2;
    orig[2 * J] = lo1;
    orig[2 * J + 1] = lo2;
    shift[2 * J] = E1;
    shift[2 * J + 1] = E2;
    gofs[2 * J] = xorig[2 * J] - lo1 - E1;
    gofs[2 * J + 1] = xorig[2 * J + 1] - lo2 - E2;
    size[J] = (int64_t)W1 * W2;
}

__global__ void comp_dims_kernel(int ncell, const int32_t* __restrict__ members,
                                 const int32_t* __restrict__ box, int32_t* dims) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= ncell) return;
    int lo1 = 0x7fffffff, lo2 = 0x7fffffff, hi1 = -0x7fffffff, hi2 = -0x7fffffff;
    for (int k = 0; k < 4; ++k) {
        const int i = members[4 * J + k];
        if (i < 0) continue;
        lo1 = min(lo1, box[4 * i]);
        lo2 = min(lo2, box[4 * i + 1]);
        hi1 = max(hi1, box[4 * i] + box[4 * i + 2]);
        hi2 = max(hi2, box[4 * i + 1] + box[4 * i + 3]);
    }
    dims[2 * J] = hi1 - lo1;
    dims[2 * J + 1] = hi2 - lo2;
}

__global__ void dims_check_kernel(int n, const int32_t* a, const int32_t* b, int32_t* flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && a[k] != b[k]) flag[0] = 1;
}

__global__ void comp_max_kernel(int ncell, const int32_t* dims, int32_t* info) {
    __shared__ int s1[kT / 64], s2[kT / 64];
    int m1 = 0, m2 = 0;
    for (int J = threadIdx.x; J < ncell; J += blockDim.x) {
        m1 = max(m1, dims[2 * J]);
        m2 = max(m2, dims[2 * J + 1]);
    }
    m1 = wave_max_i(m1);
    m2 = wave_max_i(m2);
    if ((threadIdx.x & 63) == 0) {
        s1[threadIdx.x >> 6] = m1;
        s2[threadIdx.x >> 6] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            m1 = max(m1, s1[w]);
            m2 = max(m2, s2[w]);
        }
        info[0] = m1;
        info[1] = m2;
    }
}

// out[0..n-1] = exclusive prefix sums of in, out[n] = total.  One workgroup of 1024.
__global__ void __launch_bounds__(1024) scan_kernel(const int64_t* in, int64_t* out, int n) {
    __shared__ int64_t part[1024];
    const int T = blockDim.x, t = threadIdx.x;
    const int chunk = (n + T - 1) / T;
    const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t ? part[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
        out[i] = run;
        run += in[i];
    }
    if (t == T - 1) out[n] = part[T - 1];
}

template <typename T>
__global__ void __launch_bounds__(kT)
    b2c_kernel(int ncell, const int32_t* __restrict__ members, const int32_t* __restrict__ box,
               const int64_t* __restrict__ bbase, const double* __restrict__ data,
               const int32_t* __restrict__ cdims, const int32_t* __restrict__ corig,
               const int64_t* __restrict__ cbase, double* nuJ, T* lognu) {
    __shared__ int mb[4][5];
    __shared__ int64_t mbase[4];
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        __syncthreads();
        if (threadIdx.x < 4) {
            const int i = members[4 * J + threadIdx.x];
            mb[threadIdx.x][4] = i;
            if (i >= 0) {
                for (int q = 0; q < 4; ++q) mb[threadIdx.x][q] = box[4 * i + q];
                mbase[threadIdx.x] = bbase[i];
            }
        }
        __syncthreads();
        const int W1 = cdims[2 * J], W2 = cdims[2 * J + 1];
        const int lo1 = corig[2 * J], lo2 = corig[2 * J + 1];
        const int64_t cb = cbase[J];
        for (int o = threadIdx.x; o < W1 * W2; o += blockDim.x) {
            const int y1 = lo1 + o / W2, y2 = lo2 + o % W2;
            double v = 0.0;
            for (int k = 0; k < 4; ++k) {
                if (mb[k][4] < 0) continue;
                const int r = y1 - mb[k][0], c = y2 - mb[k][1];
                if (r >= 0 && r < mb[k][2] && c >= 0 && c < mb[k][3])
                    v += data[mbase[k] + (int64_t)r * mb[k][3] + c];
            }
            nuJ[cb + o] = v;
            lognu[cb + o] = v > 0.0 ? (T)log(v) : neg_sentinel<T>();
        }
    }
}

// f in the gauge of this solve.  G = pX - pY - E fixes the i-dependent part of the gauge:
// f_E(i) = alpha(i)/eps - 2 <G, i>/kappa up to a constant, so a stored f with gauge G_old at
// kappa_old becomes (kappa_old/kappa_new) f + 2 <G_old - G_new, i>/kappa_new (alpha kept).
template <typename T>
__global__ void __launch_bounds__(kT)
    warm_start_kernel(int ncell, int xside, const int32_t* __restrict__ gofs, T* a,
                      int32_t* g_stored, double kold, double knew, int use_prev) {
    const int N2 = xside * xside;
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int g1 = gofs[2 * J], g2 = gofs[2 * J + 1];
        const int o1 = g_stored[2 * J], o2 = g_stored[2 * J + 1];
        for (int il = threadIdx.x; il < N2; il += blockDim.x) {
            const int i1 = il / xside, i2 = il % xside;
            double v;
            if (use_prev)
                v = (kold / knew) * (double)a[(int64_t)J * N2 + il] +
                    2.0 * ((double)(o1 - g1) * i1 + (double)(o2 - g2) * i2) / knew;
            else
                v = -2.0 * ((double)g1 * i1 + (double)g2 * i2) / knew;  // alpha = 0
            a[(int64_t)J * N2 + il] = (T)v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            g_stored[2 * J] = g1;
            g_stored[2 * J + 1] = g2;
        }
    }
}

template <typename T>
__device__ __forceinline__ T lse_line_c(const T* __restrict__ in, int stride, int K, int q, int e,
                                        T invk) {
    T d = T(e - q);
    T m = in[0] - d * d * invk;
    for (int k = 1; k < K; ++k) {
        d = T(k - q + e);
        const T v = in[k * stride] - d * d * invk;
        m = v > m ? v : m;
    }
    T s = T(0);
    for (int k = 0; k < K; ++k) {
        d = T(k - q + e);
        s += fexp(in[k * stride] - d * d * invk - m);
    }
    return m + flog(s);
}

template <typename T>
__global__ void __launch_bounds__(kT)
    c2b_kernel(int ncell, int xside, int s, int maxw2, const int32_t* __restrict__ members,
               const int32_t* __restrict__ cdims, const int32_t* __restrict__ corig,
               const int32_t* __restrict__ cshift, const int64_t* __restrict__ cbase,
               const T* __restrict__ a, const T* __restrict__ logmu, const double* __restrict__ nuJ,
               double invk_d, double h, double* tmp, double* py2) {
    extern __shared__ __align__(16) char smem[];
    double* red = reinterpret_cast<double*>(smem);
    T* sa = reinterpret_cast<T*>(smem + 64);
    const int W2p = maxw2 + 1;
    T* th = sa + xside * xside;  // [2][xside][W2p]
    const int N2 = xside * xside;
    const T invk = (T)invk_d;
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int W1 = cdims[2 * J], W2 = cdims[2 * J + 1];
        const int E1 = cshift[2 * J], E2 = cshift[2 * J + 1];
        const int lo1 = corig[2 * J], lo2 = corig[2 * J + 1];
        const int64_t cb = cbase[J];
        const int64_t nW = (int64_t)W1 * W2;
        int mem[4];
        for (int k = 0; k < 4; ++k) mem[k] = members[4 * J + k];
        __syncthreads();
        for (int il = threadIdx.x; il < N2; il += blockDim.x)
            sa[il] = a[(int64_t)J * N2 + il] + logmu[(int64_t)J * N2 + il];
        __syncthreads();
        // T_h(i1, j2) = LSE over the column half h of row i1
        for (int o = threadIdx.x; o < 2 * xside * W2; o += blockDim.x) {
            const int hh = o / (xside * W2), r = o - hh * xside * W2;
            const int i1 = r / W2, j2 = r - i1 * W2;
            th[(hh * xside + i1) * W2p + j2] = lse_line_c(sa + i1 * xside + hh * s, 1, s, j2,
                                                          E2 + hh * s, invk);
        }
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int o = threadIdx.x; o < (int)nW; o += blockDim.x) {
            const int j1 = o / W2, j2 = o - j1 * W2;
            T L[4];
            T mx = neg_sentinel<T>();
            for (int k = 0; k < 4; ++k) {
                if (mem[k] < 0) continue;
                const int v = k >> 1, hh = k & 1;
                L[k] = lse_line_c(th + (hh * xside + v * s) * W2p + j2, W2p, s, j1, E1 + v * s,
                                  invk);
                mx = L[k] > mx ? L[k] : mx;
            }
            double p[4], ps = 0.0;
            for (int k = 0; k < 4; ++k) {
                p[k] = mem[k] < 0 ? 0.0 : exp((double)(L[k] - mx));
                ps += p[k];
            }
            const double nj = nuJ[cb + o];
            const double y1 = (lo1 + j1 + 0.5) * h, y2 = (lo2 + j2 + 0.5) * h;
            const double yy = y1 * y1 + y2 * y2;
            for (int k = 0; k < 4; ++k) {
                const double v = (nj > 0.0 && ps > 0.0) ? nj * (p[k] / ps) : 0.0;
                tmp[4 * cb + k * nW + o] = v;
                acc[k] += yy * v;
            }
        }
        for (int k = 0; k < 4; ++k) {
            const double t = block_sum(acc[k], red);
            if (threadIdx.x == 0 && mem[k] >= 0) py2[mem[k]] = t;
        }
    }
}

__global__ void __launch_bounds__(kT)
    balance_kernel(int ncell, const int32_t* __restrict__ members, const int32_t* __restrict__ cdims,
                   const int64_t* __restrict__ cbase, const double* __restrict__ m, double* tmp) {
    __shared__ double red[8];
    __shared__ double M[4];
    __shared__ int ntr, tsrc[4], tdst[4];
    __shared__ double tf[4];
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int64_t nW = (int64_t)cdims[2 * J] * cdims[2 * J + 1];
        const int64_t cb = cbase[J];
        int mem[4];
        for (int k = 0; k < 4; ++k) mem[k] = members[4 * J + k];
        for (int k = 0; k < 4; ++k) {
            double s = 0.0;
            if (mem[k] >= 0)
                for (int64_t o = threadIdx.x; o < nW; o += blockDim.x) s += tmp[4 * cb + k * nW + o];
            s = block_sum(s, red);
            if (threadIdx.x == 0) M[k] = s;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // pair the first excess with the first deficit (ascending basic id), move
            // t = min(excess, deficit) in proportion to nu_src; each step zeroes one side
            double e[4], Mk[4];
            for (int k = 0; k < 4; ++k) {
                Mk[k] = M[k];
                e[k] = mem[k] >= 0 ? M[k] - m[mem[k]] : 0.0;
            }
            int n = 0;
            for (int guard = 0; guard < 4; ++guard) {
                int src = -1, dst = -1;
                for (int k = 0; k < 4 && src < 0; ++k)
                    if (mem[k] >= 0 && e[k] > 0.0) src = k;
                for (int k = 0; k < 4 && dst < 0; ++k)
                    if (mem[k] >= 0 && e[k] < 0.0) dst = k;
                if (src < 0 || dst < 0) break;
                const double t = fmin(e[src], -e[dst]);
                tsrc[n] = src;
                tdst[n] = dst;
                tf[n] = t / Mk[src];
                ++n;
                Mk[src] -= t;
                Mk[dst] += t;
                if (e[src] <= -e[dst]) {
                    e[dst] += e[src];
                    e[src] = 0.0;
                } else {
                    e[src] += e[dst];
                    e[dst] = 0.0;
                }
            }
            ntr = n;
        }
        __syncthreads();
        const int n = ntr;
        for (int64_t o = threadIdx.x; o < nW; o += blockDim.x) {
            for (int q = 0; q < n; ++q) {
                const int64_t ps = 4 * cb + tsrc[q] * nW + o, pd = 4 * cb + tdst[q] * nW + o;
                const double moved = tf[q] * tmp[ps];
                tmp[pd] = tmp[pd] + moved;
                tmp[ps] = tmp[ps] - moved;
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kT)
    trunc_boxes_kernel(int ncell, const int32_t* __restrict__ members,
                       const int32_t* __restrict__ cdims, const int32_t* __restrict__ corig,
                       const int64_t* __restrict__ cbase, const double* __restrict__ tmp,
                       double trunc, int nI, int32_t* nbox, int64_t* nsize, int32_t* flags) {
    __shared__ int r[4][kT / 64];
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int W1 = cdims[2 * J], W2 = cdims[2 * J + 1];
        const int64_t nW = (int64_t)W1 * W2, cb = cbase[J];
        for (int k = 0; k < 4; ++k) {
            const int i = members[4 * J + k];
            if (i < 0) continue;
            int mn1 = 0x7fffffff, mn2 = 0x7fffffff, mx1 = -1, mx2 = -1;
            for (int64_t o = threadIdx.x; o < nW; o += blockDim.x) {
                if (tmp[4 * cb + k * nW + o] >= trunc) {
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
                if (mx1 < 0) {  // nothing above the threshold: keep the whole box untruncated
                    mn1 = 0;
                    mn2 = 0;
                    mx1 = W1 - 1;
                    mx2 = W2 - 1;
                    keep_all = 1;
                    atomicAdd(&flags[nI], 1);
                }
                flags[i] = keep_all;
                nbox[4 * i] = corig[2 * J] + mn1;
                nbox[4 * i + 1] = corig[2 * J + 1] + mn2;
                nbox[4 * i + 2] = mx1 - mn1 + 1;
                nbox[4 * i + 3] = mx2 - mn2 + 1;
                nsize[i] = (int64_t)(mx1 - mn1 + 1) * (mx2 - mn2 + 1);
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(kT)
    compact_kernel(int ncell, const int32_t* __restrict__ members, const int32_t* __restrict__ cdims,
                   const int32_t* __restrict__ corig, const int64_t* __restrict__ cbase,
                   const double* __restrict__ tmp, double trunc, const int32_t* __restrict__ nbox,
                   const int64_t* __restrict__ nbase, const int32_t* __restrict__ flags,
                   double* ndata) {
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int W2 = cdims[2 * J + 1];
        const int64_t nW = (int64_t)cdims[2 * J] * W2, cb = cbase[J];
        for (int k = 0; k < 4; ++k) {
            const int i = members[4 * J + k];
            if (i < 0) continue;
            const int r0 = nbox[4 * i] - corig[2 * J], c0 = nbox[4 * i + 1] - corig[2 * J + 1];
            const int w1 = nbox[4 * i + 2], w2 = nbox[4 * i + 3];
            const double thr = flags[i] ? 0.0 : trunc;
            const int64_t nb = nbase[i];
            for (int o = threadIdx.x; o < w1 * w2; o += blockDim.x) {
                const int rr = o / w2, cc = o - rr * w2;
                const double v = tmp[4 * cb + k * nW + (int64_t)(r0 + rr) * W2 + (c0 + cc)];
                ndata[nb + o] = v >= thr ? v : 0.0;
            }
        }
    }
}

__global__ void fill_i32_kernel(int32_t* p, int n, int32_t v) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) p[k] = v;
}

int grid_cells(int ncell) { return std::max(1, std::min(ncell, 4096)); }

// ---- coarse-to-fine refinement of multiscale DD ------------------------------------------

// Fine basic cell i' = (r', c') is a child of coarse basic cell (r'/2, c'/2); its Y box covers
// the 2 x 2 children of every pixel of the parent's box.
__global__ void refine_boxes_kernel(int nf, int nc, const int32_t* __restrict__ cbox,
                                    int32_t* __restrict__ fbox, int64_t* __restrict__ fsize) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf * nf) return;
    const int p = (i / nf / 2) * nc + (i % nf) / 2;
    const int w1 = cbox[4 * p + 2], w2 = cbox[4 * p + 3];
    fbox[4 * i] = 2 * cbox[4 * p];
    fbox[4 * i + 1] = 2 * cbox[4 * p + 1];
    fbox[4 * i + 2] = 2 * w1;
    fbox[4 * i + 3] = 2 * w2;
    fsize[i] = 4 * (int64_t)w1 * w2;
}

// nu_i'(y') = (m_i' / m_i) nu_i(P(y')) nu_f(y') / nu_c(P(y')); one workgroup per fine cell.
__global__ void __launch_bounds__(kT)
    refine_values_kernel(int nf, int nc, int Nc, const int32_t* __restrict__ cbox,
                         const int64_t* __restrict__ cbase, const double* __restrict__ cdata,
                         const double* __restrict__ cm, const double* __restrict__ cnu,
                         const int64_t* __restrict__ fbase, const double* __restrict__ fm,
                         const double* __restrict__ fnu, double* __restrict__ fdata) {
    const int Nf = 2 * Nc;
    for (int i = blockIdx.x; i < nf * nf; i += gridDim.x) {
        const int p = (i / nf / 2) * nc + (i % nf) / 2;
        const int o1 = cbox[4 * p], o2 = cbox[4 * p + 1], w2 = cbox[4 * p + 3];
        const int W2 = 2 * w2;
        const int64_t n = fbase[i + 1] - fbase[i];
        const double share = fm[i] / cm[p];
        for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
            const int r = (int)(e / W2), q = (int)(e - (int64_t)r * W2);
            const int c1 = o1 + (r >> 1), c2 = o2 + (q >> 1);
            const double v = cdata[cbase[p] + (int64_t)(r >> 1) * w2 + (q >> 1)];
            const double nc_p = cnu[(int64_t)c1 * Nc + c2];
            const double nf_y = fnu[(int64_t)(2 * o1 + r) * Nf + (2 * o2 + q)];
            fdata[fbase[i] + e] = nc_p > 0.0 ? share * v * (nf_y / nc_p) : 0.0;
        }
    }
}

// The fine X potentials of one partition in units of eps: bilinear interpolation of the
// coarse stitched potential (same units) at the fine pixel centres, fine pixel k at coarse
// index (k - 1/2) / 2, extrapolated linearly beyond the outermost coarse centres; padding
// pixels outside the grid get 0.
__global__ void refine_alpha_kernel(int ncell, int xside, int Nc, const int32_t* __restrict__ xorig,
                                    const double* __restrict__ fc, double* __restrict__ a) {
    const int N2 = xside * xside, Nf = 2 * Nc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)ncell * N2;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int J = (int)(t / N2), il = (int)(t - (int64_t)J * N2);
        const int k1 = xorig[2 * J] + il / xside, k2 = xorig[2 * J + 1] + il % xside;
        if (k1 < 0 || k1 >= Nf || k2 < 0 || k2 >= Nf) {
            a[t] = 0.0;
            continue;
        }
        const double u1 = (k1 - 0.5) * 0.5, u2 = (k2 - 0.5) * 0.5;
        const int a1 = min(max((int)floor(u1), 0), Nc - 2), a2 = min(max((int)floor(u2), 0), Nc - 2);
        const double t1 = u1 - a1, t2 = u2 - a2;
        const double* r0 = fc + (int64_t)a1 * Nc;
        const double* r1 = r0 + Nc;
        const double lo = (1.0 - t1) * r0[a2] + t1 * r1[a2];
        const double hi = (1.0 - t1) * r0[a2 + 1] + t1 * r1[a2 + 1];
        a[t] = (1.0 - t2) * lo + t2 * hi;
    }
}

// ---- sequential batches of composite cells (bounding-box clusters) ----------------------

// dst[j][k] = src[idx[j]][k] (k < width), or the reverse direction with `back`
template <typename V>
__global__ void rows_kernel(int n, const int32_t* __restrict__ idx, int width, const V* src, V* dst,
                            int back) {
    const int64_t total = (int64_t)n * width;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t / width), k = (int)(t - (int64_t)j * width);
        const int64_t far = (int64_t)idx[j] * width + k;
        if (back)
            dst[far] = src[t];
        else
            dst[t] = src[far];
    }
}

// sizes of the listed basic cells, in list order
__global__ void list_sizes_kernel(int n, const int32_t* __restrict__ list,
                                  const int64_t* __restrict__ nsize, int64_t* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = nsize[list[k]];
}

// staging offsets of the listed basic cells: offset + their exclusive prefix sums
__global__ void stage_base_kernel(int n, const int32_t* __restrict__ list,
                                  const int64_t* __restrict__ local, int64_t offset,
                                  int64_t* stage_base) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) stage_base[list[k]] = offset + local[k];
}

// every basic cell's truncated box from its staging slot to its place in the new state
__global__ void __launch_bounds__(kT)
    unstage_kernel(int nI, const int64_t* __restrict__ nsize, const int64_t* __restrict__ stage_base,
                   const double* __restrict__ staging, const int64_t* __restrict__ nbase,
                   double* ndata) {
    for (int i = blockIdx.x; i < nI; i += gridDim.x) {
        const int64_t n = nsize[i], src = stage_base[i], dst = nbase[i];
        for (int64_t o = threadIdx.x; o < n; o += blockDim.x) ndata[dst + o] = staging[src + o];
    }
}

}  // namespace

void launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st) {
    fill_i32_kernel<<<std::max(1, std::min((n + 255) / 256, 4096)), 256, 0, st>>>(p, n, v);
}

void launch_comp_boxes(const PartDev& P, const BoxSet& S, int xside, CompDev& C, hipStream_t st) {
    const int nb = (P.ncell + 255) / 256;
    comp_boxes_kernel<<<std::max(nb, 1), 256, 0, st>>>(P.ncell, P.members, P.xorig, S.box, xside,
                                                      C.dims, C.orig, C.shift, C.gofs, C.size);
}

void launch_comp_dims(const PartDev& P, const int32_t* box, int32_t* dims, hipStream_t st) {
    if (P.ncell > 0)
        comp_dims_kernel<<<(P.ncell + 255) / 256, 256, 0, st>>>(P.ncell, P.members, box, dims);
}

void launch_dims_check(int n, const int32_t* a, const int32_t* b, int32_t* flag, hipStream_t st) {
    if (n > 0) dims_check_kernel<<<(n + 255) / 256, 256, 0, st>>>(n, a, b, flag);
}

void launch_scan(const int64_t* in, int64_t* out, int n, hipStream_t st) {
    scan_kernel<<<1, 1024, 0, st>>>(in, out, n);
}

void launch_comp_max(const CompDev& C, int ncell, hipStream_t st) {
    comp_max_kernel<<<1, kT, 0, st>>>(ncell, C.dims, C.info);
}

void launch_b2c(const PartDev& P, const BoxSet& S, const CompDev& C, double* nuJ, double* lognu,
                hipStream_t st) {
    b2c_kernel<double><<<grid_cells(P.ncell), kT, 0, st>>>(P.ncell, P.members, S.box, S.base, S.data,
                                                      C.dims, C.orig, C.base, nuJ, lognu);
}

void launch_warm_start(const PartDev& P, const CompDev& C, int xside, double* a, int32_t* g_stored,
                       double kappa_old, double kappa_new, int use_prev, hipStream_t st) {
    warm_start_kernel<double><<<grid_cells(P.ncell), kT, 0, st>>>(P.ncell, xside, C.gofs, a, g_stored,
                                                             kappa_old, kappa_new, use_prev);
}

void launch_c2b(const PartDev& P, const CompDev& C, int xside, int s, int maxw2, const double* a,
                const double* logmu, const double* nuJ, double kappa, double h, double* tmp,
                double* py2, hipStream_t st) {
    const size_t lds = 64 + sizeof(double) * ((size_t)xside * xside + 2 * (size_t)xside * (maxw2 + 1));
    c2b_kernel<double><<<grid_cells(P.ncell), kT, lds, st>>>(P.ncell, xside, s, maxw2, P.members,
                                                        C.dims, C.orig, C.shift, C.base, a, logmu,
                                                        nuJ, 1.0 / kappa, h, tmp, py2);
}

void launch_balance(const PartDev& P, const CompDev& C, const double* m, double* tmp,
                    hipStream_t st) {
    balance_kernel<<<grid_cells(P.ncell), kT, 0, st>>>(P.ncell, P.members, C.dims, C.base, m, tmp);
}

void launch_trunc_boxes(const PartDev& P, const CompDev& C, const double* tmp, double trunc,
                        int nI, int32_t* nbox, int64_t* nsize, int32_t* flags, hipStream_t st) {
    trunc_boxes_kernel<<<grid_cells(P.ncell), kT, 0, st>>>(P.ncell, P.members, C.dims, C.orig,
                                                           C.base, tmp, trunc, nI, nbox, nsize,
                                                           flags);
}

void launch_compact(const PartDev& P, const CompDev& C, const double* tmp, double trunc,
                    const int32_t* nbox, const int64_t* nbase, const int32_t* flags,
                    double* ndata, hipStream_t st) {
    compact_kernel<<<grid_cells(P.ncell), kT, 0, st>>>(P.ncell, P.members, C.dims, C.orig, C.base,
                                                       tmp, trunc, nbox, nbase, flags, ndata);
}


void launch_refine_boxes(int nf, int nc, const int32_t* cbox, int32_t* fbox, int64_t* fsize,
                         hipStream_t st) {
    refine_boxes_kernel<<<(nf * nf + kT - 1) / kT, kT, 0, st>>>(nf, nc, cbox, fbox, fsize);
}

void launch_refine_values(int nf, int nc, int Nc, const BoxSet& C, const double* cm,
                          const double* cnu, const int64_t* fbase, const double* fm,
                          const double* fnu, double* fdata, hipStream_t st) {
    refine_values_kernel<<<grid_cells(nf * nf), kT, 0, st>>>(nf, nc, Nc, C.box, C.base, C.data,
                                                             cm, cnu, fbase, fm, fnu, fdata);
}

void launch_refine_alpha(const PartDev& P, int xside, int Nc, const double* fc, double* a,
                         hipStream_t st) {
    const int64_t n = (int64_t)P.ncell * xside * xside;
    refine_alpha_kernel<<<(int)std::min<int64_t>((n + kT - 1) / kT, 8192), kT, 0, st>>>(
        P.ncell, xside, Nc, P.xorig, fc, a);
}

void launch_gather_rows(int n, const int32_t* idx, int width, const double* src, double* dst,
                        hipStream_t st) {
    const int64_t t = (int64_t)n * width;
    if (t > 0)
        rows_kernel<double><<<(int)std::min<int64_t>((t + kT - 1) / kT, 8192), kT, 0, st>>>(
            n, idx, width, src, dst, 0);
}
void launch_scatter_rows(int n, const int32_t* idx, int width, const double* src, double* dst,
                         hipStream_t st) {
    const int64_t t = (int64_t)n * width;
    if (t > 0)
        rows_kernel<double><<<(int)std::min<int64_t>((t + kT - 1) / kT, 8192), kT, 0, st>>>(
            n, idx, width, src, dst, 1);
}
void launch_gather_rows_i32(int n, const int32_t* idx, int width, const int32_t* src, int32_t* dst,
                            int back, hipStream_t st) {
    const int64_t t = (int64_t)n * width;
    if (t > 0)
        rows_kernel<int32_t><<<(int)std::min<int64_t>((t + kT - 1) / kT, 8192), kT, 0, st>>>(
            n, idx, width, src, dst, back);
}
void launch_list_sizes(int n, const int32_t* list, const int64_t* nsize, int64_t* out,
                       hipStream_t st) {
    if (n > 0) list_sizes_kernel<<<(n + kT - 1) / kT, kT, 0, st>>>(n, list, nsize, out);
}
void launch_stage_base(int n, const int32_t* list, const int64_t* local, int64_t offset,
                       int64_t* stage_base, hipStream_t st) {
    if (n > 0) stage_base_kernel<<<(n + kT - 1) / kT, kT, 0, st>>>(n, list, local, offset, stage_base);
}
void launch_unstage(int nI, const int64_t* nsize, const int64_t* stage_base, const double* staging,
                    const int64_t* nbase, double* ndata, hipStream_t st) {
    unstage_kernel<<<grid_cells(nI), kT, 0, st>>>(nI, nsize, stage_base, staging, nbase, ndata);
}

}  // namespace dd
