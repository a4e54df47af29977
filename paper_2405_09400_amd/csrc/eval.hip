// Float64 quality reductions of the current state (App. A.2.2 "Solution quality") and the
// per-cell moments the flow update needs.
//
//   ymarg       sum_i nu_i accumulated on the dense Y grid (float64 atomics: the order of
//               the additions, and so the last bits, may vary between runs)
//   basic_mass  max_i |sum_y nu_i - m_i| and total stored mass
//   cell_eval   per composite cell of the last solve: the X-marginal
//               m0(x) = mu(x) exp(f(x) + s0(x)) with s0 = LSE_j [g + log nu_J - C], the first moments m1, m2 = sum_y y_k pi(x, y)
//               (weighted separable LSEs), and from them
//                 * the primal objective E(pi_J) = eps sum_x m0 (alpha/eps) +
//                   eps sum_y nu_J (beta/eps) - eps sum pi (exact for plans of the form
//                   exp((alpha + beta - c)/eps) mu nu),
//                 * the transport cost <c, pi_J>,
//                 * per basic cell: sum m0, sum |x|^2 m0, sum <x, y> pi.
#include <algorithm>

#include "eval.hpp"

namespace dd {

namespace {

constexpr int kT = 256;

__global__ void ymarg_kernel(int nI, const int32_t* __restrict__ box, const int64_t* __restrict__ base,
                             const double* __restrict__ data, int N, double* acc) {
    for (int i = blockIdx.x; i < nI; i += gridDim.x) {
        const int o1 = box[4 * i], o2 = box[4 * i + 1], w2 = box[4 * i + 3];
        const int64_t b = base[i], n = base[i + 1] - base[i];
        for (int64_t o = threadIdx.x; o < n; o += blockDim.x) {
            const double v = data[b + o];
            if (v != 0.0) {
                const int r = (int)(o / w2), c = (int)(o % w2);
                atomicAdd(&acc[(int64_t)(o1 + r) * N + (o2 + c)], v);
            }
        }
    }
}

__global__ void fill_kernel(double* p, size_t n, double v) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ void l1diff_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                              double* out) {
    __shared__ double red[8];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) s += fabs(a[k] - b[k]);
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void basic_mass_kernel(int nI, const int64_t* __restrict__ base,
                                  const double* __restrict__ data, const double* __restrict__ m,
                                  double* per_cell) {
    __shared__ double red[8];
    for (int i = blockIdx.x; i < nI; i += gridDim.x) {
        double s = 0.0;
        for (int64_t o = base[i] + threadIdx.x; o < base[i + 1]; o += blockDim.x) s += data[o];
        s = block_sum(s, red);
        if (threadIdx.x == 0) per_cell[i] = s;
    }
}

__global__ void mass_summary_kernel(int nI, const double* per_cell, const double* m, double* out) {
    __shared__ double red[8];
    __shared__ double smax[kT / 64];
    double s = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < nI; i += blockDim.x) {
        s += per_cell[i];
        mx = fmax(mx, fabs(per_cell[i] - m[i]));
    }
    s = block_sum(s, red);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, smax[w]);
        out[0] = s;
        out[1] = mx;
    }
}

template <typename T>
__device__ __forceinline__ double lse_w(const T* __restrict__ in, int stride, int K, int q, int e,
                                        double invk, const double* __restrict__ logw) {
    // LSE_k (in[k] + logw[k] - (k - q + e)^2 invk) in float64 (logw may be null)
    double m = -1e300;
    for (int k = 0; k < K; ++k) {
        const double d = (double)(k - q + e);
        const double v = (double)in[k * stride] + (logw ? logw[k] : 0.0) - d * d * invk;
        m = v > m ? v : m;
    }
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
        const double d = (double)(k - q + e);
        s += exp((double)in[k * stride] + (logw ? logw[k] : 0.0) - d * d * invk - m);
    }
    return m + log(s);
}

// One workgroup per composite cell.  LDS: b box [W1][W2p] (T), U0/U2 [W1][xside+1] (double),
// log y1 [W1], log y2 [W2] (double).
template <typename T>
__global__ void __launch_bounds__(kT)
    cell_eval_kernel(int ncell, int xside, int s, int maxw1, int maxw2,
                     const int32_t* __restrict__ members, const int32_t* __restrict__ xorig,
                     const int32_t* __restrict__ cdims, const int32_t* __restrict__ corig,
                     const int32_t* __restrict__ cshift, const int32_t* __restrict__ gofs,
                     const int64_t* __restrict__ cbase, const T* __restrict__ logmu,
                     const T* __restrict__ a, const T* __restrict__ b,
                     const T* __restrict__ lognuJ, const double* __restrict__ nuJ, const double* __restrict__ lognu_glob, int N,
                     double kappa, double* cell_out /*[ncell][4]*/, double* basic_out /*[nI][3]*/,
                     double* pix_out /*[N*N][3] or null*/) {
    extern __shared__ __align__(16) char smem[];
    double* red = reinterpret_cast<double*>(smem);
    double* u0 = red + 8;
    double* u2 = u0 + (size_t)maxw1 * (xside + 1);
    double* ly1 = u2 + (size_t)maxw1 * (xside + 1);
    double* ly2 = ly1 + maxw1;
    T* sb = reinterpret_cast<T*>(ly2 + maxw2);
    const int W2p = maxw2 + 1, ASp = xside + 1, N2 = xside * xside;
    const double invk = 1.0 / kappa;
    for (int J = blockIdx.x; J < ncell; J += gridDim.x) {
        const int W1 = cdims[2 * J], W2 = cdims[2 * J + 1];
        const int E1 = cshift[2 * J], E2 = cshift[2 * J + 1];
        const int G1 = gofs[2 * J], G2 = gofs[2 * J + 1];
        const int lo1 = corig[2 * J], lo2 = corig[2 * J + 1];
        const int px1 = xorig[2 * J], px2 = xorig[2 * J + 1];
        const int64_t cb = cbase[J];
        __syncthreads();
        for (int o = threadIdx.x; o < W1 * W2; o += blockDim.x) {
            const int j1 = o / W2, j2 = o - j1 * W2;
            sb[j1 * W2p + j2] = b[cb + o] + lognuJ[cb + o];  // z = g + log nu_J
        }
        for (int j = threadIdx.x; j < W1; j += blockDim.x) ly1[j] = log(lo1 + j + 0.5);
        for (int j = threadIdx.x; j < W2; j += blockDim.x) ly2[j] = log(lo2 + j + 0.5);
        __syncthreads();
        // Y side of E: sum_y nu_J beta/eps - sum_y nu_J with
        // beta/eps = g - 2<G, j>/kappa + log nu_J - log nu (reference mu (x) nu)
        double ey = 0.0, ty = 0.0, my = 0.0;
        for (int o = threadIdx.x; o < W1 * W2; o += blockDim.x) {
            const double v = nuJ[cb + o];
            if (v > 0.0) {
                const int j1 = o / W2, j2 = o - j1 * W2;
                const double bf = (double)b[cb + o] + log(v) -
                                  2.0 * (G1 * (double)j1 + G2 * (double)j2) * invk;
                ey += v * (bf - lognu_glob[(int64_t)(lo1 + j1) * N + (lo2 + j2)]);
                my += v;
                const double y1 = lo1 + j1 + 0.5, y2 = lo2 + j2 + 0.5;
                ty += v * (y1 * y1 + y2 * y2);
            }
        }
        // X half with weights 1 and y2 along j2, then 1, y1, y2 along j1
        for (int o = threadIdx.x; o < W1 * xside; o += blockDim.x) {
            const int j1 = o / xside, i2 = o - j1 * xside;
            u0[j1 * ASp + i2] = lse_w(sb + j1 * W2p, 1, W2, i2, -E2, invk, nullptr);
            u2[j1 * ASp + i2] = lse_w(sb + j1 * W2p, 1, W2, i2, -E2, invk, ly2);
        }
        __syncthreads();
        double ex = 0.0, tx = 0.0, err = 0.0;
        double bm0[4] = {0, 0, 0, 0}, bx2[4] = {0, 0, 0, 0}, bxy[4] = {0, 0, 0, 0};
        for (int il = threadIdx.x; il < N2; il += blockDim.x) {
            const int i1 = il / xside, i2 = il - i1 * xside;
            const double lm = (double)logmu[(int64_t)J * N2 + il];
            if (lm <= kZeroMassLog) continue;
            const double s0 = lse_w(u0 + i2, ASp, W1, i1, -E1, invk, nullptr);
            const double s1 = lse_w(u0 + i2, ASp, W1, i1, -E1, invk, ly1);
            const double s2 = lse_w(u2 + i2, ASp, W1, i1, -E1, invk, nullptr);
            const double av = (double)a[(int64_t)J * N2 + il];
            const double m0 = exp(av + lm + s0), m1 = exp(av + lm + s1), m2 = exp(av + lm + s2);
            const double mu = exp(lm);
            err += fabs(m0 - mu);
            // alpha/eps = f + (2<G,E> + |G|^2 + 2<G,i>)/kappa
            const double af = av + (2.0 * (G1 * (double)E1 + G2 * (double)E2) + (double)G1 * G1 +
                                    (double)G2 * G2 + 2.0 * (G1 * (double)i1 + G2 * (double)i2)) * invk;
            ex += m0 * af;
            const double x1 = px1 + i1 + 0.5, x2 = px2 + i2 + 0.5;
            const double xx = x1 * x1 + x2 * x2;
            const double xy = x1 * m1 + x2 * m2;
            tx += xx * m0 - 2.0 * xy;
            if (pix_out) {
                // the per-pixel X moments of the plan (gluing edge candidates of the flow update)
                const int64_t px = (int64_t)(px1 + i1) * N + (px2 + i2);
                pix_out[3 * px] = m0;
                pix_out[3 * px + 1] = m1;
                pix_out[3 * px + 2] = m2;
            }
            const int k = (i1 >= s ? 2 : 0) + (i2 >= s ? 1 : 0);
            bm0[k] += m0;
            bx2[k] += xx * m0;
            bxy[k] += xy;
        }
        const double Ey = block_sum(ey, red), My = block_sum(my, red), Ty = block_sum(ty, red);
        const double Ex = block_sum(ex, red), Tx = block_sum(tx, red), Er = block_sum(err, red);
        if (threadIdx.x == 0) {
            cell_out[4 * J] = Ex + Ey - My;  // E(pi_J)/eps without the +1 of KL's reference mass
            cell_out[4 * J + 1] = Tx + Ty;   // <c, pi_J> in pixel units
            cell_out[4 * J + 2] = Er;        // X-marginal L1 error
            cell_out[4 * J + 3] = My;        // mass
        }
        for (int k = 0; k < 4; ++k) {
            const double q0 = block_sum(bm0[k], red), q1 = block_sum(bx2[k], red),
                         q2 = block_sum(bxy[k], red);
            const int i = members[4 * J + k];
            if (threadIdx.x == 0 && i >= 0 && basic_out) {
                basic_out[3 * i] = q0;
                basic_out[3 * i + 1] = q1;
                basic_out[3 * i + 2] = q2;
            }
        }
    }
}

__global__ void sum4_kernel(int n, const double* v, double* out) {
    __shared__ double red[8];
    double s[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        for (int k = 0; k < 4; ++k) s[k] += v[4 * i + k];
    for (int k = 0; k < 4; ++k) {
        const double t = block_sum(s[k], red);
        if (threadIdx.x == 0) out[k] = t;
    }
}

}  // namespace

void launch_fill(double* p, size_t n, double v, hipStream_t st) {
    const size_t nb = std::min<size_t>((n + kT - 1) / kT, 8192);
    fill_kernel<<<std::max<size_t>(nb, 1), kT, 0, st>>>(p, n, v);
}

void launch_ymarg(int nI, const int32_t* box, const int64_t* base, const double* data, int N,
                  double* acc, const double* nu, double* out, hipStream_t st) {
    launch_fill(acc, (size_t)N * N, 0.0, st);
    ymarg_kernel<<<std::max(1, std::min(nI, 4096)), kT, 0, st>>>(nI, box, base, data, N, acc);
    l1diff_kernel<<<1, kT, 0, st>>>((int64_t)N * N, acc, nu, out);
}

void launch_basic_mass(int nI, const int64_t* base, const double* data, const double* m,
                       double* per_cell, double* out, hipStream_t st) {
    basic_mass_kernel<<<std::max(1, std::min(nI, 4096)), kT, 0, st>>>(nI, base, data, m, per_cell);
    mass_summary_kernel<<<1, kT, 0, st>>>(nI, per_cell, m, out);
}

size_t cell_eval_lds(int xside, int maxw1, int maxw2, size_t elem) {
    return 64 + sizeof(double) * (2 * (size_t)maxw1 * (xside + 1) + maxw1 + maxw2) +
           elem * (size_t)maxw1 * (maxw2 + 1);
}

void launch_cell_eval(const EvalArgs& e, hipStream_t st) {
    const size_t lds = cell_eval_lds(e.xside, e.maxw1, e.maxw2, sizeof(double));
    auto k = cell_eval_kernel<double>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k<<<std::max(1, std::min(e.ncell, 4096)), kT, lds, st>>>(
        e.ncell, e.xside, e.s, e.maxw1, e.maxw2, e.members, e.xorig, e.cdims, e.corig, e.cshift,
        e.gofs, e.cbase, e.logmu, e.a, e.b, e.lognuJ, e.nuJ, e.lognu_glob, e.N, e.kappa, e.cell_out,
        e.basic_out, e.pix_out);
    sum4_kernel<<<1, kT, 0, st>>>(e.ncell, e.cell_out, e.totals);
}


}  // namespace dd
