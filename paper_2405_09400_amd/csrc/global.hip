// Global log-domain Sinkhorn on the whole N x N grid: the problem of Sec. 2.2 eq.
// (entropic-transport) solved without domain decomposition, the comparison solver of App. A.2.1
// ("Compared algorithms and implementations": a global batched Sinkhorn on the GPU).
//
// It is the single-cell problem X = Y = the grid, with the same iteration, stopping rule and
// float64 arithmetic as the cell solver's float64 path: potentials f = alpha/eps, g = beta/eps
// with reference measure mu (x) nu, the squared-Euclidean cost |k - l|^2 / kappa in pixel units
// (kappa = eps / h^2), every log-sum-exp as two 1D passes (the cost is separable), each pass
// an exact two-sweep log-sum-exp per output (the running maximum, then the sum of exponentials
// below it).  A pass reads its input lines from LDS and writes its outputs transposed, so that
// the second pass of a half-iteration again reads contiguous lines:
//   Y-update:  T[y2][x1] = LSE_x2 [f(x1,x2) + log mu(x1,x2) - (x2 - y2)^2 / kappa]
//              g(y1,y2)  = -LSE_x1 [T[y2][x1] - (x1 - y1)^2 / kappa]
//   X-update:  the same with g + log nu as input; err = sum_x mu |exp(f + s) - 1| with s the
//              pre-update LSE, and f = -s unless the solve stops.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace dd {
namespace {

constexpr int kT = 256;
constexpr int kLines = 4;  // input lines per workgroup

// out[q * N + a] = LSE_k [sgn * in[a * N + k] + add[a * N + k] - (k - q)^2 invk] for the lines
// a of this workgroup and every output q; entries at or below the zero-mass sentinel count as
// zero mass, and an output with none gets the sentinel.
__global__ void __launch_bounds__(kT)
    lse_rows_t_kernel(int N, const double* __restrict__ in, double sgn,
                      const double* __restrict__ add, double invk, double* __restrict__ out) {
    extern __shared__ double line[];
    const int a0 = blockIdx.x * kLines;
    for (int t = threadIdx.x; t < kLines * N; t += kT) {
        const int l = t / N, k = t - l * N;
        const int a = a0 + l;
        double v = kNegD;
        if (a < N) {
            const double ad = add ? add[(int64_t)a * N + k] : 0.0;
            const double x = in[(int64_t)a * N + k];
            v = (ad <= kZeroMassLog || (sgn > 0.0 ? x : -x) <= kZeroMassLog) ? kNegD : sgn * x + ad;
        }
        line[t] = v;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < kLines * N; o += kT) {
        const int l = o % kLines, q = o / kLines;
        const int a = a0 + l;
        if (a >= N) continue;
        const double* L = line + l * N;
        double m = kNegD;
        for (int k = 0; k < N; ++k) {
            const double d = k - q;
            if (L[k] > kZeroMassLog) m = fmax(m, L[k] - d * d * invk);
        }
        double r = kNegD;
        if (m > kZeroMassLog) {
            double s = 0.0;
            for (int k = 0; k < N; ++k) {
                const double d = k - q;
                if (L[k] > kZeroMassLog) s += exp(L[k] - d * d * invk - m);
            }
            r = m + log(s);
        }
        out[(int64_t)q * N + a] = r;
    }
}

// per-workgroup partial sums of mu |exp(f + s) - 1| (zero-mass pixels excluded); the host adds
// the partials in order
__global__ void __launch_bounds__(kT)
    xerr_kernel(int64_t N2, const double* __restrict__ mu, const double* __restrict__ f,
                const double* __restrict__ s, double* __restrict__ part) {
    __shared__ double red[kT / 64];
    double e = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kT + threadIdx.x; k < N2; k += (int64_t)gridDim.x * kT)
        if (mu[k] > 0.0) e += mu[k] * fabs(expm1(f[k] + s[k]));
    e = block_sum(e, red);
    if (threadIdx.x == 0) part[blockIdx.x] = e;
}

__global__ void neg_kernel(int64_t n, const double* __restrict__ in, double* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = in[k] <= kZeroMassLog ? kNegD : -in[k];
}

// f = alpha / eps (scale = 1/eps) or alpha = eps f (scale = eps); log of a measure.
__global__ void scale_kernel(int64_t n, const double* __restrict__ in, double scale,
                             double* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = in[k] * scale;
}
__global__ void log_kernel(int64_t n, const double* __restrict__ in, double* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = in[k] > 0.0 ? log(in[k]) : kNegD;
}

constexpr int kParts = 512;

struct GlobalWork {
    double *lmu = nullptr, *lnu = nullptr, *f = nullptr, *G = nullptr, *T = nullptr,
           *S = nullptr, *part = nullptr;
    ~GlobalWork() {
        for (double* p : {lmu, lnu, f, G, T, S, part})
            if (p) (void)hipFree(p);
    }
};

}  // namespace
}  // namespace dd

extern "C" dd_status global_sinkhorn(int32_t n, const double* mu, const double* nu, double eps,
                                     double* alpha, double* beta, const dd_sinkhorn_opts* opts,
                                     void* stream, dd_global_stats* stats) {
    using namespace dd;
    if (!mu || !nu || !alpha || !beta || !opts) {
        set_global_error("global_sinkhorn: null argument");
        return DD_EINVAL;
    }
    if (n < 1 || n > 4096 || !(eps > 0.0) || !std::isfinite(eps) || opts->max_iter < 1 ||
        opts->fixed_iters < 0 || !(opts->tol >= 0.0)) {
        set_global_error("global_sinkhorn: need 1 <= n <= 4096, eps > 0, max_iter >= 1, tol >= 0");
        return DD_EINVAL;
    }
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t N2 = (int64_t)n * n;
    const double h = 1.0 / n, kappa = eps / (h * h), invk = 1.0 / kappa;
    GlobalWork w;
    Status S;
    auto dev = [&](double*& p, size_t cnt) -> bool {
        return hipMalloc(&p, std::max<size_t>(cnt, 1) * sizeof(double)) == hipSuccess;
    };
    if (!dev(w.lmu, N2) || !dev(w.lnu, N2) || !dev(w.f, N2) || !dev(w.G, N2) || !dev(w.T, N2) ||
        !dev(w.S, N2) || !dev(w.part, kParts)) {
        set_global_error("global_sinkhorn: device allocation failed");
        return DD_ENOMEM;
    }
    const size_t lds = (size_t)kLines * n * sizeof(double);
    if (lds > 160 * 1024 ||
        hipFuncSetAttribute((const void*)lse_rows_t_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        set_global_error("global_sinkhorn: grid too large for the LDS of a workgroup");
        return DD_EINVAL;
    }
    const int eg = (int)std::min<int64_t>((N2 + kT - 1) / kT, 4096);
    const int lg = (n + kLines - 1) / kLines;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, st);
    log_kernel<<<eg, kT, 0, st>>>(N2, mu, w.lmu);
    log_kernel<<<eg, kT, 0, st>>>(N2, nu, w.lnu);
    scale_kernel<<<eg, kT, 0, st>>>(N2, alpha, 1.0 / eps, w.f);
    const bool fixed = opts->fixed_iters > 0;
    const int limit = fixed ? opts->fixed_iters : opts->max_iter;
    std::vector<double> part(kParts);
    double err = NAN;
    int it = 0;
    bool conv = false;
    while (true) {
        // Y-update: G = LSE_x [f + log mu - C], g = -G
        lse_rows_t_kernel<<<lg, kT, lds, st>>>(n, w.f, 1.0, w.lmu, invk, w.T);
        lse_rows_t_kernel<<<lg, kT, lds, st>>>(n, w.T, 1.0, nullptr, invk, w.G);
        ++it;
        // X side: s = LSE_y [g + log nu - C], error, then f = -s unless stopping
        lse_rows_t_kernel<<<lg, kT, lds, st>>>(n, w.G, -1.0, w.lnu, invk, w.T);
        lse_rows_t_kernel<<<lg, kT, lds, st>>>(n, w.T, 1.0, nullptr, invk, w.S);
        xerr_kernel<<<kParts, kT, 0, st>>>(N2, mu, w.f, w.S, w.part);
        if (hipMemcpyAsync(part.data(), w.part, kParts * sizeof(double), hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_global_error("global_sinkhorn: a kernel failed");
            return DD_EDEVICE;
        }
        err = 0.0;
        for (double v : part) err += v;
        if (!std::isfinite(err)) {
            set_global_error("global_sinkhorn: non-finite marginal error");
            return DD_ENUMERIC;
        }
        conv = fixed ? it >= limit : err <= opts->tol;
        if (conv || it >= limit) break;
        neg_kernel<<<eg, kT, 0, st>>>(N2, w.S, w.f);
    }
    // alpha = eps f; beta = eps g = -eps G
    scale_kernel<<<eg, kT, 0, st>>>(N2, w.f, eps, alpha);
    neg_kernel<<<eg, kT, 0, st>>>(N2, w.G, w.T);
    scale_kernel<<<eg, kT, 0, st>>>(N2, w.T, eps, beta);
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        set_global_error("global_sinkhorn: a kernel failed");
        return DD_EDEVICE;
    }
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) {
        *stats = dd_global_stats{};
        stats->iters = it;
        stats->converged = conv ? 1 : 0;
        stats->err = err;
        stats->time_ms = ms;
        stats->lse_terms = 4.0 * (double)it * (double)N2 * n;
    }
    if (!conv) {
        set_global_error("global_sinkhorn: iteration limit reached before the tolerance");
        return DD_NOTCONV;
    }
    return DD_OK;
}
