// Stitched global dual point of a domain-decomposition state and its dual value (the
// primal-dual gap of App. A.2.2 needs a dual point for the whole problem).
//
// Each composite cell carries its own X potential, defined up to a constant (the gauge of
// the cell problem, Sec. 2.3).  With the A and B cells as the nodes of a graph whose edges
// are their overlaps (one basic cell each), a breadth-first walk from A cell 0 (offset 0)
// fixes the constants so that the mu-weighted means of the two partitions' potentials agree
// on every tree edge's basic cell; cells are expanded in FIFO order and neighbours reached
// through their members in ascending basic-cell order.  alpha+ is the offset A potential;
// beta+ is its exact Y-update against mu (x) nu over the whole grid (a separable global
// log-sum-exp, two 1D passes), so that D = <alpha+, mu> + <beta+, nu>.
//
// In units of eps: a cell's solved potential f (box-local gauge) is alpha/eps - 2<G, i>/kappa
// up to a constant, G the gauge offset of its last solve; a partition last solved at another
// eps is rescaled to the evaluation's eps (alpha is in energy units).
#include "dual.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace dd {

namespace {

constexpr int kT = 256;

int grid_n(long n, int cap) { return (int)std::max(1L, std::min<long>(n, cap)); }

// alpha/eps of every pixel covered by a partition, from the cells' potentials and gauges.
__global__ void alpha_glob_kernel(int ncell, int xside, int N, const int32_t* __restrict__ xorig,
                                  const double* __restrict__ a, const int32_t* __restrict__ gst,
                                  double two_invk, double scale, double* __restrict__ out) {
    const int N2 = xside * xside;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)ncell * N2;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int J = (int)(t / N2), i = (int)(t - (int64_t)J * N2);
        const int i1 = i / xside, i2 = i - i1 * xside;
        const int k1 = xorig[2 * J] + i1, k2 = xorig[2 * J + 1] + i2;
        if (k1 < 0 || k1 >= N || k2 < 0 || k2 >= N) continue;
        out[(int64_t)k1 * N + k2] =
            scale * (a[t] + two_invk * ((double)gst[2 * J] * i1 + (double)gst[2 * J + 1] * i2));
    }
}

// d[i] = sum_{x in X_i} mu (fA - fB) / sum_{x in X_i} mu for every basic cell.
__global__ void basic_diff_kernel(int n, int s, int N, const double* __restrict__ mu,
                                  const double* __restrict__ fA, const double* __restrict__ fB,
                                  double* __restrict__ d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += gridDim.x * blockDim.x) {
        const int r = i / n, c = i - r * n;
        double sw = 0.0, swd = 0.0;
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b) {
                const int64_t k = (int64_t)(r * s + a) * N + c * s + b;
                sw += mu[k];
                swd += mu[k] * (fA[k] - fB[k]);
            }
        d[i] = swd / sw;
    }
}

// w = alpha+/eps + log mu (the offset A potential; zero-mass pixels get the sentinel), and
// alpha+/eps itself.
__global__ void alpha_dag_kernel(int n, int s, int N, const double* __restrict__ mu,
                                 const double* __restrict__ fA, const int32_t* __restrict__ ownA,
                                 const double* __restrict__ sA, double* __restrict__ fdag,
                                 double* __restrict__ w) {
    const int64_t N2 = (int64_t)N * N;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N2;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int k1 = (int)(k / N), k2 = (int)(k - (int64_t)k1 * N);
        const int i = (k1 / s) * n + k2 / s;
        const double f = fA[k] - sA[ownA[i]];
        fdag[k] = f;
        w[k] = mu[k] > 0.0 ? f + log(mu[k]) : kNegD;
    }
}

// T[x1][y2] = LSE_{x2} [w[x1][x2] - (x2 - y2)^2 / kappa]
__global__ void gy_pass1_kernel(int N, const double* __restrict__ w, double invk,
                                double* __restrict__ T) {
    const int64_t N2 = (int64_t)N * N;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < N2;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int x1 = (int)(o / N), y2 = (int)(o - (int64_t)x1 * N);
        const double* row = w + (int64_t)x1 * N;
        double m = -1e300;
        for (int x2 = 0; x2 < N; ++x2) {
            const double d = x2 - y2;
            m = fmax(m, row[x2] - d * d * invk);
        }
        double sum = 0.0;
        for (int x2 = 0; x2 < N; ++x2) {
            const double d = x2 - y2;
            sum += exp(row[x2] - d * d * invk - m);
        }
        T[o] = m + log(sum);
    }
}

// g[y1][y2] = -LSE_{x1} [T[x1][y2] - (x1 - y1)^2 / kappa]
__global__ void gy_pass2_kernel(int N, const double* __restrict__ T, double invk,
                                double* __restrict__ g) {
    const int64_t N2 = (int64_t)N * N;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < N2;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int y1 = (int)(o / N), y2 = (int)(o - (int64_t)y1 * N);
        double m = -1e300;
        for (int x1 = 0; x1 < N; ++x1) {
            const double d = x1 - y1;
            m = fmax(m, T[(int64_t)x1 * N + y2] - d * d * invk);
        }
        double sum = 0.0;
        for (int x1 = 0; x1 < N; ++x1) {
            const double d = x1 - y1;
            sum += exp(T[(int64_t)x1 * N + y2] - d * d * invk - m);
        }
        g[o] = -(m + log(sum));
    }
}

// per-block partial sums of mu f+ + nu g+ (nu > 0 only); the host adds the partials in order
__global__ void __launch_bounds__(kT)
    dual_sum_kernel(int64_t N2, const double* __restrict__ mu, const double* __restrict__ f,
                    const double* __restrict__ nu, const double* __restrict__ g,
                    double* __restrict__ part) {
    __shared__ double red[8];
    double s = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kT + threadIdx.x; k < N2; k += (int64_t)gridDim.x * kT) {
        if (mu[k] > 0.0) s += mu[k] * f[k];
        if (nu[k] > 0.0) s += nu[k] * g[k];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

Status stitched_alpha(const DualArgs& a, DualWork& w, hipStream_t st, const double** fdag_out) {
    Status S;
    const int N = a.N, s = a.s, n = N / s;
    const int64_t N2 = (int64_t)N * N;
    const int nI = n * n;
    constexpr int kParts = 1024;
    if (!w.buf) {
        DD_HIP(w.mem.get(&w.buf, (size_t)5 * N2 * sizeof(double)), S);
        DD_HIP(w.mem.get(&w.d, (size_t)nI * sizeof(double)), S);
        DD_HIP(w.mem.get(&w.own, (size_t)nI * sizeof(int32_t)), S);
        DD_HIP(w.mem.get(&w.sA, (size_t)a.ncell[0] * sizeof(double)), S);
        DD_HIP(w.mem.get(&w.part, kParts * sizeof(double)), S);
    }
    double* fA = w.buf;
    double* fB = w.buf + N2;
    double* fdag = w.buf + 2 * N2;
    double* wv = w.buf + 3 * N2;
    const double two_invk[2] = {2.0 / a.kappa[0], 2.0 / a.kappa[1]};
    double* fx[2] = {fA, fB};
    for (int q = 0; q < 2; ++q)
        alpha_glob_kernel<<<grid_n((long)a.ncell[q] * a.xside * a.xside / kT + 1, 4096), kT, 0,
                            st>>>(a.ncell[q], a.xside, N, a.xorig[q], a.a[q], a.gst[q],
                                  two_invk[q], a.kappa[q] / a.kappa_eval, fx[q]);
    basic_diff_kernel<<<grid_n(nI / kT + 1, 4096), kT, 0, st>>>(n, s, N, a.mu, fA, fB, w.d);
    std::vector<double> d(nI);
    DD_HIP(hipMemcpyAsync(d.data(), w.d, nI * sizeof(double), hipMemcpyDeviceToHost, st), S);
    DD_HIP(hipStreamSynchronize(st), S);
    // breadth-first offsets over the A/B overlap graph
    const int nA = a.ncell[0], nB = a.ncell[1];
    std::vector<int32_t> ownA(nI, -1), ownB(nI, -1);
    for (int J = 0; J < nA; ++J)
        for (int k = 0; k < 4; ++k)
            if (a.members[0][4 * J + k] >= 0) ownA[a.members[0][4 * J + k]] = J;
    for (int J = 0; J < nB; ++J)
        for (int k = 0; k < 4; ++k)
            if (a.members[1][4 * J + k] >= 0) ownB[a.members[1][4 * J + k]] = J;
    std::vector<double> sA(nA, NAN), sB(nB, NAN);
    std::vector<std::pair<int, int>> queue;
    queue.reserve(nA + nB);
    sA[0] = 0.0;
    queue.emplace_back(0, 0);
    for (size_t head = 0; head < queue.size(); ++head) {
        const int q = queue[head].first, J = queue[head].second;
        int mem[4];
        for (int k = 0; k < 4; ++k) mem[k] = a.members[q][4 * J + k];
        std::sort(mem, mem + 4);
        for (int i : mem) {
            if (i < 0) continue;
            if (q == 0) {
                const int K = ownB[i];
                if (K >= 0 && std::isnan(sB[K])) {
                    sB[K] = sA[J] - d[i];
                    queue.emplace_back(1, K);
                }
            } else {
                const int K = ownA[i];
                if (K >= 0 && std::isnan(sA[K])) {
                    sA[K] = sB[J] + d[i];
                    queue.emplace_back(0, K);
                }
            }
        }
    }
    for (int J = 0; J < nA; ++J)
        if (std::isnan(sA[J])) {
            S.code = DD_ENUMERIC;
            S.msg = "stitched dual: the overlap graph does not reach every A cell";
            return S;
        }
    DD_HIP(hipMemcpyAsync(w.own, ownA.data(), nI * sizeof(int32_t), hipMemcpyHostToDevice, st), S);
    DD_HIP(hipMemcpyAsync(w.sA, sA.data(), nA * sizeof(double), hipMemcpyHostToDevice, st), S);
    alpha_dag_kernel<<<grid_n(N2 / kT + 1, 8192), kT, 0, st>>>(n, s, N, a.mu, fA, w.own, w.sA,
                                                              fdag, wv);
    *fdag_out = fdag;
    return S;
}

Status stitched_dual(const DualArgs& a, DualWork& w, hipStream_t st, double* D) {
    const double* fdag_c = nullptr;
    Status S = stitched_alpha(a, w, st, &fdag_c);
    if (S.code) return S;
    const int N = a.N;
    const int64_t N2 = (int64_t)N * N;
    constexpr int kParts = 1024;
    double* fB = w.buf + N2;
    double* fdag = w.buf + 2 * N2;
    double* wv = w.buf + 3 * N2;
    double* T = w.buf + 4 * N2;
    const double invk = 1.0 / a.kappa_eval;
    gy_pass1_kernel<<<grid_n(N2 / kT + 1, 8192), kT, 0, st>>>(N, wv, invk, T);
    double* g = fB;  // fB is no longer needed
    gy_pass2_kernel<<<grid_n(N2 / kT + 1, 8192), kT, 0, st>>>(N, T, invk, g);
    dual_sum_kernel<<<kParts, kT, 0, st>>>(N2, a.mu, fdag, a.nu, g, w.part);
    std::vector<double> part(kParts);
    DD_HIP(hipMemcpyAsync(part.data(), w.part, kParts * sizeof(double), hipMemcpyDeviceToHost, st),
           S);
    DD_HIP(hipStreamSynchronize(st), S);
    double tot = 0.0;
    for (double v : part) tot += v;
    *D = a.eps * tot;
    return S;
}

void dual_release(DualWork& w) {
    for (void* p : {(void*)w.buf, (void*)w.d, (void*)w.own, (void*)w.sA, (void*)w.part})
        w.mem.put(p);
    const Mem m = w.mem;
    w = DualWork{};
    w.mem = m;
}

}  // namespace dd
