// Domain-decomposition context: setup, one DD iteration, plan extraction and evaluation.
//
// Alg. "DomDecIter" as App. A Alg. "DomDecIterGPU" lays it out, with all composite cells of
// a partition in one batch (no CreateBatches / CombineBatches loop):
//   BasicToComposite -> warm start -> batched cell Sinkhorn -> CompositeToBasic ->
//   balancing -> truncation and repacking.
// The state is the set of basic-cell Y-marginals nu_i in per-cell bounding boxes on the
// device (float64).  The host only reads back a few sizes per iteration (to size buffers
// and the solver's LDS tiles) and the statistics.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "cells.hpp"
#include "ctx.hpp"
#include "eval.hpp"
#include "net.hpp"
#include "sinkhorn.hpp"

using namespace dd;

namespace {

template <typename P>
Status grow(const Mem& M, P*& p, size_t& cap, size_t need, Status& st, double slack = 1.25) {
    if (need <= cap && p) return st;
    M.put(p);
    p = nullptr;
    const size_t n = std::max<size_t>((size_t)(need * slack) + 16, 64);
    DD_HIP(M.get(&p, n * sizeof(P)), st);
    cap = n;
    return st;
}

template <typename P>
Status alloc(const Mem& M, P*& p, size_t n, Status& st) {
    DD_HIP(M.get(&p, std::max<size_t>(n, 1) * sizeof(P)), st);
    return st;
}

template <typename P>
Status upload(const Mem& M, P*& p, const std::vector<P>& v, hipStream_t s, Status& st) {
    if (alloc(M, p, v.size(), st).code) return st;
    if (!v.empty()) {
        // the host vector may be a temporary: finish the copy before returning
        DD_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(P), hipMemcpyHostToDevice, s), st);
        DD_HIP(hipStreamSynchronize(s), st);
    }
    return st;
}

dd_status fail(dd_ctx* c, dd_status code, const std::string& m) {
    if (c) c->err = m;
    set_global_error(m);
    return code;
}

dd_status fail(dd_ctx* c, const Status& s) { return fail(c, s.code, s.msg); }

// every device buffer of the context, its solver workspace and its dual workspace from M
void use_mem(dd_ctx* c, const Mem& M) {
    c->mem = M;
    c->skw.mem = M;
    c->dual.mem = M;
}

}  // namespace

void dd_ctx_release(dd_ctx* c) {
    auto F = [c](auto& p) {
        c->mem.put(p);
        p = nullptr;
    };
    F(c->d_mu);
    F(c->d_nu);
    F(c->d_lognu_glob);
    F(c->d_m);
    for (int q = 0; q < 2; ++q) {
        F(c->part[q].members);
        F(c->part[q].xorig);
        F(c->d_logmu[q]);
        F(c->d_a[q]);
        F(c->d_gst[q]);
    }
    for (BoxSet* S : {&c->S, &c->S2}) {
        F(S->box);
        F(S->base);
        F(S->data);
    }
    F(c->C.dims);
    F(c->C.orig);
    F(c->C.shift);
    F(c->C.gofs);
    F(c->C.size);
    F(c->C.base);
    F(c->C.info);
    F(c->d_nuJ);
    F(c->d_lognu);
    F(c->d_b);
    F(c->d_nx);
    F(c->d_ng);
    F(c->d_a0);
    dual_release(c->dual);
    F(c->snap.box);
    F(c->snap.base);
    F(c->snap.data);
    for (int q = 0; q < 2; ++q) {
        F(c->snap.a[q]);
        F(c->snap.gst[q]);
    }
    F(c->d_tmp);
    F(c->d_py2);
    F(c->d_nsize);
    F(c->d_flags);
    F(c->d_iters);
    F(c->d_cerr);
    F(c->d_scratch);
    F(c->d_cell_out);
    F(c->d_basic_out);
    F(c->d_eval);
    for (int q = 0; q < 2; ++q) {
        F(c->d_pred[q]);
        if (c->h_pred[q]) (void)hipHostFree(c->h_pred[q]);
        c->h_pred[q] = nullptr;
    }
    F(c->d_pcheck);
    dd_forget_pred(c);
    for (int32_t** q : {&c->bt.C.dims, &c->bt.C.orig, &c->bt.C.shift, &c->bt.C.gofs, &c->bt.C.info,
                        &c->bt.idx, &c->bt.members, &c->bt.xorig, &c->bt.gst, &c->bt.list})
        F(*q);
    F(c->bt.C.size);
    F(c->bt.C.base);
    F(c->bt.a);
    F(c->bt.logmu);
    F(c->bt.lsize);
    F(c->bt.stage_base);
    F(c->bt.staging);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->h_small) (void)hipHostFree(c->h_small);
    c->h_small = nullptr;
    sk_work_release(c->skw);
    flow_release(c);
}

namespace {

// Everything of a layer but its coupling: grid, basic-cell masses, both partitions (members,
// X origins, log mu on the padded blocks, zero potentials), mu, nu and log nu on the device,
// and the work buffers sized by the layer.  c->s, prec, trunc and st are set by the caller.
Status setup_layer(dd_ctx* c, int N, const double* mu, const double* nu) {
    Status st;
    const int s = c->s;
    c->N = N;
    c->n = N / s;
    c->nI = c->n * c->n;
    c->AS = 2 * s;
    c->h = 1.0 / N;
    const hipStream_t hs = c->st;
    const int64_t NN = (int64_t)N * N;
    for (auto& e : c->ev)
        if (!e) DD_HIP(hipEventCreate(&e), st);
    const int n = c->n, AS = c->AS;
    // basic cell masses (pixel order inside the block, row-major)
    c->m.assign(c->nI, 0.0);
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) {
            double t = 0.0;
            for (int a = 0; a < s; ++a)
                for (int b = 0; b < s; ++b) t += mu[(int64_t)(r * s + a) * N + (q * s + b)];
            c->m[r * n + q] = t;
            if (!(t > 0.0)) {
                st.code = DD_EINVAL;
                st.msg = "domdec_init: every basic cell needs positive mass";
                return st;
            }
        }
    // partitions
    for (int q = 0; q < 2; ++q) {
        const int nc = q == 0 ? n / 2 : n / 2 + 1;
        const int off = q == 0 ? 0 : -1;
        std::vector<int32_t> mem, xo;
        std::vector<double> lm;
        for (int R = 0; R < nc; ++R)
            for (int Cc = 0; Cc < nc; ++Cc) {
                for (int dr = 0; dr < 2; ++dr)
                    for (int dc = 0; dc < 2; ++dc) {
                        const int r = 2 * R + off + dr, cc = 2 * Cc + off + dc;
                        mem.push_back((r >= 0 && r < n && cc >= 0 && cc < n) ? r * n + cc : -1);
                    }
                const int p1 = (2 * R + off) * s, p2 = (2 * Cc + off) * s;
                xo.push_back(p1);
                xo.push_back(p2);
                for (int i1 = 0; i1 < AS; ++i1)
                    for (int i2 = 0; i2 < AS; ++i2) {
                        const int k1 = p1 + i1, k2 = p2 + i2;
                        double v = kNegD;
                        if (k1 >= 0 && k1 < N && k2 >= 0 && k2 < N && mu[(int64_t)k1 * N + k2] > 0)
                            v = std::log(mu[(int64_t)k1 * N + k2]);
                        lm.push_back(v);
                    }
            }
        c->part[q].ncell = nc * nc;
        c->pmembers[q] = mem;
        c->pxorig[q] = xo;
        if (upload(c->mem, c->part[q].members, mem, hs, st).code) return st;
        if (upload(c->mem, c->part[q].xorig, xo, hs, st).code) return st;
        if (upload(c->mem, c->d_logmu[q], lm, hs, st).code) return st;
        if (upload(c->mem, c->d_a[q], std::vector<double>(lm.size(), 0.0), hs, st).code) return st;
        if (upload(c->mem, c->d_gst[q], std::vector<int32_t>(2 * (size_t)nc * nc, 0), hs, st).code)
            return st;
    }
    std::vector<double> vmu(mu, mu + NN), vnu(nu, nu + NN), lnu(NN);
    for (int64_t k = 0; k < NN; ++k) lnu[k] = nu[k] > 0 ? std::log(nu[k]) : -INFINITY;
    if (upload(c->mem, c->d_mu, vmu, hs, st).code || upload(c->mem, c->d_nu, vnu, hs, st).code ||
        upload(c->mem, c->d_lognu_glob, lnu, hs, st).code || upload(c->mem, c->d_m, c->m, hs, st).code)
        return st;
    const int mc = std::max(c->part[0].ncell, c->part[1].ncell);
    if (alloc(c->mem, c->S.box, 4 * (size_t)c->nI, st).code || alloc(c->mem, c->S.base, c->nI + 1, st).code ||
        alloc(c->mem, c->S2.box, 4 * (size_t)c->nI, st).code || alloc(c->mem, c->S2.base, c->nI + 1, st).code ||
        alloc(c->mem, c->C.dims, 2 * (size_t)mc, st).code || alloc(c->mem, c->C.orig, 2 * (size_t)mc, st).code ||
        alloc(c->mem, c->C.shift, 2 * (size_t)mc, st).code || alloc(c->mem, c->C.gofs, 2 * (size_t)mc, st).code ||
        alloc(c->mem, c->C.size, mc, st).code || alloc(c->mem, c->C.base, mc + 1, st).code ||
        alloc(c->mem, c->C.info, 8, st).code || alloc(c->mem, c->d_py2, c->nI, st).code ||
        alloc(c->mem, c->d_nsize, c->nI, st).code || alloc(c->mem, c->d_flags, c->nI + 1, st).code ||
        alloc(c->mem, c->d_iters, mc, st).code || alloc(c->mem, c->d_cerr, mc, st).code ||
        alloc(c->mem, c->d_scratch, std::max<int64_t>(NN, c->nI), st).code ||
        alloc(c->mem, c->d_cell_out, 4 * (size_t)mc, st).code ||
        alloc(c->mem, c->d_basic_out, 3 * (size_t)c->nI, st).code || alloc(c->mem, c->d_eval, 8, st).code)
        return st;
    return st;
}

// The layer's basic-cell Y-marginals in bounding-box form from a host coupling: the product
// coupling nu_i = m_i nu (n_init == 0), or a sparse (x, y, mass) list with marginals mu, nu.
Status boxes_from_host(dd_ctx* c, const double* mu, const double* nu, int64_t n_init,
                       const int64_t* init_x, const int64_t* init_y, const double* init_m) {
    Status st;
    const int N = c->N, s = c->s, n = c->n;
    const int64_t NN = (int64_t)N * N;
    std::vector<int32_t> box(4 * (size_t)c->nI);
    std::vector<int64_t> base(c->nI + 1, 0);
    std::vector<double> data;
    if (n_init == 0) {
        int lo1 = N, lo2 = N, hi1 = -1, hi2 = -1;
        for (int k1 = 0; k1 < N; ++k1)
            for (int k2 = 0; k2 < N; ++k2)
                if (nu[(int64_t)k1 * N + k2] > 0) {
                    lo1 = std::min(lo1, k1);
                    hi1 = std::max(hi1, k1);
                    lo2 = std::min(lo2, k2);
                    hi2 = std::max(hi2, k2);
                }
        const int64_t w1 = hi1 - lo1 + 1, w2 = hi2 - lo2 + 1;
        if ((double)w1 * w2 * c->nI > 4.0e8) {
            st.code = DD_ENOMEM;
            st.msg = "domdec_init: the product coupling is too large here; pass a sparse init";
            return st;
        }
        data.resize((size_t)(w1 * w2 * c->nI));
        for (int i = 0; i < c->nI; ++i) {
            box[4 * i] = lo1;
            box[4 * i + 1] = lo2;
            box[4 * i + 2] = (int32_t)w1;
            box[4 * i + 3] = (int32_t)w2;
            base[i + 1] = base[i] + w1 * w2;
            for (int64_t r = 0; r < w1; ++r)
                for (int64_t q = 0; q < w2; ++q)
                    data[base[i] + r * w2 + q] = c->m[i] * nu[(lo1 + r) * N + (lo2 + q)];
        }
    } else {
        std::vector<double> px(NN, 0.0), py(NN, 0.0);
        std::vector<int32_t> cell(n_init);
        std::vector<int64_t> cnt(c->nI + 1, 0);
        for (int64_t e = 0; e < n_init; ++e) {
            const int64_t x = init_x[e], y = init_y[e];
            if (x < 0 || x >= NN || y < 0 || y >= NN || !(init_m[e] >= 0.0)) {
                st.code = DD_EINVAL;
                st.msg = "domdec_init: initial coupling entry out of range or negative";
                return st;
            }
            px[x] += init_m[e];
            py[y] += init_m[e];
            const int k1 = (int)(x / N), k2 = (int)(x % N);
            cell[e] = (k1 / s) * n + (k2 / s);
            cnt[cell[e] + 1]++;
        }
        for (int64_t k = 0; k < NN; ++k)
            if (std::fabs(px[k] - mu[k]) > 1e-12 || std::fabs(py[k] - nu[k]) > 1e-12) {
                st.code = DD_EINVAL;
                st.msg = "domdec_init: the initial coupling's marginals differ from mu, nu";
                return st;
            }
        for (int i = 0; i < c->nI; ++i) cnt[i + 1] += cnt[i];
        std::vector<int64_t> order(n_init), fill(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < n_init; ++e) order[fill[cell[e]]++] = e;
        for (int i = 0; i < c->nI; ++i) {
            int lo1 = N, lo2 = N, hi1 = -1, hi2 = -1;
            for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q) {
                const int64_t y = init_y[order[q]];
                const int y1 = (int)(y / N), y2 = (int)(y % N);
                lo1 = std::min(lo1, y1);
                hi1 = std::max(hi1, y1);
                lo2 = std::min(lo2, y2);
                hi2 = std::max(hi2, y2);
            }
            if (hi1 < 0) {
                st.code = DD_EINVAL;
                st.msg = "domdec_init: a basic cell has no mass in the initial coupling";
                return st;
            }
            const int w1 = hi1 - lo1 + 1, w2 = hi2 - lo2 + 1;
            box[4 * i] = lo1;
            box[4 * i + 1] = lo2;
            box[4 * i + 2] = w1;
            box[4 * i + 3] = w2;
            base[i + 1] = base[i] + (int64_t)w1 * w2;
        }
        data.assign((size_t)base[c->nI], 0.0);
        for (int i = 0; i < c->nI; ++i)
            for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q) {
                const int64_t e = order[q];
                const int y1 = (int)(init_y[e] / N), y2 = (int)(init_y[e] % N);
                data[base[i] + (int64_t)(y1 - box[4 * i]) * box[4 * i + 3] + (y2 - box[4 * i + 1])] +=
                    init_m[e];
            }
    }
    const hipStream_t hs = c->st;
    if (hipMemcpyAsync(c->S.box, box.data(), box.size() * 4, hipMemcpyHostToDevice, hs) !=
            hipSuccess ||
        hipMemcpyAsync(c->S.base, base.data(), base.size() * 8, hipMemcpyHostToDevice, hs) !=
            hipSuccess) {
        st.code = DD_EDEVICE;
        st.msg = "domdec_init: copying the initial coupling failed";
        return st;
    }
    if (upload(c->mem, c->S.data, data, hs, st).code) return st;
    c->S.cap = std::max<size_t>(data.size(), 1);
    DD_HIP(hipStreamSynchronize(hs), st);
    return st;
}

// 2 x 2 block sums of an N x N array.
std::vector<double> coarsen(const std::vector<double>& a, int N) {
    const int M = N / 2;
    std::vector<double> out((size_t)M * M);
    for (int r = 0; r < M; ++r)
        for (int q = 0; q < M; ++q)
            out[(size_t)r * M + q] = a[(size_t)(2 * r) * N + 2 * q] + a[(size_t)(2 * r) * N + 2 * q + 1] +
                                     a[(size_t)(2 * r + 1) * N + 2 * q] +
                                     a[(size_t)(2 * r + 1) * N + 2 * q + 1];
    return out;
}

}  // namespace

extern "C" dd_status domdec_init(const dd_params* prm, const double* mu, const double* nu,
                                 int64_t n_init, const int64_t* init_x, const int64_t* init_y,
                                 const double* init_m, void* stream, dd_ctx** out) {
    if (out) *out = nullptr;
    if (!prm || !mu || !nu || !out) return fail(nullptr, DD_EINVAL, "domdec_init: null argument");
    const int N = prm->n, s = prm->s, L = prm->levels;
    if (N < 2 || s < 1 || s > 8 || N % (2 * s) != 0 ||
        (prm->prec != DD_PREC_F32 && prm->prec != DD_PREC_F64) || !(prm->trunc >= 0.0))
        return fail(nullptr, DD_EINVAL,
                    "domdec_init: need N % (2s) == 0, 1 <= s <= 8, prec F32|F64, trunc >= 0");
    if (L < 0 || L > 12 || N % (1 << L) != 0 || (N >> L) % (2 * s) != 0)
        return fail(nullptr, DD_EINVAL,
                    "domdec_init: levels must be >= 0 with N / 2^levels a multiple of 2s");
    if (n_init < 0 || (n_init > 0 && (!init_x || !init_y || !init_m)))
        return fail(nullptr, DD_EINVAL, "domdec_init: bad initial coupling arrays");
    const int64_t NN = (int64_t)N * N;
    double smu = 0, snu = 0;
    for (int64_t k = 0; k < NN; ++k) {
        if (!(mu[k] >= 0.0) || !(nu[k] >= 0.0) || !std::isfinite(mu[k]) || !std::isfinite(nu[k]))
            return fail(nullptr, DD_EINVAL, "domdec_init: masses must be finite and >= 0");
        smu += mu[k];
        snu += nu[k];
    }
    if (std::fabs(smu - 1.0) > 1e-12 || std::fabs(snu - 1.0) > 1e-12)
        return fail(nullptr, DD_EINVAL, "domdec_init: mu and nu must each sum to 1 (within 1e-12)");

    if ((prm->dev_alloc == nullptr) != (prm->dev_free == nullptr))
        return fail(nullptr, DD_EINVAL, "domdec_init: dev_alloc and dev_free must both be set or "
                                        "both be NULL");
    dd_ctx* c = new dd_ctx();
    use_mem(c, Mem{prm->dev_alloc, prm->dev_free, prm->alloc_ud});
    c->s = s;
    c->trunc = prm->trunc;
    c->prec = prm->prec;
    c->st = reinterpret_cast<hipStream_t>(stream);
    c->levels = L;
    c->layer = 0;
    // the layers: 2 x 2 block sums, coarsest first
    c->pyr_mu.assign(L + 1, {});
    c->pyr_nu.assign(L + 1, {});
    c->pyr_mu[L].assign(mu, mu + NN);
    c->pyr_nu[L].assign(nu, nu + NN);
    for (int l = L; l > 0; --l) {
        c->pyr_mu[l - 1] = coarsen(c->pyr_mu[l], N >> (L - l));
        c->pyr_nu[l - 1] = coarsen(c->pyr_nu[l], N >> (L - l));
    }
    const int Nc = N >> L;
    const double* cmu = c->pyr_mu[0].data();
    const double* cnu = c->pyr_nu[0].data();
    Status st = setup_layer(c, Nc, cmu, cnu);
    if (!st.code) {
        if (L == 0 || n_init == 0) {
            st = boxes_from_host(c, cmu, cnu, n_init, init_x, init_y, init_m);
        } else {
            // the coupling on the finest grid, summed over the blocks of the coarsest layer
            std::vector<double> px(NN, 0.0), py(NN, 0.0);
            std::vector<int64_t> cx(n_init), cy(n_init);
            bool ok = true;
            for (int64_t e = 0; e < n_init && ok; ++e) {
                const int64_t x = init_x[e], y = init_y[e];
                if (x < 0 || x >= NN || y < 0 || y >= NN || !(init_m[e] >= 0.0)) {
                    ok = false;
                    break;
                }
                px[x] += init_m[e];
                py[y] += init_m[e];
                cx[e] = ((x / N) >> L) * Nc + ((x % N) >> L);
                cy[e] = ((y / N) >> L) * Nc + ((y % N) >> L);
            }
            for (int64_t k = 0; k < NN && ok; ++k)
                ok = std::fabs(px[k] - mu[k]) <= 1e-12 && std::fabs(py[k] - nu[k]) <= 1e-12;
            if (!ok) {
                st.code = DD_EINVAL;
                st.msg = "domdec_init: initial coupling out of range, negative, or with marginals "
                         "other than mu, nu";
            } else {
                st = boxes_from_host(c, cmu, cnu, n_init, cx.data(), cy.data(), init_m);
            }
        }
    }
    if (!st.code && hipStreamSynchronize(c->st) != hipSuccess) {
        st.code = DD_EDEVICE;
        st.msg = "domdec_init: stream synchronisation failed";
    }
    if (st.code) {
        dd_ctx_release(c);
        delete c;
        return fail(nullptr, st);
    }
    *out = c;
    return DD_OK;
}

extern "C" dd_status domdec_refine(dd_ctx* c) {
    if (!c) return fail(c, DD_EINVAL, "domdec_refine: null context");
    dd_forget_pred(c);
    if (c->layer >= c->levels)
        return fail(c, DD_ESTATE, "domdec_refine: already on the finest layer");
    if (!c->visited[0] || !c->visited[1])
        return fail(c, DD_ESTATE, "domdec_refine: both partitions must be iterated on this layer");
    const hipStream_t hs = c->st;
    // the stitched potential of this layer, in units of eps of the A partition's last solve
    DualArgs a;
    a.N = c->N;
    a.s = c->s;
    a.xside = c->AS;
    for (int q = 0; q < 2; ++q) {
        a.ncell[q] = c->part[q].ncell;
        a.members[q] = c->pmembers[q].data();
        a.xorig[q] = c->part[q].xorig;
        a.a[q] = c->d_a[q];
        a.gst[q] = c->d_gst[q];
        a.kappa[q] = c->kappa_a[q];
    }
    a.kappa_eval = c->kappa_a[0];
    a.eps = a.kappa_eval * c->h * c->h;
    a.mu = c->d_mu;
    a.nu = c->d_nu;
    const double* fdag = nullptr;
    Status st = stitched_alpha(a, c->dual, hs, &fdag);
    if (st.code) return fail(c, st);
    // the finer layer, its coupling and its potentials
    dd_ctx* f = new dd_ctx();
    use_mem(f, c->mem);
    f->clusters = c->clusters;
    f->s = c->s;
    f->trunc = c->trunc;
    f->prec = c->prec;
    f->st = hs;
    f->levels = c->levels;
    f->layer = c->layer + 1;
    const int Nc = c->N, Nf = 2 * Nc;
    st = setup_layer(f, Nf, c->pyr_mu[f->layer].data(), c->pyr_nu[f->layer].data());
    int64_t total = 0;
    if (!st.code) {
        launch_refine_boxes(f->n, c->n, c->S.box, f->S.box, f->d_nsize, hs);
        launch_scan(f->d_nsize, f->S.base, f->nI, hs);
        if (hipMemcpyAsync(&total, f->S.base + f->nI, sizeof total, hipMemcpyDeviceToHost, hs) !=
                hipSuccess ||
            hipStreamSynchronize(hs) != hipSuccess) {
            st.code = DD_EDEVICE;
            st.msg = "domdec_refine: reading the refined sizes failed";
        }
    }
    if (!st.code && !grow(c->mem, f->S.data, f->S.cap, (size_t)std::max<int64_t>(total, 1), st).code) {
        launch_refine_values(f->n, c->n, Nc, c->S, c->d_m, c->d_nu, f->S.base, f->d_m, f->d_nu,
                             f->S.data, hs);
        const double kappa_f = a.kappa_eval * 4.0;  // the same eps in units of the finer h^2
        for (int q = 0; q < 2; ++q) {
            launch_refine_alpha(f->part[q], f->AS, Nc, fdag, f->d_a[q], hs);
            f->visited[q] = true;
            f->kappa_a[q] = kappa_f;
        }
        if (hipStreamSynchronize(hs) != hipSuccess || hipGetLastError() != hipSuccess) {
            st.code = DD_EDEVICE;
            st.msg = "domdec_refine: a kernel failed";
        }
    }
    if (st.code) {
        dd_ctx_release(f);
        delete f;
        return fail(c, st);
    }
    f->pyr_mu = std::move(c->pyr_mu);
    f->pyr_nu = std::move(c->pyr_nu);
    f->net = c->net;
    std::swap(*c, *f);
    dd_ctx_release(f);  // the coarse layer
    delete f;
    return DD_OK;
}

static dd_status iterate_impl(dd_ctx* c, int p, double eps, const dd_sinkhorn_opts& o,
                              dd_iter_stats* out) {
    Status st;
    const hipStream_t hs = c->st;
    PartDev& P = c->part[p];
    const int nc = P.ncell;
    const double kappa = eps / (c->h * c->h);
    // the composite dims predicted by the last iteration (consumed here; the end of this one
    // predicts them again)
    const bool use_pred = c->pred_ok[p] && c->h_pred[p] && c->d_pred[p];
    dd_forget_pred(c);
    const int64_t waits0 = c->skw.waits;
    int waits = 0;  // the waits here (the solver counts its own)
    bool resumed = false;
    if (!c->h_small && hipHostMalloc((void**)&c->h_small, 8 * sizeof(int64_t)) != hipSuccess)
        return fail(c, DD_ENOMEM, "domdec_iterate: pinned host buffer");
    for (int q = 0; q < 2; ++q) {
        const size_t n2 = 2 * (size_t)std::max(c->part[q].ncell, 1);
        if (!c->d_pred[q] && alloc(c->mem, c->d_pred[q], n2, st).code) return fail(c, st);
        if (!c->h_pred[q] && hipHostMalloc((void**)&c->h_pred[q], n2 * sizeof(int32_t)) != hipSuccess)
            return fail(c, DD_ENOMEM, "domdec_iterate: pinned host buffer");
    }
    if (!c->d_pcheck && alloc(c->mem, c->d_pcheck, 1, st).code) return fail(c, st);
    (void)hipEventRecord(c->ev[0], hs);
    launch_comp_boxes(P, c->S, c->AS, c->C, hs);
    launch_scan(c->C.size, c->C.base, nc, hs);
    launch_comp_max(c->C, nc, hs);
    launch_fill_i32(c->d_pcheck, 1, 0, hs);
    int mw1 = 1, mw2 = 1;
    int64_t total = 0;
    c->h_dims.resize(2 * (size_t)nc);
    if (use_pred) {
        // no wait: the dims come from the prediction, which the device checks against the
        // boxes it has just computed
        std::copy(c->h_pred[p], c->h_pred[p] + 2 * (size_t)nc, c->h_dims.begin());
        for (int J = 0; J < nc; ++J) {
            mw1 = std::max(mw1, c->h_dims[2 * J]);
            mw2 = std::max(mw2, c->h_dims[2 * J + 1]);
            total += (int64_t)c->h_dims[2 * J] * c->h_dims[2 * J + 1];
        }
        launch_dims_check(2 * nc, c->C.dims, c->d_pred[p], c->d_pcheck, hs);
    } else {
        // the composite sizes and box dims (which the solver plans its launches from)
        int32_t info[2];
        if (hipMemcpyAsync(info, c->C.info, sizeof info, hipMemcpyDeviceToHost, hs) != hipSuccess ||
            hipMemcpyAsync(&total, c->C.base + nc, sizeof total, hipMemcpyDeviceToHost, hs) !=
                hipSuccess ||
            hipMemcpyAsync(c->h_dims.data(), c->C.dims, c->h_dims.size() * 4,
                           hipMemcpyDeviceToHost, hs) != hipSuccess ||
            hipStreamSynchronize(hs) != hipSuccess)
            return fail(c, DD_EDEVICE, "domdec_iterate: reading composite sizes failed");
        ++waits;
        mw1 = info[0];
        mw2 = info[1];
    }
    // the new state's entries are at most four times the composite entries (each basic cell's
    // truncated box lies in its composite cell's box), so its buffer is sized here and the
    // truncated sizes are read only at the end
    if (grow(c->mem, c->d_nuJ, c->nuJ_cap, (size_t)total, st).code ||
        grow(c->mem, c->d_lognu, c->lognu_cap, (size_t)total, st).code ||
        grow(c->mem, c->d_b, c->b_cap, (size_t)total, st).code ||
        grow(c->mem, c->d_tmp, c->tmp_cap, 4 * (size_t)total, st).code ||
        grow(c->mem, c->S2.data, c->S2.cap, std::max<size_t>(4 * (size_t)total, 1), st).code)
        return fail(c, st);
    double* lognu = c->d_lognu;
    double* bpot = c->d_b;
    double* apot = c->d_a[p];
    const double* logmu = c->d_logmu[p];
    launch_b2c(P, c->S, c->C, c->d_nuJ, lognu, hs);
    (void)hipEventRecord(c->ev[1], hs);
    // the zero or previous-iterate start; a copy is kept as the base of the learned start's
    // training samples (domdec_net_samples)
    const size_t na = (size_t)nc * c->AS * c->AS;
    if (grow(c->mem, c->d_a0, c->a0_cap, na, st).code) return fail(c, st);
    const int use_prev = (o.init != DD_INIT_ZERO && c->visited[p]) ? 1 : 0;
    launch_warm_start(P, c->C, c->AS, apot, c->d_gst[p], c->kappa_a[p], kappa, use_prev, hs);
    if (hipMemcpyAsync(c->d_a0, apot, na * sizeof(double), hipMemcpyDeviceToDevice, hs) !=
        hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_iterate: copying the start failed");
    if (o.init == DD_INIT_NET) {
        // learned start: features of the previous-iterate start -> net -> one X-update, over
        // the whole box, of the corrected Y potential
        if (grow(c->mem, c->d_nx, c->nx_cap, (size_t)nc * kNetCin * kNetWin * kNetWin, st).code ||
            grow(c->mem, c->d_ng, c->ng_cap, (size_t)nc * kNetWin * kNetWin, st).code)
            return fail(c, st);
        launch_net_features(nc, c->AS, c->C.dims, c->C.shift, c->C.base, logmu, lognu, apot,
                            kappa, nullptr, c->d_nx, nullptr, nullptr, hs);
        const Status ns = net_infer(c->net, nc, c->d_nx, c->d_ng, hs);
        if (ns.code) return fail(c, ns);
        // (the c2b scratch, 4 doubles per box entry, is free until the solve has finished)
        launch_net_start(nc, c->AS, c->C.dims, c->C.shift, c->C.base, logmu, lognu, c->C.gofs,
                         c->d_ng, kappa, reinterpret_cast<float*>(c->d_tmp), apot, c->d_gst[p],
                         hs);
    }
    (void)hipEventRecord(c->ev[4], hs);
    SkBatch B;
    B.ncells = nc;
    B.xside = c->AS;
    B.dims = c->C.dims;
    B.base = c->C.base;
    B.shift = c->C.shift;
    B.logmu = logmu;
    B.lognu = lognu;
    B.a = apot;
    B.b = bpot;
    B.kappa = kappa;
    B.max_w1 = mw1;
    B.max_w2 = mw2;
    B.prec = c->prec;
    dd_batch_stats bs{};
    // the solve is enqueued whole where it can be (speculative rounds, sk_solve), so that the
    // one wait of the iteration is the one at its end
    const Status ss = sk_solve(B, o, hs, c->skw, &bs, c->d_iters, c->d_cerr, c->h_dims.data(),
                               /*defer=*/true, /*spec=*/true);
    if (ss.code) return fail(c, ss);
    // CompositeToBasic, balance, truncate and compact into S2; then the next iteration's
    // composite dims of both partitions from S2; then the one wait: the new state's size, the
    // untruncated cells, the prediction check, the solve's statistics
    auto tail = [&]() -> bool {
        ++waits;
        (void)hipEventRecord(c->ev[2], hs);
        launch_c2b(P, c->C, c->AS, c->s, mw2, apot, logmu, c->d_nuJ, kappa, c->h, c->d_tmp,
                   c->d_py2, hs);
        launch_balance(P, c->C, c->d_m, c->d_tmp, hs);
        launch_fill_i32(c->d_flags, c->nI + 1, 0, hs);
        launch_trunc_boxes(P, c->C, c->d_tmp, c->trunc, c->nI, c->S2.box, c->d_nsize, c->d_flags,
                           hs);
        launch_scan(c->d_nsize, c->S2.base, c->nI, hs);
        launch_compact(P, c->C, c->d_tmp, c->trunc, c->S2.box, c->S2.base, c->d_flags,
                       c->S2.data, hs);
        (void)hipEventRecord(c->ev[3], hs);
        for (int q = 0; q < 2; ++q) {
            launch_comp_dims(c->part[q], c->S2.box, c->d_pred[q], hs);
            if (hipMemcpyAsync(c->h_pred[q], c->d_pred[q],
                               2 * (size_t)c->part[q].ncell * sizeof(int32_t),
                               hipMemcpyDeviceToHost, hs) != hipSuccess)
                return false;
        }
        return hipMemcpyAsync(c->h_small, c->S2.base + c->nI, sizeof(int64_t),
                              hipMemcpyDeviceToHost, hs) == hipSuccess &&
               hipMemcpyAsync(c->h_small + 1, c->d_flags + c->nI, sizeof(int32_t),
                              hipMemcpyDeviceToHost, hs) == hipSuccess &&
               hipMemcpyAsync(c->h_small + 2, c->d_pcheck, sizeof(int32_t),
                              hipMemcpyDeviceToHost, hs) == hipSuccess &&
               hipStreamSynchronize(hs) == hipSuccess && hipGetLastError() == hipSuccess;
    };
    if (!tail()) return fail(c, DD_EDEVICE, "domdec_iterate: a kernel failed");
    Status fs = sk_finish(c->skw, &bs);
    if (c->skw.spec.need_resume) {
        // the speculative rounds were not enough: continue the solve where it stands, then
        // redo the steps behind it
        resumed = true;
        const Status rs = sk_resume(c->skw);
        if (rs.code) return fail(c, rs);
        if (!tail()) return fail(c, DD_EDEVICE, "domdec_iterate: a kernel failed");
        fs = sk_finish(c->skw, &bs);
        if (c->skw.spec.need_resume)
            return fail(c, DD_EDEVICE, "domdec_iterate: the resumed solve did not finish");
    }
    if (fs.code != DD_OK && fs.code != DD_NOTCONV) return fail(c, fs);
    if (*reinterpret_cast<const int32_t*>(c->h_small + 2) != 0)
        return fail(c, DD_EDEVICE, "domdec_iterate: predicted composite boxes were stale");
    std::swap(c->S, c->S2);
    c->visited[p] = true;
    c->kappa_a[p] = kappa;
    c->pred_ok[0] = c->pred_ok[1] = true;
    const int64_t ntot = c->h_small[0];
    const int32_t kept = *reinterpret_cast<const int32_t*>(c->h_small + 1);
    c->last_part = p;
    c->last_eps = eps;
    c->last_mw1 = mw1;
    c->last_mw2 = mw2;
    c->untruncated_cells = kept;
    if (out) {
        dd_iter_stats s{};
        s.sk = bs;
        s.partition = p;
        s.max_w1 = mw1;
        s.max_w2 = mw2;
        s.grid_n = c->N;
        s.nu_entries = ntot;
        s.comp_entries = total;
        s.batches = 1;
        s.peak_comp_entries = total;
        s.host_waits = waits + (int32_t)(c->skw.waits - waits0);
        s.spec_resumed = resumed ? 1 : 0;
        float t = 0.f;
        (void)hipEventElapsedTime(&t, c->ev[0], c->ev[1]);
        s.t_b2c_ms = t;
        s.t_sinkhorn_ms = bs.time_ms;
        (void)hipEventElapsedTime(&t, c->ev[2], c->ev[3]);
        s.t_c2b_ms = t;
        (void)hipEventElapsedTime(&t, c->ev[0], c->ev[3]);
        s.t_total_ms = t;
        (void)hipEventElapsedTime(&t, c->ev[1], c->ev[4]);
        s.t_init_ms = t;
        *out = s;
    }
    if (fs.code == DD_NOTCONV) {
        c->err = fs.msg;
        return DD_NOTCONV;
    }
    return DD_OK;
}

namespace {

// K-means on the composite Y-box dimensions (W1, W2) into at most k clusters (Lloyd's
// iteration from the boxes at evenly spaced ranks of the area order); returns the clusters'
// cells, each in ascending order, the clusters by decreasing centre area.  Deterministic.
std::vector<std::vector<int32_t>> kmeans_batches(const std::vector<int32_t>& dims, int k) {
    const int n = (int)(dims.size() / 2);
    k = std::max(1, std::min(k, n));
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto area = [&](int i) { return (int64_t)dims[2 * i] * dims[2 * i + 1]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return area(a) < area(b); });
    std::vector<double> c1(k), c2(k);
    for (int q = 0; q < k; ++q) {
        const int i = order[std::min<size_t>(n - 1, (size_t)(((double)q + 0.5) * n / k))];
        c1[q] = dims[2 * i];
        c2[q] = dims[2 * i + 1];
    }
    std::vector<int> lab(n, -1);
    for (int it = 0; it < 100; ++it) {
        bool changed = false;
        for (int i = 0; i < n; ++i) {
            int best = 0;
            double bd = 1e300;
            for (int q = 0; q < k; ++q) {
                const double d1 = dims[2 * i] - c1[q], d2 = dims[2 * i + 1] - c2[q];
                const double d = d1 * d1 + d2 * d2;
                if (d < bd) {
                    bd = d;
                    best = q;
                }
            }
            changed |= lab[i] != best;
            lab[i] = best;
        }
        if (!changed) break;
        std::vector<double> s1(k, 0.0), s2(k, 0.0);
        std::vector<int> cnt(k, 0);
        for (int i = 0; i < n; ++i) {
            s1[lab[i]] += dims[2 * i];
            s2[lab[i]] += dims[2 * i + 1];
            ++cnt[lab[i]];
        }
        for (int q = 0; q < k; ++q)
            if (cnt[q]) {
                c1[q] = s1[q] / cnt[q];
                c2[q] = s2[q] / cnt[q];
            }
    }
    std::vector<std::vector<int32_t>> groups(k);
    for (int i = 0; i < n; ++i) groups[lab[i]].push_back(i);
    std::vector<int> qs(k);
    std::iota(qs.begin(), qs.end(), 0);
    std::stable_sort(qs.begin(), qs.end(), [&](int a, int b) { return c1[a] * c2[a] > c1[b] * c2[b]; });
    std::vector<std::vector<int32_t>> out;
    for (int q : qs)
        if (!groups[q].empty()) out.push_back(std::move(groups[q]));
    return out;
}

Status reserve_batches(dd_ctx* c, int n) {
    Status st;
    auto& B = c->bt;
    if (!B.stage_base && alloc(c->mem, B.stage_base, (size_t)c->nI, st).code) return st;
    if (n <= B.cap) return st;
    auto F = [c](auto& p) {
        c->mem.put(p);
        p = nullptr;
    };
    for (int32_t** q : {&B.C.dims, &B.C.orig, &B.C.shift, &B.C.gofs, &B.idx, &B.members, &B.xorig,
                        &B.gst, &B.list})
        F(*q);
    F(B.C.size);
    F(B.C.base);
    F(B.a);
    F(B.logmu);
    F(B.lsize);
    B.cap = 0;
    const size_t A2 = (size_t)c->AS * c->AS;
    if (alloc(c->mem, B.C.dims, 2 * (size_t)n, st).code ||
        alloc(c->mem, B.C.orig, 2 * (size_t)n, st).code ||
        alloc(c->mem, B.C.shift, 2 * (size_t)n, st).code ||
        alloc(c->mem, B.C.gofs, 2 * (size_t)n, st).code || alloc(c->mem, B.C.size, n, st).code ||
        alloc(c->mem, B.C.base, (size_t)n + 1, st).code ||
        (!B.C.info && alloc(c->mem, B.C.info, 8, st).code) || alloc(c->mem, B.idx, n, st).code ||
        alloc(c->mem, B.members, 4 * (size_t)n, st).code ||
        alloc(c->mem, B.xorig, 2 * (size_t)n, st).code || alloc(c->mem, B.gst, 2 * (size_t)n, st).code ||
        alloc(c->mem, B.a, A2 * n, st).code || alloc(c->mem, B.logmu, A2 * n, st).code ||
        alloc(c->mem, B.list, 4 * (size_t)n, st).code ||
        alloc(c->mem, B.lsize, 2 * (4 * (size_t)n + 1), st).code)
        return st;
    B.cap = n;
    return st;
}

// staging buffer of at least `need` entries that keeps its first `used` entries
Status grow_staging(dd_ctx* c, size_t need, size_t used) {
    Status st;
    auto& B = c->bt;
    if (need <= B.staging_cap && B.staging) return st;
    const size_t cap = std::max<size_t>((size_t)(need * 1.25) + 64, 1024);
    double* fresh = nullptr;
    if (alloc(c->mem, fresh, cap, st).code) return st;
    if (used > 0)
        DD_HIP(hipMemcpyAsync(fresh, B.staging, used * sizeof(double), hipMemcpyDeviceToDevice,
                              c->st),
               st);
    DD_HIP(hipStreamSynchronize(c->st), st);  // the old buffer is read until here
    c->mem.put(B.staging);
    B.staging = fresh;
    B.staging_cap = cap;
    return st;
}

void add_stats(dd_batch_stats& a, const dd_batch_stats& b, bool first) {
    if (first) {
        a = b;
        return;
    }
    a.ncells += b.ncells;
    a.iters_max = std::max(a.iters_max, b.iters_max);
    a.iters_min = std::min(a.iters_min, b.iters_min);
    a.converged = a.converged && b.converged;
    a.cell_iters += b.cell_iters;
    a.err += b.err;
    a.mass += b.mass;
    a.lse_terms += b.lse_terms;
    a.alg_bytes += b.alg_bytes;
    a.time_ms += b.time_ms;
    a.main_ms += b.main_ms;
    a.finish_iters_max = std::max(a.finish_iters_max, b.finish_iters_max);
    a.n_big += b.n_big;
    a.n_giant += b.n_giant;
    for (int k = 0; k < 3; ++k) {
        a.kernel_launches[k] += b.kernel_launches[k];
        a.kernel_ms[k] += b.kernel_ms[k];
        a.kernel_terms[k] += b.kernel_terms[k];
    }
}

}  // namespace

// One DD half-iteration with the partition's composite cells split into bounding-box clusters
// solved one after another (App. A.1 "Batching and clustering": CreateBatches /
// CombineBatches): the composite work arrays hold one batch at a time.  Each batch runs
// BasicToComposite, the start, the cell solve (its own stopping rule), CompositeToBasic,
// balancing and truncation; its truncated basic-cell boxes are staged, and the new state is
// assembled from the staging once every batch is done.
static dd_status iterate_batched(dd_ctx* c, int p, double eps, const dd_sinkhorn_opts& o,
                                 dd_iter_stats* out) {
    Status st;
    const hipStream_t hs = c->st;
    dd_forget_pred(c);
    PartDev& P = c->part[p];
    const int nc = P.ncell, AS = c->AS, A2 = AS * AS;
    const double kappa = eps / (c->h * c->h);
    auto& B = c->bt;
    (void)hipEventRecord(c->ev[0], hs);
    // every composite cell's box: the clustering's input
    launch_comp_boxes(P, c->S, AS, c->C, hs);
    std::vector<int32_t> dims(2 * (size_t)nc);
    if (hipMemcpyAsync(dims.data(), c->C.dims, dims.size() * 4, hipMemcpyDeviceToHost, hs) !=
            hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_iterate: reading composite boxes failed");
    const std::vector<std::vector<int32_t>> groups = kmeans_batches(dims, c->clusters);
    size_t most = 0;
    for (const auto& g : groups) most = std::max(most, g.size());
    {
        const Status rs = reserve_batches(c, (int)most);
        if (rs.code) return fail(c, rs);
    }
    launch_fill_i32(c->d_flags, c->nI + 1, 0, hs);
    const int use_prev = (o.init != DD_INIT_ZERO && c->visited[p]) ? 1 : 0;
    const double kappa_old = c->kappa_a[p];
    dd_batch_stats agg{};
    int64_t staged = 0, comp_total = 0, peak = 0;
    int mw1_all = 0, mw2_all = 0;
    bool notconv = false;
    std::string notconv_msg;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const std::vector<int32_t>& g = groups[gi];
        const int nb = (int)g.size();
        std::vector<int32_t> mem(4 * (size_t)nb), xo(2 * (size_t)nb), list;
        for (int j = 0; j < nb; ++j) {
            for (int k = 0; k < 4; ++k) {
                mem[4 * j + k] = c->pmembers[p][4 * (size_t)g[j] + k];
                if (mem[4 * j + k] >= 0) list.push_back(mem[4 * j + k]);
            }
            xo[2 * j] = c->pxorig[p][2 * (size_t)g[j]];
            xo[2 * j + 1] = c->pxorig[p][2 * (size_t)g[j] + 1];
        }
        const int nl = (int)list.size();
        PartDev Pb;
        Pb.ncell = nb;
        Pb.members = B.members;
        Pb.xorig = B.xorig;
        // (the host vectors stay alive until the synchronisation below)
        if (hipMemcpyAsync(B.idx, g.data(), (size_t)nb * 4, hipMemcpyHostToDevice, hs) != hipSuccess ||
            hipMemcpyAsync(B.members, mem.data(), mem.size() * 4, hipMemcpyHostToDevice, hs) !=
                hipSuccess ||
            hipMemcpyAsync(B.xorig, xo.data(), xo.size() * 4, hipMemcpyHostToDevice, hs) !=
                hipSuccess ||
            hipMemcpyAsync(B.list, list.data(), (size_t)nl * 4, hipMemcpyHostToDevice, hs) !=
                hipSuccess)
            return fail(c, DD_EDEVICE, "domdec_iterate: uploading a batch failed");
        launch_gather_rows(nb, B.idx, A2, c->d_logmu[p], B.logmu, hs);
        launch_gather_rows(nb, B.idx, A2, c->d_a[p], B.a, hs);
        launch_gather_rows_i32(nb, B.idx, 2, c->d_gst[p], B.gst, 0, hs);
        launch_comp_boxes(Pb, c->S, AS, B.C, hs);
        launch_scan(B.C.size, B.C.base, nb, hs);
        launch_comp_max(B.C, nb, hs);
        int32_t info[2];
        int64_t total = 0;
        if (hipMemcpyAsync(info, B.C.info, sizeof info, hipMemcpyDeviceToHost, hs) != hipSuccess ||
            hipMemcpyAsync(&total, B.C.base + nb, sizeof total, hipMemcpyDeviceToHost, hs) !=
                hipSuccess ||
            hipStreamSynchronize(hs) != hipSuccess)
            return fail(c, DD_EDEVICE, "domdec_iterate: reading a batch's sizes failed");
        const int mw1 = info[0], mw2 = info[1];
        mw1_all = std::max(mw1_all, mw1);
        mw2_all = std::max(mw2_all, mw2);
        comp_total += total;
        peak = std::max(peak, total);
        if (grow(c->mem, c->d_nuJ, c->nuJ_cap, (size_t)total, st).code ||
            grow(c->mem, c->d_lognu, c->lognu_cap, (size_t)total, st).code ||
            grow(c->mem, c->d_b, c->b_cap, (size_t)total, st).code ||
            grow(c->mem, c->d_tmp, c->tmp_cap, 4 * (size_t)total, st).code)
            return fail(c, st);
        launch_b2c(Pb, c->S, B.C, c->d_nuJ, c->d_lognu, hs);
        launch_warm_start(Pb, B.C, AS, B.a, B.gst, kappa_old, kappa, use_prev, hs);
        SkBatch sb;
        sb.ncells = nb;
        sb.xside = AS;
        sb.dims = B.C.dims;
        sb.base = B.C.base;
        sb.shift = B.C.shift;
        sb.logmu = B.logmu;
        sb.lognu = c->d_lognu;
        sb.a = B.a;
        sb.b = c->d_b;
        sb.kappa = kappa;
        sb.max_w1 = mw1;
        sb.max_w2 = mw2;
        sb.prec = c->prec;
        dd_batch_stats bs{};
        const Status ss = sk_solve(sb, o, hs, c->skw, &bs, c->d_iters, c->d_cerr);
        if (ss.code != DD_OK && ss.code != DD_NOTCONV) return fail(c, ss);
        if (ss.code == DD_NOTCONV) {
            notconv = true;
            notconv_msg = ss.msg;
        }
        add_stats(agg, bs, gi == 0);
        launch_c2b(Pb, B.C, AS, c->s, mw2, B.a, B.logmu, c->d_nuJ, kappa, c->h, c->d_tmp,
                   c->d_py2, hs);
        launch_balance(Pb, B.C, c->d_m, c->d_tmp, hs);
        launch_trunc_boxes(Pb, B.C, c->d_tmp, c->trunc, c->nI, c->S2.box, c->d_nsize, c->d_flags,
                           hs);
        // the batch's truncated boxes go to the staging, after the earlier batches'
        int64_t* lpre = B.lsize + 4 * (size_t)B.cap + 1;
        launch_list_sizes(nl, B.list, c->d_nsize, B.lsize, hs);
        launch_scan(B.lsize, lpre, nl, hs);
        int64_t add = 0;
        if (hipMemcpyAsync(&add, lpre + nl, sizeof add, hipMemcpyDeviceToHost, hs) != hipSuccess ||
            hipStreamSynchronize(hs) != hipSuccess)
            return fail(c, DD_EDEVICE, "domdec_iterate: reading a batch's truncated sizes failed");
        {
            const Status gs = grow_staging(c, (size_t)(staged + add), (size_t)staged);
            if (gs.code) return fail(c, gs);
        }
        launch_stage_base(nl, B.list, lpre, staged, B.stage_base, hs);
        launch_compact(Pb, B.C, c->d_tmp, c->trunc, c->S2.box, B.stage_base, c->d_flags, B.staging,
                       hs);
        staged += add;
        launch_scatter_rows(nb, B.idx, A2, B.a, c->d_a[p], hs);
        launch_gather_rows_i32(nb, B.idx, 2, B.gst, c->d_gst[p], 1, hs);
    }
    // CombineBatches: the new state in basic-cell order
    launch_scan(c->d_nsize, c->S2.base, c->nI, hs);
    int64_t ntot = 0;
    int32_t kept = 0;
    if (hipMemcpyAsync(&ntot, c->S2.base + c->nI, sizeof ntot, hipMemcpyDeviceToHost, hs) !=
            hipSuccess ||
        hipMemcpyAsync(&kept, c->d_flags + c->nI, sizeof kept, hipMemcpyDeviceToHost, hs) !=
            hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_iterate: reading truncated sizes failed");
    if (grow(c->mem, c->S2.data, c->S2.cap, (size_t)std::max<int64_t>(ntot, 1), st).code)
        return fail(c, st);
    launch_unstage(c->nI, c->d_nsize, B.stage_base, B.staging, c->S2.base, c->S2.data, hs);
    std::swap(c->S, c->S2);
    (void)hipEventRecord(c->ev[3], hs);
    if (hipStreamSynchronize(hs) != hipSuccess || hipGetLastError() != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_iterate: a kernel failed");
    c->visited[p] = true;
    c->kappa_a[p] = kappa;
    // the composite plans of this iteration were spread over the batches: the evaluation of
    // composite quantities, beta and the flow update need an unbatched iteration
    c->last_part = -1;
    c->last_eps = eps;
    c->untruncated_cells = kept;
    B.peak_entries = peak;
    B.count = (int)groups.size();
    if (out) {
        dd_iter_stats s{};
        s.sk = agg;
        s.partition = p;
        s.max_w1 = mw1_all;
        s.max_w2 = mw2_all;
        s.grid_n = c->N;
        s.nu_entries = ntot;
        s.comp_entries = comp_total;
        s.batches = (int32_t)groups.size();
        s.peak_comp_entries = peak;
        s.t_sinkhorn_ms = agg.time_ms;
        float t = 0.f;
        (void)hipEventElapsedTime(&t, c->ev[0], c->ev[3]);
        s.t_total_ms = t;
        *out = s;
    }
    if (notconv) {
        c->err = notconv_msg;
        return DD_NOTCONV;
    }
    return DD_OK;
}

extern "C" dd_status domdec_set_clusters(dd_ctx* c, int32_t clusters) {
    if (!c) return fail(c, DD_EINVAL, "domdec_set_clusters: null context");
    if (clusters < 1) return fail(c, DD_EINVAL, "domdec_set_clusters: clusters must be >= 1");
    dd_forget_pred(c);
    c->clusters = clusters;
    return DD_OK;
}

extern "C" dd_status domdec_iterate(dd_ctx* c, int32_t partition, double eps,
                                    const dd_sinkhorn_opts* o, dd_iter_stats* out) {
    if (!c || !o) return fail(c, DD_EINVAL, "domdec_iterate: null argument");
    if (partition != DD_PART_A && partition != DD_PART_B)
        return fail(c, DD_EINVAL, "domdec_iterate: partition must be DD_PART_A or DD_PART_B");
    if (!(eps > 0.0) || !std::isfinite(eps))
        return fail(c, DD_EINVAL, "domdec_iterate: eps must be positive and finite");
    if (o->init != DD_INIT_ZERO && o->init != DD_INIT_PREV && o->init != DD_INIT_NET)
        return fail(c, DD_EINVAL,
                    "domdec_iterate: init must be DD_INIT_ZERO, DD_INIT_PREV or DD_INIT_NET");
    if (o->init == DD_INIT_NET && !c->net)
        return fail(c, DD_ESTATE, "domdec_iterate: DD_INIT_NET needs a net (domdec_set_net)");
    if (o->init == DD_INIT_NET && c->AS > 8)
        return fail(c, DD_EINVAL, "domdec_iterate: DD_INIT_NET needs X blocks of side <= 8");
    if (c->clusters > 1) {
        if (o->init == DD_INIT_NET)
            return fail(c, DD_EINVAL, "domdec_iterate: DD_INIT_NET runs unbatched (clusters 1)");
        return iterate_batched(c, partition, eps, *o, out);
    }
    return iterate_impl(c, partition, eps, *o, out);
}

extern "C" dd_status extract_plan(dd_ctx* c, dd_plan_view* v) {
    if (!c || !v) return fail(c, DD_EINVAL, "extract_plan: null argument");
    int64_t total = 0;
    if (hipMemcpyAsync(&total, c->S.base + c->nI, sizeof total, hipMemcpyDeviceToHost, c->st) !=
            hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return fail(c, DD_EDEVICE, "extract_plan: copy failed");
    v->n_cells = c->nI;
    v->n_entries = total;
    if (!v->offsets && !v->dims && !v->base && !v->data) return DD_OK;
    std::vector<int32_t> box(4 * (size_t)c->nI);
    if (hipMemcpyAsync(box.data(), c->S.box, box.size() * 4, hipMemcpyDeviceToHost, c->st) !=
            hipSuccess ||
        (v->base && hipMemcpyAsync(v->base, c->S.base, (c->nI + 1) * sizeof(int64_t),
                                   hipMemcpyDeviceToHost, c->st) != hipSuccess) ||
        (v->data && total > 0 &&
         hipMemcpyAsync(v->data, c->S.data, total * sizeof(double), hipMemcpyDeviceToHost, c->st) !=
             hipSuccess) ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return fail(c, DD_EDEVICE, "extract_plan: copy failed");
    for (int i = 0; i < c->nI; ++i) {
        if (v->offsets) {
            v->offsets[2 * i] = box[4 * i];
            v->offsets[2 * i + 1] = box[4 * i + 1];
        }
        if (v->dims) {
            v->dims[2 * i] = box[4 * i + 2];
            v->dims[2 * i + 1] = box[4 * i + 3];
        }
    }
    return DD_OK;
}

// Potentials in energy units with the paper's reference measure mu_J (x) nu (Sec. 2.3).  The
// solver's f, g use reference mu_J (x) nu_J and the local cost C = |i - j + E|^2 / kappa of a
// box at pixel origin pY, with G = pX - pY - E; the true cost over eps is
// C + 2<G, i>/kappa - 2<G, j - E>/kappa + |G|^2/kappa, hence
//   alpha(i) = eps (f(i) + 2<G, i>/kappa),
//   beta(j)  = eps (g(j) - 2<G, j - E>/kappa + |G|^2/kappa + log nu_J(j) - log nu(j)).
extern "C" dd_status extract_potentials(dd_ctx* c, dd_potentials_view* v) {
    if (!c || !v) return fail(c, DD_EINVAL, "extract_potentials: null argument");
    const int p = v->partition;
    if (p != DD_PART_A && p != DD_PART_B)
        return fail(c, DD_EINVAL, "extract_potentials: partition must be DD_PART_A or DD_PART_B");
    if (!c->visited[p])
        return fail(c, DD_ESTATE, "extract_potentials: the partition has not been iterated");
    const hipStream_t hs = c->st;
    const int nc = c->part[p].ncell, AS = c->AS, A2 = AS * AS;
    const double kappa = c->kappa_a[p];
    const double eps = kappa * c->h * c->h;
    const bool has_beta = c->last_part == p;
    int64_t ny = 0;
    if (has_beta && (hipMemcpyAsync(&ny, c->C.base + nc, sizeof ny, hipMemcpyDeviceToHost, hs) !=
                         hipSuccess ||
                     hipStreamSynchronize(hs) != hipSuccess))
        return fail(c, DD_EDEVICE, "extract_potentials: copy failed");
    v->n_cells = nc;
    v->xside = AS;
    v->has_beta = has_beta ? 1 : 0;
    v->eps = eps;
    v->n_y = ny;
    if (!v->xorig && !v->alpha && !v->yorig && !v->ydims && !v->ybase && !v->beta) return DD_OK;
    std::vector<double> f((size_t)nc * A2);
    std::vector<int32_t> gst(2 * (size_t)nc);
    if (hipMemcpyAsync(f.data(), c->d_a[p], f.size() * sizeof(double), hipMemcpyDeviceToHost, hs) !=
            hipSuccess ||
        hipMemcpyAsync(gst.data(), c->d_gst[p], gst.size() * 4, hipMemcpyDeviceToHost, hs) !=
            hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "extract_potentials: copy failed");
    if (v->xorig) std::copy(c->pxorig[p].begin(), c->pxorig[p].end(), v->xorig);
    if (v->alpha)
        for (int J = 0; J < nc; ++J)
            for (int il = 0; il < A2; ++il) {
                const int i1 = il / AS, i2 = il % AS;
                const double lin = 2.0 * ((double)gst[2 * J] * i1 + (double)gst[2 * J + 1] * i2);
                v->alpha[(size_t)J * A2 + il] = eps * (f[(size_t)J * A2 + il] + lin / kappa);
            }
    const bool want_y = v->yorig || v->ydims || v->ybase || v->beta;
    if (!want_y) return DD_OK;
    if (!has_beta)
        return fail(c, DD_ESTATE,
                    "extract_potentials: beta needs the partition's iteration to be the last one");
    std::vector<int32_t> dims(2 * (size_t)nc), orig(2 * (size_t)nc), shift(2 * (size_t)nc),
        gofs(2 * (size_t)nc);
    std::vector<int64_t> base((size_t)nc + 1);
    bool ok = hipMemcpyAsync(dims.data(), c->C.dims, dims.size() * 4, hipMemcpyDeviceToHost, hs) ==
                  hipSuccess &&
              hipMemcpyAsync(orig.data(), c->C.orig, orig.size() * 4, hipMemcpyDeviceToHost, hs) ==
                  hipSuccess &&
              hipMemcpyAsync(shift.data(), c->C.shift, shift.size() * 4, hipMemcpyDeviceToHost,
                             hs) == hipSuccess &&
              hipMemcpyAsync(gofs.data(), c->C.gofs, gofs.size() * 4, hipMemcpyDeviceToHost, hs) ==
                  hipSuccess &&
              hipMemcpyAsync(base.data(), c->C.base, base.size() * 8, hipMemcpyDeviceToHost, hs) ==
                  hipSuccess;
    std::vector<double> g, lnuJ, lnu;
    if (ok && v->beta) {
        g.resize((size_t)ny);
        lnuJ.resize((size_t)ny);
        lnu.resize((size_t)c->N * c->N);
        ok = (ny == 0 || (hipMemcpyAsync(g.data(), c->d_b, ny * sizeof(double),
                                         hipMemcpyDeviceToHost, hs) == hipSuccess &&
                          hipMemcpyAsync(lnuJ.data(), c->d_lognu, ny * sizeof(double),
                                         hipMemcpyDeviceToHost, hs) == hipSuccess)) &&
             hipMemcpyAsync(lnu.data(), c->d_lognu_glob, lnu.size() * sizeof(double),
                            hipMemcpyDeviceToHost, hs) == hipSuccess;
    }
    if (!ok || hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "extract_potentials: copy failed");
    if (v->yorig) std::copy(orig.begin(), orig.end(), v->yorig);
    if (v->ydims) std::copy(dims.begin(), dims.end(), v->ydims);
    if (v->ybase) std::copy(base.begin(), base.end(), v->ybase);
    if (v->beta) {
        const double nan = std::nan("");
        for (int J = 0; J < nc; ++J) {
            const int W1 = dims[2 * J], W2 = dims[2 * J + 1];
            const double G1 = gofs[2 * J], G2 = gofs[2 * J + 1];
            const int E1 = shift[2 * J], E2 = shift[2 * J + 1];
            const double cst = (G1 * G1 + G2 * G2) / kappa;
            for (int j1 = 0; j1 < W1; ++j1)
                for (int j2 = 0; j2 < W2; ++j2) {
                    const int64_t k = base[J] + (int64_t)j1 * W2 + j2;
                    const int y1 = orig[2 * J] + j1, y2 = orig[2 * J + 1] + j2;
                    const double ln = lnu[(size_t)y1 * c->N + y2];
                    if (!(lnuJ[k] > -1e29) || !(ln > -1e29)) {
                        v->beta[k] = nan;
                        continue;
                    }
                    const double lin = 2.0 * (G1 * (j1 - E1) + G2 * (j2 - E2)) / kappa;
                    v->beta[k] = eps * (g[k] - lin + cst + lnuJ[k] - ln);
                }
        }
    }
    return DD_OK;
}

void dd_eval_cells(dd_ctx* c, double* pix_out) {
    const int p = c->last_part;
    EvalArgs e;
    e.ncell = c->part[p].ncell;
    e.xside = c->AS;
    e.s = c->s;
    e.maxw1 = c->last_mw1;
    e.maxw2 = c->last_mw2;
    e.N = c->N;
    e.members = c->part[p].members;
    e.xorig = c->part[p].xorig;
    e.cdims = c->C.dims;
    e.corig = c->C.orig;
    e.cshift = c->C.shift;
    e.gofs = c->C.gofs;
    e.cbase = c->C.base;
    e.logmu = c->d_logmu[p];
    e.a = c->d_a[p];
    e.b = c->d_b;
    e.lognuJ = c->d_lognu;
    e.nuJ = c->d_nuJ;
    e.lognu_glob = c->d_lognu_glob;
    e.kappa = c->last_eps / (c->h * c->h);
    e.cell_out = c->d_cell_out;
    e.basic_out = c->d_basic_out;
    e.totals = c->d_eval + 4;
    e.pix_out = pix_out;
    launch_cell_eval(e, c->st);
}

extern "C" dd_status domdec_evaluate(dd_ctx* c, dd_eval* out) {
    if (!c || !out) return fail(c, DD_EINVAL, "domdec_evaluate: null argument");
    dd_eval r{};
    launch_ymarg(c->nI, c->S.box, c->S.base, c->S.data, c->N, c->d_scratch, c->d_nu, c->d_eval,
                 c->st);
    launch_basic_mass(c->nI, c->S.base, c->S.data, c->d_m, c->d_scratch, c->d_eval + 1, c->st);
    if (c->last_part >= 0) dd_eval_cells(c);
    double h[8] = {0};
    if (hipMemcpyAsync(h, c->d_eval, sizeof h, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_evaluate: reduction failed");
    r.y_marginal_l1 = h[0];
    r.total_mass = h[1];
    r.basic_mass_err = h[2];
    r.dual = r.pd_gap = NAN;
    if (c->last_part >= 0) {
        const double eps = c->last_eps;
        r.primal = eps * h[4] + eps * 1.0;  // + eps * (sum mu)(sum nu), the KL reference mass
        r.transport = h[5] * c->h * c->h;
        r.x_marginal_l1 = h[6];
        if (c->visited[0] && c->visited[1]) {
            DualArgs a;
            a.N = c->N;
            a.s = c->s;
            a.xside = c->AS;
            for (int q = 0; q < 2; ++q) {
                a.ncell[q] = c->part[q].ncell;
                a.members[q] = c->pmembers[q].data();
                a.xorig[q] = c->part[q].xorig;
                a.a[q] = c->d_a[q];
                a.gst[q] = c->d_gst[q];
                a.kappa[q] = c->kappa_a[q];
            }
            a.kappa_eval = eps / (c->h * c->h);
            a.eps = eps;
            a.mu = c->d_mu;
            a.nu = c->d_nu;
            double D = NAN;
            const Status ds = stitched_dual(a, c->dual, c->st, &D);
            if (ds.code) return fail(c, ds);
            r.dual = D;
            r.pd_gap = r.primal - D;
        }
    } else {
        r.primal = r.transport = r.x_marginal_l1 = NAN;
    }
    *out = r;
    return DD_OK;
}

extern "C" void domdec_free(dd_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    dd_ctx_release(c);
    delete c;
}

extern "C" const char* domdec_strerror(const dd_ctx* c, dd_status) {
    return c ? c->err.c_str() : global_error();
}

extern "C" dd_status domdec_set_net(dd_ctx* c, dd_net* net) {
    if (!c) return fail(c, DD_EINVAL, "domdec_set_net: null context");
    dd_forget_pred(c);
    c->net = net;
    return DD_OK;
}

extern "C" dd_status domdec_net_samples(dd_ctx* c, float* x, float* target, float* weight,
                                        int32_t cap, int32_t* n) {
    if (!c || !n) return fail(c, DD_EINVAL, "domdec_net_samples: null argument");
    if (c->last_part < 0)
        return fail(c, DD_ESTATE, "domdec_net_samples: needs a preceding domdec_iterate");
    const int p = c->last_part;
    const int nc = c->part[p].ncell;
    *n = nc;
    if (!x && !target && !weight) return DD_OK;
    if (!x || !target || !weight || cap < nc)
        return fail(c, DD_EINVAL, "domdec_net_samples: buffers missing or cap < cells");
    if (c->AS > 8) return fail(c, DD_EINVAL, "domdec_net_samples: needs X blocks of side <= 8");
    launch_net_features(nc, c->AS, c->C.dims, c->C.shift, c->C.base, c->d_logmu[p], c->d_lognu,
                        c->d_a0, c->last_eps / (c->h * c->h), c->d_b, x, target, weight, c->st);
    if (hipStreamSynchronize(c->st) != hipSuccess || hipGetLastError() != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_net_samples: kernel failed");
    return DD_OK;
}

namespace {
hipError_t d2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
}
}  // namespace

extern "C" dd_status domdec_save(dd_ctx* c) {
    if (!c) return fail(c, DD_EINVAL, "domdec_save: null context");
    Status st;
    auto& S = c->snap;
    const hipStream_t hs = c->st;
    int64_t ntot = 0;
    if (hipMemcpyAsync(&ntot, c->S.base + c->nI, sizeof ntot, hipMemcpyDeviceToHost, hs) !=
            hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_save: copy failed");
    if ((!S.box && alloc(c->mem, S.box, 4 * (size_t)c->nI, st).code) ||
        (!S.base && alloc(c->mem, S.base, (size_t)c->nI + 1, st).code) ||
        grow(c->mem, S.data, S.data_cap, (size_t)std::max<int64_t>(ntot, 1), st).code)
        return fail(c, st);
    for (int q = 0; q < 2; ++q) {
        const size_t nc = c->part[q].ncell;
        if ((!S.a[q] && alloc(c->mem, S.a[q], nc * c->AS * c->AS, st).code) ||
            (!S.gst[q] && alloc(c->mem, S.gst[q], 2 * nc, st).code))
            return fail(c, st);
    }
    bool ok = d2d(S.box, c->S.box, 4 * (size_t)c->nI * sizeof(int32_t), hs) == hipSuccess &&
              d2d(S.base, c->S.base, ((size_t)c->nI + 1) * sizeof(int64_t), hs) == hipSuccess &&
              d2d(S.data, c->S.data, (size_t)ntot * sizeof(double), hs) == hipSuccess;
    for (int q = 0; q < 2 && ok; ++q) {
        const size_t nc = c->part[q].ncell;
        ok = d2d(S.a[q], c->d_a[q], nc * c->AS * c->AS * sizeof(double), hs) == hipSuccess &&
             d2d(S.gst[q], c->d_gst[q], 2 * nc * sizeof(int32_t), hs) == hipSuccess;
        S.visited[q] = c->visited[q];
        S.kappa_a[q] = c->kappa_a[q];
    }
    if (!ok || hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_save: copy failed");
    S.ntot = ntot;
    S.valid = true;
    return DD_OK;
}

extern "C" dd_status domdec_restore(dd_ctx* c) {
    if (!c) return fail(c, DD_EINVAL, "domdec_restore: null context");
    dd_forget_pred(c);
    auto& S = c->snap;
    if (!S.valid) return fail(c, DD_ESTATE, "domdec_restore: nothing saved");
    Status st;
    const hipStream_t hs = c->st;
    if (grow(c->mem, c->S.data, c->S.cap, (size_t)std::max<int64_t>(S.ntot, 1), st).code)
        return fail(c, st);
    bool ok = d2d(c->S.box, S.box, 4 * (size_t)c->nI * sizeof(int32_t), hs) == hipSuccess &&
              d2d(c->S.base, S.base, ((size_t)c->nI + 1) * sizeof(int64_t), hs) == hipSuccess &&
              d2d(c->S.data, S.data, (size_t)S.ntot * sizeof(double), hs) == hipSuccess;
    for (int q = 0; q < 2 && ok; ++q) {
        const size_t nc = c->part[q].ncell;
        ok = d2d(c->d_a[q], S.a[q], nc * c->AS * c->AS * sizeof(double), hs) == hipSuccess &&
             d2d(c->d_gst[q], S.gst[q], 2 * nc * sizeof(int32_t), hs) == hipSuccess;
        c->visited[q] = S.visited[q];
        c->kappa_a[q] = S.kappa_a[q];
    }
    if (!ok || hipStreamSynchronize(hs) != hipSuccess)
        return fail(c, DD_EDEVICE, "domdec_restore: copy failed");
    // the last iteration's composite data no longer belongs to the state
    c->last_part = -1;
    return DD_OK;
}
