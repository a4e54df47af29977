/*
 * Oracle for entropic-OT domain decomposition with flow updates -- TEST
 * INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library; the product path never does.
 *
 * Plain, slow, obviously correct float64 C.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Contents
 *   orc_sinkhorn_cells  dense, non-separable log-domain Sinkhorn on a batch of
 *                       cell problems (paper Sec. 2.3 Alg. "DomDecIter", the
 *                       cell problem with reference measure mu_J (x) nu; the
 *                       optimality form of Prop. "Optimal entropic transport
 *                       couplings"; stopping rule of App. A.2.1 "Stopping
 *                       criterion and measure truncation").
 *   orc_cell_plan       instantiate pi_J(x,y) = exp((alpha+beta-c)/eps) mu nu
 *                       densely for one cell.
 *   orc_mcf_ssp         integer min-cost flow on a bipartite transportation
 *                       graph by successive shortest paths (Dijkstra with
 *                       node potentials), used for the flow update's
 *                       problem (MinCostFlow), Sec. 3.1-3.2.
 *
 * Cost: c(x,y) = |x - y|^2 with explicit 2D coordinates; everything float64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static double sqdist(const double* x, const double* y) {
    double d0 = x[0] - y[0], d1 = x[1] - y[1];
    return d0 * d0 + d1 * d1;
}

/*
 * One cell.  X points k = 0..nx-1 with coordinates xc[2k..2k+1] and masses
 * mu[k] >= 0; Y points l = 0..ny-1 with coordinates yc, cell target marginal
 * nuJ[l] > 0 and reference marginal nuref[l] >= nuJ[l] > 0.
 *
 * Y-update (makes the Y-marginal equal nuJ):
 *   beta(y) = eps*log(nuJ(y)/nu(y)) - eps*log sum_x exp((alpha(x)-c(x,y))/eps) mu(x)
 * X-marginal of the current plan:
 *   pX(x) = mu(x) * sum_y exp((alpha(x)+beta(y)-c(x,y))/eps) nu(y)
 * X-update (makes the X-marginal equal mu):
 *   alpha(x) = -eps*log sum_y exp((beta(y)-c(x,y))/eps) nu(y)
 * Log-sum-exp is the textbook max-shifted form.
 */
static void cell_y_update(int nx, const double* xc, const double* mu, int ny, const double* yc,
                          const double* nuJ, const double* nuref, double eps, const double* alpha,
                          double* beta) {
    double* lmu = (double*)malloc(sizeof(double) * (size_t)(nx > 0 ? nx : 1));
    for (int k = 0; k < nx; ++k) lmu[k] = (mu[k] > 0.0) ? log(mu[k]) : -INFINITY;
    for (int l = 0; l < ny; ++l) {
        double m = -INFINITY;
        for (int k = 0; k < nx; ++k) {
            if (mu[k] <= 0.0) continue;
            double v = (alpha[k] - sqdist(xc + 2 * k, yc + 2 * l)) / eps + lmu[k];
            if (v > m) m = v;
        }
        double s = 0.0;
        for (int k = 0; k < nx; ++k) {
            if (mu[k] <= 0.0) continue;
            double v = (alpha[k] - sqdist(xc + 2 * k, yc + 2 * l)) / eps + lmu[k];
            s += exp(v - m);
        }
        beta[l] = eps * log(nuJ[l] / nuref[l]) - eps * (m + log(s));
    }
    free(lmu);
}

/* log sum_y exp((beta(y) - c(x,y))/eps) nu(y) for every x */
static void cell_x_lse(int nx, const double* xc, int ny, const double* yc, const double* nuref,
                       double eps, const double* beta, double* out) {
    double* lnu = (double*)malloc(sizeof(double) * (size_t)(ny > 0 ? ny : 1));
    for (int l = 0; l < ny; ++l) lnu[l] = log(nuref[l]);
    for (int k = 0; k < nx; ++k) {
        double m = -INFINITY;
        for (int l = 0; l < ny; ++l) {
            double v = (beta[l] - sqdist(xc + 2 * k, yc + 2 * l)) / eps + lnu[l];
            if (v > m) m = v;
        }
        double s = 0.0;
        for (int l = 0; l < ny; ++l) {
            double v = (beta[l] - sqdist(xc + 2 * k, yc + 2 * l)) / eps + lnu[l];
            s += exp(v - m);
        }
        out[k] = m + log(s);
    }
    free(lnu);
}

/* L1 error of the X-marginal of the current plan against mu (after a Y-update) */
static double cell_x_error(int nx, const double* mu, double eps, const double* alpha,
                           const double* lse) {
    double e = 0.0;
    for (int k = 0; k < nx; ++k) {
        if (mu[k] <= 0.0) continue;
        double px = mu[k] * exp(alpha[k] / eps + lse[k]);
        e += fabs(px - mu[k]);
    }
    return e;
}

/*
 * Batch of cells, packed: cell j owns X points xoff[j]..xoff[j+1]-1 and Y
 * points yoff[j]..yoff[j+1]-1.
 *
 * One Sinkhorn iteration = Y-update, then the X-marginal error, then (unless
 * stopped) the X-update.  The solve therefore always ends on a Y-update.
 *
 * rule 0 (batch, as in the paper): stop after the Y-update of iteration k
 *   once sum_J err_J <= tol * sum_J mu(X_J), or when k == max_iter.
 * rule 1 (per cell): cell J stops once err_J <= tol * mu(X_J) or k == max_iter.
 * fixed_iters > 0 overrides both: exactly fixed_iters Y-updates.
 *
 * alpha: in = initial X potential (energy units), out = final; beta: out.
 * iters[j], err[j]: iterations run and final error per cell.
 * Returns the number of iterations of the batch (max over cells).
 */
int orc_sinkhorn_cells(int ncells, const int64_t* xoff, const double* xc, const double* mu,
                       const int64_t* yoff, const double* yc, const double* nuJ,
                       const double* nuref, double eps, double tol, int max_iter, int fixed_iters,
                       int rule, double* alpha, double* beta, int* iters, double* err,
                       int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t nxtot = xoff[ncells];
    double* lse = (double*)malloc(sizeof(double) * (size_t)(nxtot > 0 ? nxtot : 1));
    char* active = (char*)malloc((size_t)(ncells > 0 ? ncells : 1));
    double mass = 0.0;
    for (int j = 0; j < ncells; ++j) {
        active[j] = 1;
        iters[j] = 0;
        err[j] = 0.0;
        for (int64_t k = xoff[j]; k < xoff[j + 1]; ++k) mass += mu[k];
    }
    int limit = fixed_iters > 0 ? fixed_iters : max_iter;
    int k_done = 0;
    for (int it = 1; it <= limit; ++it) {
        double total = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
        for (int j = 0; j < ncells; ++j) {
            if (!active[j]) continue;
            int nx = (int)(xoff[j + 1] - xoff[j]);
            int ny = (int)(yoff[j + 1] - yoff[j]);
            const double* X = xc + 2 * xoff[j];
            const double* Y = yc + 2 * yoff[j];
            cell_y_update(nx, X, mu + xoff[j], ny, Y, nuJ + yoff[j], nuref + yoff[j], eps,
                          alpha + xoff[j], beta + yoff[j]);
            cell_x_lse(nx, X, ny, Y, nuref + yoff[j], eps, beta + yoff[j], lse + xoff[j]);
            err[j] = cell_x_error(nx, mu + xoff[j], eps, alpha + xoff[j], lse + xoff[j]);
            iters[j] = it;
            total += err[j];
        }
        k_done = it;
        int stop_all = (it == limit);
        if (fixed_iters <= 0 && rule == 0 && total <= tol * mass) stop_all = 1;
        if (stop_all) break;
        int any = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : any)
        for (int j = 0; j < ncells; ++j) {
            if (!active[j]) continue;
            double mj = 0.0;
            for (int64_t k = xoff[j]; k < xoff[j + 1]; ++k) mj += mu[k];
            if (fixed_iters <= 0 && rule == 1 && err[j] <= tol * mj) {
                active[j] = 0;
                continue;
            }
            any = 1;
            for (int64_t k = xoff[j]; k < xoff[j + 1]; ++k)
                alpha[k] = (mu[k] > 0.0) ? -eps * lse[k] : 0.0;
        }
        if (!any) break;
    }
    free(lse);
    free(active);
    return k_done;
}

/* pi(x,y) = exp((alpha(x)+beta(y)-c(x,y))/eps) mu(x) nu(y), dense nx*ny row-major */
void orc_cell_plan(int nx, const double* xc, const double* mu, const double* alpha, int ny,
                   const double* yc, const double* nuref, const double* beta, double eps,
                   double* plan) {
    for (int k = 0; k < nx; ++k)
        for (int l = 0; l < ny; ++l) {
            double v = (alpha[k] + beta[l] - sqdist(xc + 2 * k, yc + 2 * l)) / eps;
            plan[(size_t)k * ny + l] = (mu[k] > 0.0) ? exp(v) * mu[k] * nuref[l] : 0.0;
        }
}

/* ------------------------------------------------------------------------ */
/* Min-cost flow: successive shortest paths on integers.                     */
/*                                                                          */
/* Bipartite transportation graph: left nodes 0..n-1 with supply sup[i] and  */
/* right nodes 0..n-1 with demand dem[j]; arcs a = 0..m-1 from left tail[a]  */
/* to right head[a] with integer cost cost[a] and unbounded capacity.        */
/* Sum of supplies must equal sum of demands.  Each round runs Dijkstra from */
/* all left nodes with remaining supply over the residual graph with reduced */
/* costs, then pushes along the shortest path to the nearest right node with */
/* remaining demand.  Returns 0 on success, -1 if infeasible.               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t key;
    int node;
} heap_item;

static void heap_push(heap_item* h, int* n, heap_item it) {
    int i = (*n)++;
    h[i] = it;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h[p].key <= h[i].key) break;
        heap_item t = h[p];
        h[p] = h[i];
        h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item* h, int* n) {
    heap_item top = h[0];
    h[0] = h[--(*n)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, s = i;
        if (l < *n && h[l].key < h[s].key) s = l;
        if (r < *n && h[r].key < h[s].key) s = r;
        if (s == i) break;
        heap_item t = h[s];
        h[s] = h[i];
        h[i] = t;
        i = s;
    }
    return top;
}

int orc_mcf_ssp(int n, int m, const int32_t* tail, const int32_t* head, const int64_t* cost,
                const int64_t* sup, const int64_t* dem, int64_t* flow, int64_t* pot_out) {
    /* node ids: left i -> i, right j -> n + j */
    int V = 2 * n;
    const int64_t INF = INT64_MAX / 4;
    int64_t* rs = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* rd = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* pot = (int64_t*)calloc((size_t)V, sizeof(int64_t));
    int64_t* dist = (int64_t*)malloc(sizeof(int64_t) * V);
    int* pred_arc = (int*)malloc(sizeof(int) * V); /* arc index; sign: >=0 forward, <0 backward */
    char* done = (char*)malloc((size_t)V);
    heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (size_t)(2 * m + V + 1));
    /* adjacency: out-arcs of left nodes (forward), in-arcs of right nodes (backward residual) */
    int* lstart = (int*)calloc((size_t)n + 1, sizeof(int));
    int* rstart = (int*)calloc((size_t)n + 1, sizeof(int));
    int* ladj = (int*)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    int* radj = (int*)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int a = 0; a < m; ++a) {
        lstart[tail[a] + 1]++;
        rstart[head[a] + 1]++;
        flow[a] = 0;
    }
    for (int i = 0; i < n; ++i) {
        lstart[i + 1] += lstart[i];
        rstart[i + 1] += rstart[i];
    }
    {
        int* lp = (int*)malloc(sizeof(int) * (size_t)n);
        int* rp = (int*)malloc(sizeof(int) * (size_t)n);
        memcpy(lp, lstart, sizeof(int) * (size_t)n);
        memcpy(rp, rstart, sizeof(int) * (size_t)n);
        for (int a = 0; a < m; ++a) {
            ladj[lp[tail[a]]++] = a;
            radj[rp[head[a]]++] = a;
        }
        free(lp);
        free(rp);
    }
    int64_t tot_s = 0, tot_d = 0;
    for (int i = 0; i < n; ++i) {
        rs[i] = sup[i];
        rd[i] = dem[i];
        tot_s += sup[i];
        tot_d += dem[i];
    }
    int status = 0;
    if (tot_s != tot_d) status = -1;
    /* initial potentials: left 0, right = min incoming arc cost (graph is a DAG left->right) */
    for (int j = 0; j < n; ++j) {
        int64_t best = INF;
        for (int q = rstart[j]; q < rstart[j + 1]; ++q)
            if (cost[radj[q]] < best) best = cost[radj[q]];
        pot[n + j] = (best == INF) ? 0 : best;
    }
    int64_t remaining = tot_s;
    while (status == 0 && remaining > 0) {
        for (int v = 0; v < V; ++v) {
            dist[v] = INF;
            done[v] = 0;
            pred_arc[v] = INT32_MIN;
        }
        int hn = 0;
        for (int i = 0; i < n; ++i)
            if (rs[i] > 0) {
                dist[i] = 0;
                heap_push(heap, &hn, (heap_item){0, i});
            }
        int target = -1;
        while (hn > 0) {
            heap_item it = heap_pop(heap, &hn);
            int u = it.node;
            if (done[u] || it.key != dist[u]) continue;
            done[u] = 1;
            if (u >= n && rd[u - n] > 0) {
                target = u;
                break;
            }
            if (u < n) {
                for (int q = lstart[u]; q < lstart[u + 1]; ++q) {
                    int a = ladj[q];
                    int v = n + head[a];
                    int64_t rc = cost[a] + pot[u] - pot[v];
                    if (dist[u] + rc < dist[v]) {
                        dist[v] = dist[u] + rc;
                        pred_arc[v] = a;
                        heap_push(heap, &hn, (heap_item){dist[v], v});
                    }
                }
            } else {
                int j = u - n;
                for (int q = rstart[j]; q < rstart[j + 1]; ++q) {
                    int a = radj[q];
                    if (flow[a] <= 0) continue;
                    int v = tail[a];
                    int64_t rc = -cost[a] + pot[u] - pot[v];
                    if (dist[u] + rc < dist[v]) {
                        dist[v] = dist[u] + rc;
                        pred_arc[v] = -a - 1;
                        heap_push(heap, &hn, (heap_item){dist[v], v});
                    }
                }
            }
        }
        if (target < 0) {
            status = -1;
            break;
        }
        int64_t dt = dist[target];
        for (int v = 0; v < V; ++v) {
            if (done[v]) pot[v] += dist[v] - dt;
        }
        /* bottleneck: remaining supply at the path source, demand at target, reverse flows */
        int64_t push = rd[target - n];
        int v = target;
        while (pred_arc[v] != INT32_MIN) {
            int pa = pred_arc[v];
            if (pa >= 0) {
                v = tail[pa];
            } else {
                int a = -pa - 1;
                if (flow[a] < push) push = flow[a];
                v = n + head[a];
            }
        }
        if (rs[v] < push) push = rs[v];
        int src = v;
        v = target;
        while (pred_arc[v] != INT32_MIN) {
            int pa = pred_arc[v];
            if (pa >= 0) {
                flow[pa] += push;
                v = tail[pa];
            } else {
                int a = -pa - 1;
                flow[a] -= push;
                v = n + head[a];
            }
        }
        rs[src] -= push;
        rd[target - n] -= push;
        remaining -= push;
    }
    if (pot_out)
        for (int v = 0; v < V; ++v) pot_out[v] = pot[v];
    free(rs);
    free(rd);
    free(pot);
    free(dist);
    free(pred_arc);
    free(done);
    free(heap);
    free(lstart);
    free(rstart);
    free(ladj);
    free(radj);
    return status;
}
