/*
 * domdec.h -- C ABI of the MI355X (gfx950) domain-decomposition library for
 * entropic optimal transport with flow updates (Medina & Schmitzer, "Flow
 * updates for domain decomposition of entropic optimal transport").
 *
 * Problem (Sec. 2.2, eq. entropic-transport): mu, nu are probability measures
 * on the same regular N x N pixel grid of [0,1]^2 (pixel (k1,k2) has centre
 * ((k1+1/2)h, (k2+1/2)h), h = 1/N, row-major, k1 slow), cost c(x,y) = |x-y|^2,
 * regularisation eps > 0.  The library keeps a feasible coupling as its basic
 * cell Y-marginals nu_i (Sec. 2.3 eq. basic-cell-Y-marginal) in per-cell
 * bounding boxes (App. A.1 "Bounding box representation") on the device, and
 * updates it by domain-decomposition iterations (Alg. "DomDecIter", App. A
 * Alg. "DomDecIterGPU") and flow updates (Sec. 3.2 Def. "Flow update").
 *
 * Conventions for every entry point:
 *   - No function aborts or exits.  A status is returned; every status other
 *     than DD_OK / DD_NOTCONV leaves a message readable by domdec_strerror.
 *   - DD_NOTCONV is a warning: max_iter was reached before the tolerance.
 *   - Pointers marked (host) are host memory, (dev) device memory of the
 *     current HIP device.  The caller owns every pointer it passes in; the
 *     library copies what it keeps.  A dd_ctx owns its device memory and
 *     releases it in domdec_free.
 *   - Streams are hipStream_t passed as void*; NULL means the null stream.
 *     Entry points that return statistics synchronise that stream.
 *   - One dd_ctx must not be used by two host threads at once.
 */
#ifndef DOMDEC_H
#define DOMDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DD_OK = 0,
    DD_NOTCONV = 1,    /* warning: iteration limit hit before the tolerance        */
    DD_EINVAL = -1,    /* invalid argument (shape, value, NaN, unsupported option) */
    DD_ENOMEM = -2,    /* device or host allocation failed                         */
    DD_EDEVICE = -3,   /* a HIP call failed                                        */
    DD_ESTATE = -4,    /* call out of order (e.g. flow_update before a B iteration)*/
    DD_ENUMERIC = -5   /* a non-finite value appeared in a reduction               */
} dd_status;

enum { DD_PREC_F32 = 0, DD_PREC_F64 = 1 };      /* arithmetic of the cell log-sum-exp */
enum { DD_STOP_BATCH = 0, DD_STOP_CELL = 1 };   /* Sinkhorn stopping rule             */
enum { DD_INIT_ZERO = 0, DD_INIT_PREV = 1, DD_INIT_NET = 2 }; /* X-potential start        */
enum { DD_PART_A = 0, DD_PART_B = 1 };          /* composite partition                */

/* Sinkhorn options (App. A.2.1 "Stopping criterion and measure truncation").
 * One iteration = Y-update, X-marginal L1 error, then (unless stopped) the
 * X-update; a solve always ends on a Y-update, so the Y-marginal is exact.
 *   DD_STOP_BATCH: stop once sum_J err_J <= tol * sum_J mu(X_J) (the paper's rule).
 *   DD_STOP_CELL : cell J stops once err_J <= tol * mu(X_J); this implies the batch
 *                  rule, so it never loosens the tolerance.
 *   fixed_iters > 0: exactly fixed_iters Y-updates per cell, tol ignored.          */
typedef struct {
    double tol;           /* Err, e.g. 1e-5                                        */
    int32_t max_iter;     /* iteration cap (>= 1)                                  */
    int32_t fixed_iters;  /* 0 = use tol                                           */
    int32_t stop_rule;    /* DD_STOP_BATCH | DD_STOP_CELL                          */
    int32_t check_every;  /* batch rule, k (0 = 8).  The float32 register-blocked
                             path tests the error after 4k iterations, again 4k later,
                             then after 80% of the iterations the decay of the last two
                             tests predicts are still needed (at least k, at most 32k);
                             its stop trails the first iteration that meets the rule by
                             the overshoot of the last prediction (< k when the error
                             decays no faster than predicted), which only lowers the
                             error.  The other kernels test every iteration and poll
                             the flag every k launches                                 */
    int32_t init;         /* DD_INIT_ZERO | PREV | NET (domdec_iterate only)      */
    int32_t reserved;     /* must be 0                                             */
} dd_sinkhorn_opts;

/* Statistics of one batched cell solve. */
typedef struct {
    int32_t ncells;
    int32_t iters_max;         /* iterations of the batch (max over cells), both phases
                                  of a float32 solve with its float64 finish              */
    int32_t iters_min;
    int32_t converged;         /* 1 if the stopping rule was met                       */
    int64_t cell_iters;        /* sum over cells of iterations run                     */
    double err;                /* final sum over cells of X-marginal L1 errors         */
    double mass;               /* sum over cells of mu(X_J)                            */
    double lse_terms;          /* log-sum-exp terms evaluated (exponentials)           */
    double alg_bytes;          /* algorithmic bytes: 12 (|X_J| + W1 W2) per cell-iter  */
    double time_ms;            /* device time of the whole solve (HIP events)          */
    double main_ms;            /* device time of the main (float32 or float64) loop    */
    int32_t finish_iters_max;  /* of those, float64-finish iterations (tolerance mode)  */
    int32_t n_big;             /* cells solved by a whole workgroup (the rest by a wave) */
    int32_t n_giant;           /* of those, cells in the whole-CU-LDS launch             */
    int32_t lds_kb[2];         /* LDS budget per workgroup, small and big launches (KB)  */
    int32_t tile_small[2];     /* LDS tile of the small-cell launch (W1, W2)             */
    int32_t tile_big[2];       /* LDS tile of the big-cell launch (W1, W2)               */
    int32_t path;              /* 0: general kernels; 1: register-blocked float32 path for
                                  8 x 8 blocks.  For path 1: n_big = cells solved by a
                                  workgroup (the rest one per wave), n_giant = of those, the
                                  cells of more than 2048 box entries (eight waves each, the
                                  others four); lds_kb = LDS per workgroup of the wave class
                                  and the largest of the workgroup classes; fallback counts:
                                  tile_small = first-X-pass outputs held as upper bounds,
                                  exact second-X-pass outputs; tile_big = second-X-pass
                                  repeats after exact first-pass outputs, wave blocks with
                                  exact Y-update entries                                    */
    int32_t kernel_launches[3]; /* path 1, batch rule: launches per class (0: one wave per
                                   cell; 1: four waves per cell; 2: eight waves per cell),
                                   the final g launch and the launches after the stop (which
                                   exit at once) included                                   */
    int32_t wave_side;         /* path 1: the class thresholds used -- boxes whose long side
                                  is at most wave_side take one wave, ...                   */
    double kernel_ms[3];       /* their summed duration (HIP events on each launch's stream) */
    double kernel_terms[3];    /* LSE terms they evaluated                                   */
    int32_t big_entries;       /* ... boxes of more entries than this eight waves, the rest
                                  four (sinkhorn_set_classes; the tuner's pick otherwise)    */
    int32_t reserved4;
} dd_batch_stats;

/*
 * sinkhorn_batch / sinkhorn_batch_f64 -- batched log-domain cell Sinkhorn
 * (App. A.1 "Custom CUDA Sinkhorn": batched, log-domain, online cost,
 * separable for the squared cost; the cell problem of Alg. "DomDecIter").
 *
 * Cell c has an X block of xside x xside pixels (local index i = (i1,i2),
 * row-major) and a Y box of W1 x W2 pixels (local j = (j1,j2), row-major).
 * With an integer gauge shift E = (E1,E2) per cell and kappa = eps / h^2 > 0
 * the local cost is
 *     C(i,j) = ((i1 - j1 + E1)^2 + (i2 - j2 + E2)^2) / kappa.
 * For an X block at pixel origin pX and a Y box at pixel origin pY the true
 * cost |x - y|^2 / eps equals |pX - pY + i - j|^2 / kappa, which differs from
 * C by f(i) + g(j); such terms leave the optimal plan unchanged (they move
 * into the potentials), so the plan solved here is the paper's cell plan for
 * any choice of E.  A shift near the mean displacement keeps the potentials
 * small, which is what lets float32 reach tol = 1e-5.
 *
 * Potentials f = alpha/eps (X) and g = beta/eps (Y) are taken with reference measure
 * mu_J (x) nu_J, which differs from the paper's mu_J (x) nu by a constant (Sec. 2.3):
 *     pi(i,j) = mu(i) nu_J(j) exp(f(i) + g(j) - C(i,j))
 *     g(j) = -LSE_i [f(i) + log mu(i) - C(i,j)]                   (Y-update)
 *     err  = sum_i mu(i) |exp(f(i) + LSE_j[g(j) + log nu_J(j) - C(i,j)]) - 1|
 *     f(i) = -LSE_j [g(j) + log nu_J(j) - C(i,j)]                 (X-update)
 * Each LSE runs as two 1D passes, one per axis (the cost is separable).
 * Arguments (all arrays (dev), cells packed in order c = 0..ncells-1):
 *   xside         X block side (2..16); each cell's X block has xside^2 entries.
 *   dims          int32 [ncells][2]: W1, W2 >= 1.
 *   base          int64 [ncells]: offset of cell c's Y box in lognu and b.
 *   shift         int32 [ncells][2]: E1, E2.
 *   logmu         [ncells][xside^2]: log mu; entries <= -1e30 mark zero mass.
 *   lognu         packed Y boxes: log nu_J; entries <= -1e30 mark zero mass.
 *   a             [ncells][xside^2] in: initial f; out: final f.
 *   b             packed Y boxes, out: final g (g of the last Y-update).
 *   kappa         eps / h^2.
 *   max_w1/max_w2 upper bounds of W1, W2 over the batch (size the on-chip tiles).
 *   opts          (host) options; init and reserved are ignored here.
 *   cell_iters    int32 [ncells] out, may be NULL: iterations per cell (Y-updates of
 *                 the iterate sequence; after a float64 finish both phases, the
 *                 finish's first Y-update -- the float32 phase's last one repeated in
 *                 float64 -- counted once).  A fixed count from the same start
 *                 reproduces the solve.
 *   cell_err      double [ncells] out, may be NULL: final error per cell.
 *   stream        hipStream_t; the call synchronises it before returning.
 *   stats         (host) out, may be NULL.
 * Errors: DD_EINVAL for ncells < 0, xside outside [2,16], kappa <= 0, a cell
 * whose W1/W2 exceed max_w1/max_w2 or is < 1, or bad opts; DD_ENUMERIC if an
 * error sum is not finite; DD_NOTCONV when max_iter stopped the solve.
 * Inputs, potentials and outputs are float64 in both entry points.  sinkhorn_batch
 * evaluates the log-sum-exp terms in float32, each 1D pass on values shifted by a
 * float64 maximum of its input line (so every float32 term is O(1)), with float64
 * line offsets, potentials, errors and masses.  When it stops on a tolerance, the
 * same rule then continues in float64 from the float32 state until the float64
 * error meets the tolerance (usually one Y-update), so the tolerance holds in
 * float64.  sinkhorn_batch_f64 is float64 throughout.  Y boxes too large for one
 * workgroup's LDS run from global memory (L2-resident) instead.
 */
dd_status sinkhorn_batch(int32_t ncells, int32_t xside, const int32_t* dims, const int64_t* base,
                         const int32_t* shift, const double* logmu, const double* lognu,
                         double* a, double* b, double kappa, int32_t max_w1, int32_t max_w2,
                         const dd_sinkhorn_opts* opts, int32_t* cell_iters, double* cell_err,
                         void* stream, dd_batch_stats* stats);

dd_status sinkhorn_batch_f64(int32_t ncells, int32_t xside, const int32_t* dims,
                             const int64_t* base, const int32_t* shift, const double* logmu,
                             const double* lognu, double* a, double* b, double kappa,
                             int32_t max_w1, int32_t max_w2, const dd_sinkhorn_opts* opts,
                             int32_t* cell_iters, double* cell_err, void* stream,
                             dd_batch_stats* stats);

/*
 * sinkhorn_batch_noalloc -- sinkhorn_batch for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, arithmetic, stopping rules and results as sinkhorn_batch; it calls no
 * hipMalloc / hipFree and creates no streams, events or graphs.  Its workspace (control
 * words, per-cell errors, masses and counts, the second X-potential buffer, processing
 * orders, global scratch for boxes beyond the on-chip tiles) is carved from one fixed
 * 64 MiB device buffer per GPU, held by the library until the process ends.  All of the
 * work runs on `stream` (the cell classes one after the other instead of side by side), and
 * the statistics carry no times (time_ms, main_ms and kernel_ms are 0).
 * Calls that overlap on one GPU share that buffer and race: serialise them.  The buffer
 * keeps the last call's contents; every call initialises what it reads.
 * Errors: those of sinkhorn_batch, and DD_EINVAL when the batch needs more workspace than
 * the buffer holds (roughly 0.6 KB per cell with 8 x 8 blocks, plus the global scratch of the
 * largest boxes); nothing is written to a or b then.
 */
/*
 * sinkhorn_set_classes -- the cell classes of the register-blocked float32 path (8 x 8 X
 * blocks; the launch side of App. A.1 "Batching and clustering"): boxes whose long side is at
 * most wave_side (8..32) are solved by one wave each, boxes of more than big_entries
 * (64..65536) entries by eight waves, the rest by four.  (0, 0) -- the default -- hands the
 * choice to the library's tuner, which then starts afresh: per key (stopping mode, mean box
 * area in powers of four, cell count in powers of two) it tries every candidate pair on
 * consecutive solves, then keeps the one with the least float32 device time per LSE term (the
 * first, measured default, unless another is faster by more than 3%); a
 * solve's pick is reported in dd_batch_stats.wave_side / big_entries.  The choice changes
 * which kernel solves a cell, not the iteration: results agree to float32 rounding (the
 * one-wave kernel holds log nu_J in float32 registers, the others read it in float64).
 * Process-wide; not safe against concurrent solves.  Errors: DD_EINVAL (out of range).
 */
dd_status sinkhorn_set_classes(int32_t wave_side, int32_t big_entries);

dd_status sinkhorn_batch_noalloc(int32_t ncells, int32_t xside, const int32_t* dims,
                                 const int64_t* base, const int32_t* shift, const double* logmu,
                                 const double* lognu, double* a, double* b, double kappa,
                                 int32_t max_w1, int32_t max_w2, const dd_sinkhorn_opts* opts,
                                 int32_t* cell_iters, double* cell_err, void* stream,
                                 dd_batch_stats* stats);

/* Statistics of a global Sinkhorn solve. */
typedef struct {
    int32_t iters;       /* Y-updates run                                              */
    int32_t converged;   /* 1 if the tolerance (or the fixed count) was reached         */
    double err;          /* X-marginal L1 error of the returned pair                    */
    double time_ms;      /* device time of the solve (HIP events)                       */
    double lse_terms;    /* log-sum-exp terms evaluated: 4 N^3 per iteration            */
} dd_global_stats;

/*
 * global_sinkhorn -- entropic OT on the whole N x N grid by log-domain Sinkhorn, without
 * domain decomposition: the comparison solver of App. A.2.1 ("Compared algorithms and
 * implementations", a global GPU Sinkhorn).  It solves eq. (entropic-transport) as the
 * single-cell problem X = Y = the grid, with the cell solver's iteration and stopping rule:
 * one iteration = Y-update, X-marginal L1 error, then (unless stopped) X-update; stop once
 * err <= opts->tol (mu, nu are probability measures), or after opts->fixed_iters Y-updates.
 * Float64 throughout; each log-sum-exp is two exact 1D passes (the cost is separable).
 *   n          grid side N (1..4096; 4 N doubles must fit the LDS of a workgroup).
 *   mu, nu     (dev) float64 [N*N], row-major, >= 0 (zero entries are zero mass).
 *   eps        regularisation, > 0 (the cost is |x - y|^2 on pixel centres of [0,1]^2).
 *   alpha      (dev) float64 [N*N] in: starting X potential (energy units; zeros for a cold
 *              start, the previous solution for eps-scaling); out: alpha of the last Y-update.
 *   beta       (dev) float64 [N*N] out: beta (energy units; reference measure mu (x) nu, so
 *              pi = exp((alpha + beta - |x - y|^2) / eps) mu nu); meaningless where nu = 0.
 *   opts       (host) tol, max_iter, fixed_iters; stop_rule, check_every, init ignored.
 *   stream     hipStream_t; the call synchronises it (it reads the error every iteration).
 *   stats      (host) out, may be NULL.
 * Work arrays (6 N^2 doubles) are allocated per call.
 * Errors: DD_EINVAL, DD_ENOMEM, DD_EDEVICE, DD_ENUMERIC, DD_NOTCONV (warning).
 */
dd_status global_sinkhorn(int32_t n, const double* mu, const double* nu, double eps,
                          double* alpha, double* beta, const dd_sinkhorn_opts* opts,
                          void* stream, dd_global_stats* stats);

/* ------------------------------------------------------------------------- */
/* Domain-decomposition context                                              */
/* ------------------------------------------------------------------------- */

typedef struct dd_ctx dd_ctx;

typedef struct {
    int32_t n;         /* grid side N                                              */
    int32_t s;         /* basic cell side; N % (2 s) == 0, 1 <= s <= 8              */
    double trunc;      /* truncation threshold for nu_i entries (e.g. 1e-15)       */
    int32_t prec;      /* DD_PREC_F32 | DD_PREC_F64                                */
    int32_t levels;    /* coarser layers of multiscale DD below the N x N grid
                          (0: single scale).  With L > 0 the context starts on the
                          (N / 2^L)^2 layer; domdec_refine moves to the next finer one.
                          N / 2^L must be a multiple of 2 s.                        */
    /* Device-memory supplier (optional; both NULL: hipMalloc / hipFree).  With both set,
       every device buffer of the context -- its layers, the stored nu_i, the composite work,
       the cell solver's and the dual's workspaces and the flow update's structures -- comes
       from dev_alloc(bytes, alloc_ud) and goes back through dev_free(ptr, alloc_ud), e.g. a
       caching allocator of the caller's framework.  The memory must be usable on the
       context's stream; the library returns a buffer only after every kernel that touches it
       has been ordered before the return on that stream, so a stream-ordered caching
       allocator may hand it out again at once.  dev_alloc returning NULL fails the call with
       DD_ENOMEM.  The hooks run on the calling thread, from domdec_* / extract_* / flow_*
       calls and domdec_free, never from a device callback.  Context-free entry points
       (sinkhorn_batch, global_sinkhorn) and dd_net keep hipMalloc.                       */
    void* (*dev_alloc)(size_t bytes, void* alloc_ud);
    void (*dev_free)(void* ptr, void* alloc_ud);
    void* alloc_ud;
} dd_params;

/*
 * domdec_init -- set up partitions and the initial coupling (Def. "Basic and
 * composite partitions"; Alg. "DomDec" input pi_init; App. A.2.1 "Basic and
 * composite partitions").
 *   Basic cells are the s x s pixel blocks, i = r * (N/s) + c.  Partition A
 *   groups 2x2 basic cells from the origin; partition B groups 2x2 basic cells
 *   shifted by one basic cell, boundary cells keep their in-range members (on
 *   the device they are padded to 2s x 2s with zero mass, which leaves every
 *   plan unchanged).
 *   mu, nu     (host) float64 [N*N], >= 0, each summing to 1 within 1e-12;
 *              every basic cell needs m_i = mu(X_i) > 0.
 *   n_init     0 for the product coupling nu_i = m_i nu; else the number of
 *              entries of a sparse initial coupling given by
 *   init_x, init_y (host) int64 [n_init] flat pixel indices and
 *   init_m     (host) float64 [n_init] masses; the coupling must have marginals
 *              mu and nu within 1e-12 (checked).
 *   stream     hipStream_t for all later work of this context.
 *   out        receives the context (NULL on failure).
 * Multiscale (params.levels = L > 0; App. A.2.1 "Multi-scale and eps-scaling", Sec. 5.3):
 *   the layers are the 2 x 2 block sums of mu and nu, L times; the context starts on the
 *   coarsest, with the initial coupling summed over the same blocks (the product coupling of
 *   the coarsest layer when n_init == 0).
 * Errors: DD_EINVAL (shapes, negative/NaN masses, sums, m_i == 0, marginals),
 * DD_ENOMEM, DD_EDEVICE.
 */
dd_status domdec_init(const dd_params* params, const double* mu, const double* nu, int64_t n_init,
                      const int64_t* init_x, const int64_t* init_y, const double* init_m,
                      void* stream, dd_ctx** out);

/* Statistics of one domain-decomposition iteration. */
typedef struct {
    dd_batch_stats sk;        /* the cell solve                                       */
    int32_t partition;
    int32_t max_w1, max_w2;   /* largest composite Y box                              */
    int32_t grid_n;           /* grid side of the current layer                       */
    int64_t nu_entries;       /* stored nu_i entries after truncation                 */
    int64_t comp_entries;     /* composite Y-box entries solved                       */
    double t_b2c_ms;          /* BasicToComposite                                     */
    double t_sinkhorn_ms;     /* cell solve                                           */
    double t_c2b_ms;          /* CompositeToBasic + balancing + truncation            */
    double t_total_ms;        /* whole iteration (device)                             */
    double t_init_ms;         /* X-potential start (warm start, or the net's features,
                                 inference and X-update) before the Sinkhorn solve     */
    int32_t batches;          /* composite-cell batches solved one after another       */
    int32_t host_waits;       /* times the host waited for the device during the call:
                                 1 in the steady state of one batch (the iteration's
                                 composite boxes come from the previous iteration, and
                                 the solve is enqueued whole; its end is the one wait)  */
    int64_t peak_comp_entries;/* composite Y-box entries of the largest batch: the size
                                 of the composite work arrays (7 doubles per entry)    */
    int32_t spec_resumed;     /* 1 when the solve enqueued whole was not enough and was
                                 continued after the wait (the same result either way) */
    int32_t reserved4;
} dd_iter_stats;

/*
 * domdec_iterate -- one domain-decomposition iteration on partition A or B
 * (Alg. "DomDecIter"; App. A Alg. "DomDecIterGPU" without the batch loop: all
 * composite cells run in one launch):
 *   BasicToComposite (eq. get-composite-cell-marginal), batched cell Sinkhorn
 *   at regularisation eps, CompositeToBasic (App. A.1 "Online reduction for
 *   basic cell marginals"), balancing, truncation below params.trunc.
 *   X-potentials persist per partition: opts.init = DD_INIT_PREV warm-starts
 *   from the previous visit of this partition (alpha kept in energy units across
 *   eps changes), DD_INIT_ZERO starts from zero.
 *   stats (host) may be NULL.  Synchronises the context stream.
 *   Host waits: in the steady state one, at the end.  The composite boxes come
 *   from the end of the previous call (any other call that changes the state
 *   drops them, and the next call reads them back); under the batch rule with
 *   float32 terms and max_iter >= 4 * 32 * check_every + 4, the float32 rounds
 *   and the first float64-finish iterations are enqueued without waiting and
 *   continued after the wait if they were not enough (the same iterations and
 *   results either way).  DD_SPEC=0 in the environment turns the speculative
 *   enqueueing off; DD_SPEC_FINISH=n (0..8) sets the float64-finish iterations
 *   enqueued ahead (default 2).
 * Errors: DD_EINVAL (partition, eps <= 0, opts), DD_ENOMEM (a box outgrew the
 * on-chip limit or memory), DD_ENUMERIC, DD_NOTCONV (warning), DD_EDEVICE (a
 * kernel failed, or the predicted composite boxes differed from the state's).
 */
dd_status domdec_iterate(dd_ctx* ctx, int32_t partition, double eps,
                         const dd_sinkhorn_opts* opts, dd_iter_stats* stats);

/*
 * domdec_set_clusters -- batching and clustering of the composite cells (App. A.1 "Batching
 * and clustering"; App. A.2.1 "Batching and clustering", which uses one cluster up to
 * N = 256 and N / 256 clusters above).  With k > 1 every later domdec_iterate clusters the
 * partition's composite cells by K-means on their Y-box dimensions (W1, W2) into at most k
 * clusters and solves them one after another as separate batches (CreateBatches): each batch
 * runs BasicToComposite, the start, the cell solve with its own stopping rule (the batch rule
 * then holds per batch, as in the paper), CompositeToBasic, balancing and truncation, and
 * the new basic-cell Y-marginals are assembled once every batch is done (CombineBatches).
 * The composite work arrays then hold the largest batch only (dd_iter_stats.
 * peak_comp_entries).  Each cell's result does not depend on its batch: at fixed iteration
 * counts or with DD_STOP_CELL the state is the same as unbatched.  After a batched
 * iteration the composite plans are not kept whole, so domdec_evaluate reports the basic-
 * cell quantities only (primal, dual, X-marginal NaN), and extract_potentials without beta;
 * flow_update needs an unbatched B iteration.  DD_INIT_NET runs unbatched only.
 * k = 1 (the default) restores the single batch.  The setting carries over domdec_refine.
 * Errors: DD_EINVAL (k < 1).
 */
dd_status domdec_set_clusters(dd_ctx* ctx, int32_t k);

/*
 * domdec_refine -- the coarse-to-fine step of multiscale domain decomposition (App. A.2.1
 * "Multi-scale and eps-scaling", Sec. 5.3; the paper defers the step to earlier work, so the
 * reading is stated here).  Moves the context to the next finer layer (grid side 2N, same s):
 *   coupling: a fine basic cell i' is one of the 2 x 2 children of a coarse basic cell i and a
 *     fine pixel y' one of the 2 x 2 children of a coarse pixel P(y'); the coarse mass is
 *     split among the X children in proportion to their mu mass and among the Y children in
 *     proportion to the fine nu:
 *         nu_i'(y') = (m_i' / m_i) nu_i(P(y')) nu_fine(y') / nu(P(y')),
 *     which keeps both marginal constraints exactly;
 *   potentials: the stitched global alpha of the coarse layer (the A cells' potentials offset
 *     as for the dual of domdec_evaluate), interpolated bilinearly at the fine pixel centres
 *     and extrapolated linearly beyond the outermost coarse centres, becomes the X potential
 *     of every composite cell of both fine partitions: their next iteration with
 *     DD_INIT_PREV starts from it.
 * Needs an iteration of both partitions on the current layer.  The context handle stays
 * valid; the coarse layer's state (and any saved copy, flow-update basis) is released.
 * Errors: DD_ESTATE (already on the finest layer, or a partition not iterated on this
 * layer), DD_ENOMEM, DD_EDEVICE.
 */
dd_status domdec_refine(dd_ctx* ctx);

/* Flow update statistics. */
typedef struct {
    int32_t n_nodes, n_arcs;
    double int_value;          /* optimal value of the integer min-cost flow (exact < 2^53) */
    double value;              /* sum_ij w_ij cbar_ij in float64 (<= 0)               */
    double moved_mass;         /* sum_{i != j} w_ij                                   */
    int32_t n_active_arcs;     /* arcs i != j with w_ij > 0                           */
    int32_t reserved;
    double t_costs_ms, t_mcf_ms, t_assemble_ms;
} dd_flow_stats;

enum { DD_CAND_PRODUCT = 0, DD_CAND_GLUED = 1 };  /* edge candidates of the flow update */

/*
 * flow_update -- flow update with gluing edge candidates (Sec. 3.2 Def. "Flow
 * update", Def. "Gluing edge candidate", Remark "eps-gamma"; implementation steps
 * of Sec. 5.1).  Must follow a B iteration: pi_i is the restriction to X_i x Y of
 * that iteration's composite plans.
 *   candidate   DD_CAND_PRODUCT: pihat_ij = mu_j/m_j (x) nu_i/m_i (the eps_gamma = inf
 *               limit; eps_gamma ignored);
 *               DD_CAND_GLUED: pihat_ij(x', y) = (1/m_i) sum_{x in X_i} (gamma_ij)_x(x')
 *               pi_i(x, y), gamma_ij the entropic optimal plan between mu_i/m_i and mu_j/m_j
 *               for |x - x'|^2 at regularisation eps_gamma (> 0, finite; s <= 8), computed on
 *               the device once per eps_gamma, and (gamma_ij)_x its normalised row at x.
 *   Edge costs cbar_ij = <c, pihat_ij> - <c, pi_i>/m_i over the 4-neighbourhood plus
 *   self loops (cbar_ii = 0; arcs listed per tail i = r*(N/s)+c in ascending head
 *   order), computed on the device in float64 from cell (product) or per-pixel (glued)
 *   moments of the plans; min-cost flow (MinCostFlow) on the host by network simplex,
 *   integerised with masses b_i (largest remainder to a total of 2^40, ties by
 *   index) and costs round(cbar 2^30 / max|cbar|), mapped back as
 *   w_ij = flow_ij m_i / b_i; new marginals nu_hat_j = sum_i w_ij nu_i / m_i
 *   (eq. flow-update-cell-marginals) assembled on the device, then truncated.
 *   Equivalent to flow_costs + dd_mcf_solve + flow_apply.  stats (host) may be
 *   NULL.  Synchronises the context stream.
 * Errors: DD_ESTATE if the last iteration was not on partition B; DD_EINVAL for a bad
 * candidate or eps_gamma.
 */
dd_status flow_update(dd_ctx* ctx, int32_t candidate, double eps_gamma, dd_flow_stats* stats);

/* flow_costs -- step 1 of flow_update: writes the edge costs cbar (host, float64,
 * [n_arcs], may be NULL) and the arc count (may be NULL) for the given candidates.
 * DD_ESTATE unless the last iteration was on partition B; DD_EINVAL for a bad candidate
 * or eps_gamma. */
dd_status flow_costs(dd_ctx* ctx, int32_t candidate, double eps_gamma, double* cbar,
                     int32_t* n_arcs);

/* flow_apply -- step 3 of flow_update for a given flow w (host, float64, [n_arcs], in
 * the arc order of flow_costs; w must satisfy the divergence constraint
 * eq. div-constraint-single-cell): nu_i <- sum_{i in N(j)} w_ij nu_i / m_i, truncated. */
dd_status flow_apply(dd_ctx* ctx, const double* w);

/*
 * dd_mcf_solve -- the integer min-cost flow of the flow update (host only, no GPU):
 * bipartite transportation problem, left node i supplies supply[i], right node j
 * demands supply[j], arcs tail[a] -> head[a] (0 <= tail, head < n) with integer cost
 * and no upper bound.  Network simplex with strongly feasible trees.  Writes optimal
 * flows (host int64 [m]) and, if potential is not NULL, node potentials (host int64
 * [2n], left then right) with cost + p[tail] - p[n + head] >= 0, = 0 where flow > 0.
 * Errors: DD_EINVAL (bad input), DD_ENUMERIC (infeasible or pivot limit).
 */
dd_status dd_mcf_solve(int32_t n, int32_t m, const int32_t* tail, const int32_t* head,
                       const int64_t* cost, const int64_t* supply, int64_t* flow,
                       int64_t* potential);

/* Host view of the basic-cell Y-marginals (two-call protocol). */
typedef struct {
    int64_t n_cells;     /* out: |I|                                                   */
    int64_t n_entries;   /* out: total stored entries                                  */
    int32_t* offsets;    /* (host) [|I|][2] Y-box origin (k1, k2), or NULL             */
    int32_t* dims;       /* (host) [|I|][2] Y-box dims (w1, w2), or NULL               */
    int64_t* base;       /* (host) [|I|+1] offsets into data, or NULL                  */
    double* data;        /* (host) [n_entries] row-major box entries, or NULL          */
} dd_plan_view;

/*
 * extract_plan -- copy the coupling out as basic-cell Y-marginals (Sec. 2.3
 * eq. basic-cell-Y-marginal) in bounding-box form (App. A.1).  First call with
 * all pointers NULL to read n_cells and n_entries, then with caller buffers of
 * those sizes.  Synchronises the context stream.
 */
dd_status extract_plan(dd_ctx* ctx, dd_plan_view* view);

/* Host view of one partition's composite-cell potentials (two-call protocol). */
typedef struct {
    int32_t partition;   /* in: DD_PART_A | DD_PART_B                                   */
    int32_t n_cells;     /* out: composite cells of the partition                         */
    int32_t xside;       /* out: X block side 2s                                          */
    int32_t has_beta;    /* out: 1 if this partition's iteration is the context's last one
                            (no flow update or restore since), so beta is available       */
    double eps;          /* out: eps of the partition's last iteration                    */
    int64_t n_y;         /* out: composite Y-box entries of that iteration (0 without beta) */
    int32_t* xorig;      /* (host) [n_cells][2] X block origin pixel (k1, k2); B boundary
                            cells start at -s (their block is padded), or NULL            */
    double* alpha;       /* (host) [n_cells][xside^2] alpha, row-major over the block, or
                            NULL; entries on padding pixels (outside the grid) are
                            meaningless                                                   */
    int32_t* yorig;      /* (host) [n_cells][2] composite Y-box origin, or NULL           */
    int32_t* ydims;      /* (host) [n_cells][2] composite Y-box dims (W1, W2), or NULL    */
    int64_t* ybase;      /* (host) [n_cells+1] offsets into beta, or NULL                 */
    double* beta;        /* (host) [n_y] beta, row-major per box; NaN where nu_J or nu is
                            zero, or NULL                                                 */
} dd_potentials_view;

/*
 * extract_potentials -- the dual potentials (alpha_J, beta_J) of the composite cells of one
 * partition (the optional potentials of the output plan; Sec. 2.3 Alg. "DomDecIter" cell
 * problem, Sec. 2.2 Prop. "Optimal entropic transport couplings"), in energy units with the
 * paper's reference measure mu_J (x) nu:
 *     pi_J(x, y) = exp((alpha_J(x) + beta_J(y) - |x - y|^2) / eps) mu(x) nu(y).
 * alpha is the X potential the partition's last iteration ended with (the warm start of its
 * next visit); beta that iteration's last Y-update, on the composite boxes of that iteration.
 * Both are fixed up to (alpha + t, beta - t) per cell.  First call with all pointers NULL to
 * read the sizes, then with caller buffers.  Synchronises the context stream.
 * Errors: DD_EINVAL (partition), DD_ESTATE (partition never iterated; or Y data asked for
 * while has_beta is 0), DD_EDEVICE.
 */
dd_status extract_potentials(dd_ctx* ctx, dd_potentials_view* view);

/* Quality measures (App. A.2.2 "Solution quality"). */
typedef struct {
    double y_marginal_l1;   /* sum_y |sum_i nu_i(y) - nu(y)| of the stored state      */
    double x_marginal_l1;   /* X-marginal L1 error of the last composite plans        */
    double primal;          /* E(pi) of the last composite plans                       */
    double transport;       /* <c, pi> of the last composite plans                     */
    double basic_mass_err;  /* max_i |sum_y nu_i - m_i|                                */
    double total_mass;      /* sum of all stored nu_i entries                          */
    double dual;            /* D of the stitched global dual point (NaN until both
                               partitions have been iterated)                          */
    double pd_gap;          /* primal - dual                                           */
} dd_eval;

/*
 * domdec_evaluate -- float64 reductions of the current state (App. A.2.2):
 * marginal errors and the primal objective E(pi) = <c,pi> + eps KL(pi|mu (x) nu)
 * of the composite plans pi_J of the last iteration, evaluated from their
 * potentials in float64.  Synchronises the context stream.
 */
dd_status domdec_evaluate(dd_ctx* ctx, dd_eval* out);

void domdec_free(dd_ctx* ctx);

/* Message of the last error on ctx (or of the last context-free call when ctx is
 * NULL); never NULL. */
const char* domdec_strerror(const dd_ctx* ctx, dd_status status);

/* Save a copy of the mutable state inside the context -- the basic-cell Y-marginals
 * and, for both partitions, the X potentials, their gauge offsets and visit flags --
 * replacing any earlier copy; domdec_restore brings it back (for replaying iterations
 * from one state, or checkpointing).  After a restore, flow_update / domdec_evaluate
 * need a new domdec_iterate.  Errors: DD_ENOMEM, DD_EDEVICE, DD_ESTATE (restore with
 * nothing saved). */
dd_status domdec_save(dd_ctx* ctx);
dd_status domdec_restore(dd_ctx* ctx);

/* ------------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method: an initialisation of the
 * cell problem's alpha, the input the paper's GPU Sinkhorn already takes, App. A.1).
 *
 * A 5-layer convolutional net (3x3 kernels, 32 channels, BF16 weights, FP32
 * accumulation) maps a 32x32 window of a cell, centred on the X block in the
 * box-local coordinates of the cell problem, to a correction dg of the Y potential
 * on the window.  Its base is the previous-iterate start f0 (the zero start on the
 * first visit of a partition):
 *   g0(w) = -LSE_i [f0(i) + log mu(i) - |o + i - w|^2 / kappa],  o = (32 - 2s)/2,
 * made mean-free under the weights nu_J / m_J.  The starting X potential is one
 * exact X-update, over the whole box, of the corrected potential g = g0 + dg (dg made
 * mean-free the same way, on the window part of the box; g0 elsewhere),
 *   f(i) = -LSE_j [g(j) + log nu_J(j) - C(i, j)],
 * so dg = 0 gives exactly one Sinkhorn iteration from f0.  The stopping rule is untouched:
 * the net changes only where Sinkhorn starts.  X blocks of side 2s <= 8 only.
 * Window features (8 channels): nu_J feature max(log(nu_J/m_J) + 16, 0)/4 and its
 * support, the same for mu on the X block, the two window coordinates, g0/8 on the
 * support of nu_J, and f1 - f0 on the X block where mu > 0 (f1: the X-update of g0
 * over the window).
 * ------------------------------------------------------------------------------ */
typedef struct dd_net dd_net;

/* Number of float parameters: per layer the weights [cout][cin][3][3], then bias [cout]. */
int64_t dd_net_param_count(void);

/* Create a net from host FP32 parameters (copied; the kernels use their BF16 rounding).
 * Errors: DD_EINVAL (null, non-finite), DD_ENOMEM, DD_EDEVICE. */
dd_status dd_net_create(const float* params, dd_net** out);

/* Copy the FP32 master parameters to host memory (dd_net_param_count() floats). */
dd_status dd_net_params(dd_net* net, float* params_out);

/* Inference on n samples: x (device) [n][8][32][32] float32 -> y (device) [n][32][32]. */
dd_status dd_net_forward(dd_net* net, int32_t n, const float* x, float* y, void* stream);

/* The same inference in one kernel with every layer on the matrix cores (MFMA, BF16 inputs,
 * FP32 sums): each layer's input is rounded to BF16 first; bias and ReLU are applied in FP32.
 * This is the forward pass of the DD_INIT_NET start of domdec_iterate.  Needs no memory beyond
 * x and y.  Errors: DD_EINVAL (null net, n < 0, null x or y with n > 0), DD_EDEVICE. */
dd_status dd_net_infer(dd_net* net, int32_t n, const float* x, float* y, void* stream);

/* One Adam step (lr; betas 0.9, 0.999) on the gauge-invariant weighted squared error
 *   loss_b = sum_w weight (y - target - c)^2,  c = sum_w weight (y - target) / sum_w weight,
 * averaged over the n samples (device arrays, layouts as dd_net_forward; target and
 * weight [n][32][32]).  *loss (host, may be null) receives the batch mean before the step. */
dd_status dd_net_train_step(dd_net* net, int32_t n, const float* x, const float* target,
                            const float* weight, float lr, void* stream, double* loss);

void dd_net_free(dd_net* net);
const char* dd_net_strerror(const dd_net* net);

/* Attach a net (borrowed; NULL detaches) for opts.init = DD_INIT_NET. */
dd_status domdec_set_net(dd_ctx* ctx, dd_net* net);

/* Training samples from the last domdec_iterate: for each composite cell of that
 * partition, its window features x [n][8][32][32] (from that iteration's zero or
 * previous-iterate start), the target correction -- the solved Y potential minus g0,
 * both made mean-free under the weights -- (target [n][32][32]) and the weights
 * nu_J/m_J (weight [n][32][32]); device float32 buffers of the caller.  Two-call:
 * with all three buffers NULL only *n is set.  Errors: DD_ESTATE (no iteration
 * since init or flow_apply), DD_EINVAL (cap < n, X blocks of side > 8). */
dd_status domdec_net_samples(dd_ctx* ctx, float* x, float* target, float* weight,
                             int32_t cap, int32_t* n);

#ifdef __cplusplus
}
#endif

#endif /* DOMDEC_H */
