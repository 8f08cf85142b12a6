/*
 * dualip.h -- C ABI of the MI355X dual-ascent library for matching LPs.
 *
 * The library evaluates and maximizes the ridge-regularized dual of
 *
 *     min c'x   s.t.   A x <= b,   x in C                    (Eq.(1))
 *
 *     g(lam) = min_{x in C} c'x + gamma/2 |D_v x|^2 + lam'(A x - b)   (Eq.(2))
 *
 * over lam >= 0 (Section 3.1), for the matching structure of Section 3.2:
 * a column (one per edge) holds one nonzero per matching family, A = [D_1
 * ... D_I] with diagonal D_i for one family and the stacked families of
 * Definition 1 for several, plus dense rows such as the global count
 * constraint sum x <= cap of Section 4 (at most four entries per column in
 * all), and the columns are grouped into contiguous blocks, one per source,
 * each carrying one simple constraint:
 * the simplex {x >= 0, sum x <= 1} (Eq.(4),(5)), a box {0 <= x <= u} or
 * both at once (dl_proj).
 * By Danskin's theorem grad g(lam) = A x*(lam) - b with
 * x*(lam) = Pi_C(-(A'lam + c)/gamma) blockwise (Section 3.1).
 *
 * Conventions for every entry point:
 *   - Return codes only; no exception crosses the ABI.  On failure
 *     dl_last_error() (thread-local) holds a message.  Argument validation
 *     happens before any device work.
 *   - "host" pointers are read during the call only; the library copies what
 *     it keeps.  "device" pointers are caller-owned HIP allocations on the
 *     device current when the problem was created; they must stay valid until
 *     the stream has passed the work the call enqueued.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it in order; calls that report host values wait for
 *     it.  Concurrent calls on one dl_problem from several threads are not
 *     allowed.
 *   - lam, grad and g are always in the caller's units of (A, b).  Jacobi row
 *     normalization (Section 5) is internal: the solver iterates in
 *     lam' = D^{-1} lam on A' = D A, b' = D b and converts back.
 *   - Destinations (rows) and variables (columns) keep the caller's indexing
 *     at the ABI; any internal reordering is undone on output.
 */
#ifndef DUALIP_H
#define DUALIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DL_OK = 0,
    DL_ERR_INVALID_ARG = 1,    /* malformed input; nothing was done              */
    DL_ERR_UNSUPPORTED = 2,    /* valid input outside what this library solves  */
    DL_ERR_OUT_OF_MEMORY = 3,  /* device or host allocation failed               */
    DL_ERR_DEVICE = 4,         /* a HIP call failed                              */
    DL_ERR_NUMERIC = 5,        /* a non-finite value appeared in the iteration   */
    DL_ERR_NOT_CONVERGED = 6,  /* iteration budget spent before the gap target   */
    DL_ERR_BUSY = 7,           /* server admission: no slot or HBM budget now    */
    DL_ERR_NOT_FOUND = 8       /* unknown server ticket                          */
} dl_status;

/* Simple constraint of a block (Section 3.2, "Simple constraints"):
 *   DL_PROJ_SIMPLEX  {x >= 0, sum x <= 1}                    (Eq.(4),(5))
 *   DL_PROJ_BOX      {0 <= x <= u}
 *   DL_PROJ_CAPPED   {0 <= x <= u, sum x <= 1}: the box cut by the block's
 *                    unit capacity, this library's reading of the paper's
 *                    "box-cut" set (a capacity k other than 1 is the same
 *                    set after scaling the block's columns by k).          */
typedef enum { DL_PROJ_SIMPLEX = 0, DL_PROJ_BOX = 1, DL_PROJ_CAPPED = 2 } dl_proj;
typedef enum { DL_CSC = 0, DL_CSR = 1 } dl_layout;
/* Storage of the per-nonzero values a and c on the device.  Arithmetic is
 * FP64 in every case; the choice only sets the bytes streamed per iteration. */
typedef enum { DL_F64 = 0, DL_F32 = 1, DL_BF16_AC = 2 } dl_storage;

typedef struct dl_problem dl_problem;
typedef struct dl_server dl_server;

/* LP data (all host pointers, read-only, copied by dl_problem_create).
 *   m       rows of A (destinations), n columns (variables), nnz entries.
 *   layout  DL_CSC: ptr[n+1] column pointers (NULL means ptr[e] = e, i.e.
 *           exactly one entry per column), idx[nnz] row indices.
 *           DL_CSR: ptr[m+1] row pointers, idx[nnz] column indices.
 *   val[nnz] entries of A; c[n] costs; b[m] capacities.
 *   block_off[num_blocks+1] tiles [0, n) contiguously (block_off[0] = 0,
 *           non-decreasing, block_off[num_blocks] = n); block_proj[num_blocks]
 *           holds dl_proj values; upper[n] bounds u (NULL = 1.0; ignored on
 *           simplex blocks).
 * Requirements: indices in range, values finite, at most four entries per
 * column (more: DL_ERR_UNSUPPORTED), upper >= 0, m >= 1.  Columns with
 * several entries (several families, dense rows) run a kernel variant of
 * their own; dl_batch_solve, the server and deterministic mode take one
 * entry per column (DL_ERR_UNSUPPORTED otherwise).
 * dl_solve additionally needs a >= 0 and b >= 0 (the duality-gap restoration
 * relies on them); other signs still allow dl_dual_grad. */
typedef struct {
    int64_t m, n, nnz;
    dl_layout layout;
    const int64_t* ptr;
    const int32_t* idx;
    const double* val;
    const double* c;
    const double* b;
    int64_t num_blocks;
    const int64_t* block_off;
    const uint8_t* block_proj;
    const double* upper;
} dl_problem_desc;

/* Create-time options.
 *   storage        see dl_storage.
 *   row_normalize  1 (default): Jacobi row normalization, D_j = 1/|(A D_v^{-1})_j*|
 *                  (Section 5, "Jacobi preconditioning"; zero rows keep 1).
 *   primal_scale   0: v = 1; 1: v_e = |A_{:,e}|_2 (the column-norm choice of
 *                  Section 5, "Primal scaling"); 2: v given in `v`.
 *   v              [n] host array of positive scales when primal_scale = 2.
 *   autotune       0 (default): the work layout follows the kernel variant's
 *                  register budget (largest one-lane blocks, rows per lane,
 *                  workgroup blocks only beyond 64-lane segments, one
 *                  workgroup per compute unit).  1: before building the
 *                  problem, build a sample of it (every k-th block, about 16M
 *                  nonzeros, all destinations, capacities scaled by the
 *                  sampled fraction), run 200 iterations of the solver on it
 *                  at gamma = 1e-3 (natural steps) for representative prices,
 *                  then time the gradient kernel at those prices while
 *                  changing one layout parameter at a time (largest one-lane
 *                  block, rows per lane, smallest workgroup block,
 *                  workgroups per compute unit), keeping a change only when
 *                  it is at least 1% faster; costs about a dozen sample
 *                  builds at create.  dl_problem_info reports the pick.
 *   deterministic  0 (default): the per-destination sums of A x (and of the
 *                  gap terms) are f32 partials added by LDS atomics in
 *                  whatever order the waves reach them, so two evaluations
 *                  agree to rounding (about 1e-7 relative per row), not bit
 *                  for bit.  1: every term is rounded to a 64-bit fixed-point
 *                  integer (one power-of-two scale per sum, chosen at create
 *                  from a bound on the largest row sum, so that no row can
 *                  overflow 2^60) and added with integer atomics, which are
 *                  order-independent: dl_dual_grad and dl_solve return the same
 *                  bits on every run.  Costs integer conversions per term,
 *                  and LDS (16 bytes per row kept in LDS in every pass, where
 *                  otherwise problems with more rows than fit at 16 bytes
 *                  keep 12).
 *   lane_cap, seg_rmax, wg_min, chunks_per_cu
 *                  the work layout by hand (0 = the default of each; the
 *                  starting point of autotune when it is on): largest degree
 *                  of a block on one lane, largest rows per lane of a block
 *                  on 4, 16 or 64 lanes, smallest degree of a block on a
 *                  whole workgroup (beyond the one-lane ones), workgroups of
 *                  the gradient kernel per compute unit.  The first two are
 *                  clamped to the kernel variant's register budget; a wg_min
 *                  above 64 seg_rmax changes nothing.  Values below 0, or
 *                  chunks_per_cu above 8, are DL_ERR_INVALID_ARG.  Only the
 *                  speed changes: results agree to rounding with the default.
 * The regularizer is gamma/2 sum_e v_e^2 x_e^2 (view (i) of primal scaling). */
typedef struct {
    dl_storage storage;
    int32_t row_normalize;
    int32_t primal_scale;
    const double* v;
    int32_t autotune;
    int32_t deterministic;
    int32_t lane_cap, seg_rmax, wg_min, chunks_per_cu;
} dl_problem_opts;

/* Fills opts with the defaults (DL_F32, row_normalize = 1, primal_scale = 0,
 * autotune = 0, deterministic = 0, layout fields 0). */
void dl_problem_opts_init(dl_problem_opts* opts);

/* Host-only validation of desc/opts with the rules above; no device is
 * touched.  DL_OK, DL_ERR_INVALID_ARG or DL_ERR_UNSUPPORTED. */
dl_status dl_problem_validate(const dl_problem_desc* desc, const dl_problem_opts* opts);

/* Validates, builds the device layout (blocks grouped by projection type and
 * degree, destinations relabelled by degree) and uploads it on hip_stream.
 * Blocks until the upload is complete.  *out receives a handle to release
 * with dl_problem_destroy.  Errors: those of dl_problem_validate,
 * DL_ERR_OUT_OF_MEMORY, DL_ERR_DEVICE. */
dl_status dl_problem_create(const dl_problem_desc* desc, const dl_problem_opts* opts,
                            void* hip_stream, dl_problem** out);

/* Frees every device and host resource of p (waits for its work).  NULL is a no-op. */
dl_status dl_problem_destroy(dl_problem* p);

/* Scalars reported with a dual evaluation (original units):
 *   g           dual objective of Eq.(2) at lam
 *   cx, reg     c'x*(lam) and gamma/2 |D_v x*|^2
 *   P           primal objective at the restored point x~_e = s_j(e) x*_e,
 *               s_j = min(1, b_j/(A x*)_j): feasible, so P >= optimum >= g
 *   rel_gap     (P - g)/max(1, |g|)
 *   max_infeas  max_j (A x* - b)_j^+                                        */
typedef struct {
    double g, cx, reg, P, rel_gap, max_infeas;
} dl_eval;

/* One dual-gradient evaluation (Section 3.1, Danskin):
 *   lambda_dev [m] device, FP64, any finite values (lam >= 0 for a valid bound)
 *   gamma      > 0
 *   grad_dev   [m] device, FP64, receives A x*(lam) - b
 *   x_dev      [n] device, FP64, receives x*(lam) in column order, or NULL
 *   eval_host  receives the scalars above, or NULL; when given the call waits
 *              for the stream.
 * Errors: DL_ERR_INVALID_ARG (NULL/invalid arguments), DL_ERR_DEVICE. */
dl_status dl_dual_grad(dl_problem* p, const double* lambda_dev, double gamma, double* grad_dev,
                       double* x_dev, dl_eval* eval_host, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops or harnesses that forbid hipMalloc): the same
 * evaluation as dl_dual_grad, with the same arguments, results and errors,
 * but every intermediate buffer (permuted lambda, chunk partial sums, FP64
 * accumulators of rows beyond LDS, objective and block partials, scalars) is
 * taken from one static device array of DL_NOALLOC_SCRATCH_BYTES per device,
 * held by the library until the process ends.  The call allocates nothing
 * and makes no hipMalloc/hipFree.  It must be made with the problem's device
 * current (else DL_ERR_INVALID_ARG).  A problem whose evaluation needs more
 * scratch than the array holds (roughly 4 B x chunks x LDS rows per partial
 * plane, 3 planes when eval_host is given, plus 32 B per row) fails with
 * DL_ERR_UNSUPPORTED before any device work.  All calls on one device share
 * the array: calls whose stream work overlaps on one device (other streams,
 * other threads) race and give wrong results; serialize them. */
#define DL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dl_status dl_dual_grad_noalloc(dl_problem* p, const double* lambda_dev, double gamma,
                               double* grad_dev, double* x_dev, dl_eval* eval_host,
                               void* hip_stream);

/* Accelerated dual ascent with gamma continuation (Section 5; Appendix B).
 * Step: lam+ = max(0, y + eta G'), eta = min(eta_max, 1/L^) with the running
 * Lipschitz estimate L^ = |G' - G'_prev| / |y - y_prev| (adaptive = 1) or
 * eta = eta_max (adaptive = 0); momentum y+ = max(0, lam+ + ((t-1)/t+)(lam+ - lam)),
 * t+ = (1 + sqrt(1 + 4 t^2))/2 (momentum = 1).  Stage s uses
 * gamma_s = gamma0 (gamma_final/gamma0)^(s/(n_stages-1)); the step cap and
 * the current step scale with gamma_s/gamma0 and momentum restarts at each
 * stage change, which happens after stage_iters iterations (0 = never) or
 * when rel_gap <= stage_tol at a check (0 = never).  The gap is evaluated
 * every check_every iterations and at the last one (0 = never); the solve
 * stops in the last stage once rel_gap <= tol_rel_gap (a negative tolerance
 * never stops on the gap), or after max_iters.
 *   max_step, init_step  eta_max and the first step at gamma0, in lam' units
 *                        (after row normalization |A'|^2 = 1, so L = 1/gamma
 *                        and max_step = gamma0 is the classical 1/L).
 *   warm_start           1: lambda_dev_inout holds the start point.
 *   graph_iters          iterations captured per hipGraph launch (0 = auto).
 *   time_kernels         1: launch eagerly (no graph) with HIP events around
 *                        every fused gradient launch on hip_stream; the mean
 *                        launch times are returned in grad_kernel_ms
 *                        (ordinary iterations) and check_kernel_ms (gap-check
 *                        iterations).
 *   trace_host           NULL or [max_iters * DL_TRACE_W] FP64 rows:
 *                        g, rel_gap (NaN off-check), eta, gamma, stage, |G'|.
 *   preset               how max_step and init_step are set (dl_preset):
 *                        DL_PRESET_CUSTOM uses the two fields as given; the
 *                        other presets overwrite them per problem from
 *                        gamma0 and |A'|^2, the squared spectral norm of the
 *                        matrix the solver iterates on (after primal scaling
 *                        and, when on, row normalization; dl_problem_info
 *                        reports it), so that L = |A'|^2/gamma is the dual's
 *                        Lipschitz constant (Appendix A, Lemma 2):
 *                          DL_PRESET_PAPER    max_step = 0.1 gamma0/|A'|^2,
 *                                             init_step = 1e-3 gamma0/|A'|^2:
 *                                             at gamma0 = 0.01 and |A'| = 1
 *                                             these are Appendix B's fixed
 *                                             1e-3 and 1e-5;
 *                          DL_PRESET_NATURAL  max_step = gamma0/|A'|^2 = 1/L
 *                                             (the classical safe step),
 *                                             init_step = 1e-2 gamma0/|A'|^2. */
#define DL_TRACE_W 6
typedef enum { DL_PRESET_CUSTOM = 0, DL_PRESET_PAPER = 1, DL_PRESET_NATURAL = 2 } dl_preset;
typedef struct {
    double gamma0, gamma_final;
    int32_t n_stages, momentum;
    int64_t stage_iters;
    double stage_tol, tol_rel_gap;
    int64_t max_iters, check_every;
    double max_step, init_step;
    int32_t adaptive, warm_start;
    int32_t graph_iters, time_kernels;
    double* trace_host;
    int32_t preset;
    int32_t reserved;        /* set to 0 */
} dl_solve_opts;

/* Defaults: gamma0 = gamma_final = 0.01, one stage, momentum and adaptive on,
 * tol 1e-4 checked every 10 iterations, max_iters 10000, max_step = gamma0,
 * init_step = 1e-2 gamma0 (the paper's 1e-3 / 1e-5 ratio of Appendix B),
 * preset DL_PRESET_CUSTOM. */
void dl_solve_opts_init(dl_solve_opts* opts);

/* Host only: resolves opts->preset for a problem whose iteration matrix has
 * squared norm anorm2 (> 0, finite): writes max_step and init_step as listed
 * under `preset` above; DL_PRESET_CUSTOM leaves them.  dl_solve,
 * dl_batch_solve and the server call it with each problem's own |A'|^2.
 * DL_ERR_INVALID_ARG for an unknown preset or anorm2 <= 0. */
dl_status dl_solve_opts_apply_preset(dl_solve_opts* opts, double anorm2);

typedef struct {
    dl_status status;
    int32_t converged, stage;
    int64_t iters;           /* gradient evaluations performed                  */
    double gamma, g, P, rel_gap, max_infeas;   /* at the returned point        */
    double seconds;          /* wall time of the call                           */
    double grad_kernel_ms;   /* mean fused-gradient launch time of ordinary
                                iterations (time_kernels)                       */
    int64_t grad_launches;   /* launches that time covers                       */
    double check_kernel_ms;  /* the same for gap-check iterations               */
    int64_t check_launches;
} dl_solve_result;

/* Runs the solve on hip_stream and waits for it.
 *   lambda_dev_inout [m] device FP64: start point if warm_start, receives the
 *   last evaluated iterate (the point whose g and gap are reported).
 * Returns DL_OK when converged, DL_ERR_NOT_CONVERGED after max_iters (result
 * and lambda still filled), DL_ERR_NUMERIC on a non-finite objective,
 * DL_ERR_UNSUPPORTED when the problem has a < 0 or b < 0. */
dl_status dl_solve(dl_problem* p, const dl_solve_opts* opts, double* lambda_dev_inout,
                   dl_solve_result* out, void* hip_stream);

/* Batched solve of count independent problems (all created on this device)
 * with one fused gradient launch per iteration covering every unfinished
 * problem; each problem keeps its own iteration state and stops on its own
 * test, with the same arithmetic as dl_solve.  lambdas_dev[k] as in dl_solve;
 * out[count].  Returns DL_OK if all converged, else the first failing status. */
dl_status dl_batch_solve(dl_problem* const* probs, int32_t count, const dl_solve_opts* opts,
                         double* const* lambdas_dev, dl_solve_result* out, void* hip_stream);

/* Serving: a background scheduler that admits LP solve requests while others
 * run (continuous batching).  A request is admitted when a slot is free and
 * its device footprint fits in hbm_budget_bytes; admitted requests advance
 * together, one fused iteration at a time, each with its own state, and leave
 * as they finish.  dl_server_submit copies the request (host data) and
 * returns a ticket at once; dl_server_poll reports completion and, once done,
 * the result and lambda (host [m], caller units).  A request larger than the
 * whole budget fails with DL_ERR_UNSUPPORTED at submit. */
dl_status dl_server_create(size_t hbm_budget_bytes, int32_t max_slots, dl_server** out);
dl_status dl_server_submit(dl_server* s, const dl_problem_desc* desc, const dl_problem_opts* popts,
                           const dl_solve_opts* sopts, uint64_t* ticket);
/* *done = 1 when finished (then out/lambda_host are filled if non-NULL and the
 * ticket is released), 0 while queued or running.  DL_ERR_NOT_FOUND for an
 * unknown or already collected ticket. */
dl_status dl_server_poll(dl_server* s, uint64_t ticket, int32_t* done, dl_solve_result* out,
                         double* lambda_host);
/* Times in seconds since server creation: submit, admission (start) and
 * completion of a finished, not yet collected ticket. */
dl_status dl_server_times(dl_server* s, uint64_t ticket, double* t_submit, double* t_start,
                          double* t_done);
/* Stops admissions and drops queued requests, lets running ones finish,
 * frees all of the server's device memory and joins its threads.
 * Uncollected results are discarded. */
dl_status dl_server_destroy(dl_server* s);

/* Layout and size figures of a created problem. */
typedef struct {
    int64_t m, n, num_blocks;
    int64_t lane_groups, seg_groups, wg_blocks;   /* work items: one-lane-per-block
                                                   groups, multi-lane groups,
                                                   one-workgroup blocks          */
    int64_t chunks, lds_rows;                      /* workgroups, rows kept in LDS  */
    int64_t stream_bytes;      /* per-nonzero bytes streamed by one gradient pass */
    int64_t device_bytes;      /* device memory held by the problem              */
    int32_t storage, has_box;
    int32_t lane_cap;          /* largest degree of one-lane blocks               */
    int32_t seg_rmax;          /* largest rows per lane of multi-lane blocks      */
    int32_t chunks_per_cu;     /* workgroups of the gradient kernel per CU        */
    int32_t tuned;             /* 1 when the layout was picked by autotune        */
    double anorm2;             /* |A'|^2 of the iteration matrix (see preset): 1
                                  with row normalization and one family, else
                                  max_j |(A D_v^{-1})_j*|^2 (rows are orthogonal);
                                  with several entries per column the largest
                                  eigenvalue of A'A'^T by power iteration,
                                  raised by 1e-3                                 */
    int32_t deterministic;     /* 1 when created with deterministic = 1          */
    int32_t has_capped;        /* 1 when some block is DL_PROJ_CAPPED            */
    int32_t col_entries;       /* most entries in one column (1: one family)     */
    int32_t wg_min;            /* blocks of at least this many edges (beyond the
                                  one-lane ones) run on a whole workgroup; 0:
                                  only blocks longer than 64 seg_rmax do        */
} dl_problem_info;
dl_status dl_problem_get_info(const dl_problem* p, dl_problem_info* info);

/* Timing aid: enqueues `iters` gradient-kernel launches at lambda_dev on
 * hip_stream bracketed by HIP events on that stream, waits, and reports the
 * mean duration of one launch of the fused gradient kernel in milliseconds. */
dl_status dl_time_grad_kernel(dl_problem* p, const double* lambda_dev, double gamma, int32_t iters,
                              int32_t check, double* ms_per_launch, void* hip_stream);

const char* dl_status_str(dl_status s);
const char* dl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DUALIP_H */
