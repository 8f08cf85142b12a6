/*
 * FP64 CPU oracle for the ridge-regularized dual of linear programs with
 * block-separable simple constraints (DuaLip-GPU report, arXiv 2603.04621).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It is plain,
 * single-threaded and slow on purpose: every sum runs in index order,
 * it is built with -ffp-contract=off, and it shares no code with the GPU
 * library.
 *
 * What it computes, in the paper's notation:
 *   LP, Eq.(1):             min c'x  s.t.  A x <= b,  x in C
 *   ridge dual, Eq.(2):     g(lam) = min_{x in C} c'x + gamma/2 |D_v x|^2 + lam'(A x - b)
 *                           (primal scaling, Section 5 "Primal scaling", view (i):
 *                            the regularizer weighted by v_e^2; v = 1 by default)
 *   Danskin (Section 3.1):  grad g(lam) = A x*(lam) - b,
 *                           x*(lam) = Pi_C(-(A'lam + c)/gamma)  blockwise
 *   simple sets (Section 3.2, Eq.(4),(5)):  per block the simplex
 *                           {x >= 0, sum x <= 1}, a box {0 <= x <= u}, or the
 *                           capped simplex {0 <= x <= u, sum x <= 1} (the
 *                           reading of the "box-cut" set of Section 3.2)
 *   Jacobi row normalization (Section 5): D = diag(1/|A_r*|), A' = D A, b' = D b
 *   gamma continuation (Section 5 "Regularization decay"): gamma decays on a
 *                           schedule and the step cap scales with gamma
 *   accelerated ascent (Appendix B "Optimization algorithm"): Nesterov momentum
 *                           with a running Lipschitz estimate and a capped step.
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *   - primal-feasible restoration for the duality gap: x~_e = s_e x_e with
 *     s_e = min over the rows j touching column e of min(1, b_j/(A x)_j);
 *     P = c'x~ + gamma/2 |D_v x~|^2;  rel_gap = (P - g)/max(1, |g|).
 *   - the accelerated method: FISTA-style momentum (Beck and Teboulle 2009)
 *     on the projected step lam+ = max(0, y + eta G), eta = min(eta_max,
 *     1/L^) with the secant estimate L^ = |G - G_prev| / |y - y_prev|, the
 *     momentum point projected to lam >= 0, momentum restarted at each
 *     gamma stage.
 *   - row norms are taken of A D_v^{-1} (after primal scaling).
 *   - zero rows keep D_j = 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SIMPLEX 0
#define ORC_BOX 1
#define ORC_CAPPED 2

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 3
#define ORC_ENUMERIC 5

/* A in compressed sparse column form plus the rest of the LP.  colptr may be
 * NULL, meaning column e holds exactly the entry at position e. */
typedef struct {
    int64_t m, n;
    const int64_t* colptr;     /* [n+1] or NULL                               */
    const int32_t* rowidx;     /* [nnz]                                       */
    const double* val;         /* [nnz]                                       */
    const double* c;           /* [n]                                         */
    const double* b;           /* [m]                                         */
    int64_t nblocks;
    const int64_t* block_off;  /* [nblocks+1], contiguous cover of [0, n)     */
    const uint8_t* block_proj; /* [nblocks], ORC_SIMPLEX, ORC_BOX or ORC_CAPPED */
    const double* upper;       /* [n] box bounds, NULL = 1.0                  */
    const double* v;           /* [n] primal scale, NULL = 1.0                */
} orc_lp;

static int64_t col_lo(const orc_lp* lp, int64_t e) { return lp->colptr ? lp->colptr[e] : e; }
static int64_t col_hi(const orc_lp* lp, int64_t e) { return lp->colptr ? lp->colptr[e + 1] : e + 1; }
static double vv(const orc_lp* lp, int64_t e) { return lp->v ? lp->v[e] : 1.0; }
static double uu(const orc_lp* lp, int64_t e) { return lp->upper ? lp->upper[e] : 1.0; }

/* ------------------------------------------------------------------------- */
/* Projection of one block onto its simple set, weighted by w_e = 1/(gamma v_e^2):
 *   x = argmin_{x in C_B} sum_e (1/(2 w_e)) x_e^2 - t_e x_e
 * Box: separable, x_e = clamp(w_e t_e, 0, u_e).
 * Simplex {x >= 0, sum x <= 1}: KKT gives x_e = max(0, w_e (t_e - tau)) with
 * tau >= 0 and tau (sum x - 1) = 0.  If sum_e max(0, w_e t_e) <= 1 then tau = 0.
 * Otherwise sort t descending; with the top-k set active the multiplier is
 * tau_k = (sum_{r<=k} w_(r) t_(r) - 1) / sum_{r<=k} w_(r), and the active set
 * is the top rho with rho = max{k : t_(k) > tau_k}  (Held, Wolfe and Crowder
 * 1974; Duchi et al. 2008, extended to diagonal weights). */

typedef struct { double t, w; } tw_pair;

/* Capped simplex {0 <= x <= u, sum x <= 1}: the reading of the paper's
 * "box-cut" simple constraint (Section 3.2, "Simple constraints"; Table 1
 * names it among the projection maps): a box cut by the block's unit
 * capacity.  KKT gives x_e = clamp(w_e (t_e - tau), 0, u_e) with tau >= 0 and
 * tau (sum x - 1) = 0.  phi(tau) = sum_e clamp(w_e (t_e - tau), 0, u_e) is
 * continuous, non-increasing and affine between the breakpoints t_e (where x_e
 * reaches 0) and t_e - u_e / w_e (where it leaves u_e).  If phi(0) <= 1 then
 * tau = 0.  Otherwise phi(0) > 1 > 0 = phi(max t): the breakpoints above 0
 * are sorted, a bisection over them finds consecutive b_k < b_{k+1} with
 * phi(b_k) >= 1 > phi(b_{k+1}), and tau is the root of the affine piece
 * between them (breakpoint search, Helgason, Kennington and Lall 1980). */
static double phi_capped(int64_t d, const double* t, const double* w, const double* u, double tau)
{
    double s = 0.0;
    for (int64_t e = 0; e < d; ++e) {
        double z = w[e] * (t[e] - tau);
        double ue = u ? u[e] : 1.0;
        s += z < 0.0 ? 0.0 : (z > ue ? ue : z);
    }
    return s;
}

static int cmp_dbl_asc(const void* pa, const void* pb)
{
    double a = *(const double*)pa, b = *(const double*)pb;
    return (a > b) - (a < b);
}

static int project_capped(int64_t d, const double* t, const double* w, const double* u,
                          double* x, double* tau_out)
{
    double tau = 0.0;
    if (phi_capped(d, t, w, u, 0.0) > 1.0) {
        double* bp = (double*)malloc(sizeof(double) * (size_t)(2 * d + 1));
        if (!bp) return ORC_ENOMEM;
        int64_t nb = 0;
        bp[nb++] = 0.0;
        for (int64_t e = 0; e < d; ++e) {
            double ue = u ? u[e] : 1.0;
            double lo = t[e] - ue / w[e];
            if (t[e] > 0.0) bp[nb++] = t[e];
            if (lo > 0.0) bp[nb++] = lo;
        }
        qsort(bp, (size_t)nb, sizeof(double), cmp_dbl_asc);
        int64_t lo = 0, hi = nb - 1;     /* phi(bp[lo]) >= 1 > phi(bp[hi]) */
        while (hi - lo > 1) {
            int64_t mid = lo + (hi - lo) / 2;
            if (phi_capped(d, t, w, u, bp[mid]) >= 1.0) lo = mid;
            else hi = mid;
        }
        double a = bp[lo], b = bp[hi];
        double fa = phi_capped(d, t, w, u, a), fb = phi_capped(d, t, w, u, b);
        tau = fa > fb ? a + (fa - 1.0) * (b - a) / (fa - fb) : a;
        free(bp);
    }
    for (int64_t e = 0; e < d; ++e) {
        double z = w[e] * (t[e] - tau);
        double ue = u ? u[e] : 1.0;
        x[e] = z < 0.0 ? 0.0 : (z > ue ? ue : z);
    }
    if (tau_out) *tau_out = tau;
    return ORC_OK;
}

static int cmp_t_desc(const void* pa, const void* pb)
{
    double a = ((const tw_pair*)pa)->t, b = ((const tw_pair*)pb)->t;
    return (a < b) - (a > b);
}

int orc_project_block(int proj, int64_t d, const double* t, const double* w,
                      const double* u, double* x, double* tau_out)
{
    if (d < 0) return ORC_EINVAL;
    if (proj == ORC_BOX) {
        for (int64_t e = 0; e < d; ++e) {
            double z = w[e] * t[e];
            double ue = u ? u[e] : 1.0;
            x[e] = z < 0.0 ? 0.0 : (z > ue ? ue : z);
        }
        if (tau_out) *tau_out = 0.0;
        return ORC_OK;
    }
    if (proj == ORC_CAPPED) return project_capped(d, t, w, u, x, tau_out);
    if (proj != ORC_SIMPLEX) return ORC_EINVAL;
    double s = 0.0;
    for (int64_t e = 0; e < d; ++e) {
        double z = w[e] * t[e];
        if (z > 0.0) s += z;
    }
    double tau = 0.0;
    if (s > 1.0) {
        tw_pair* p = (tw_pair*)malloc(sizeof(tw_pair) * (size_t)d);
        if (!p) return ORC_ENOMEM;
        for (int64_t e = 0; e < d; ++e) { p[e].t = t[e]; p[e].w = w[e]; }
        qsort(p, (size_t)d, sizeof(tw_pair), cmp_t_desc);
        double sw = 0.0, swt = 0.0;
        for (int64_t k = 0; k < d; ++k) {
            sw += p[k].w;
            swt += p[k].w * p[k].t;
            double tk = (swt - 1.0) / sw;
            if (p[k].t > tk) tau = tk;
        }
        free(p);
    }
    for (int64_t e = 0; e < d; ++e) {
        double z = w[e] * (t[e] - tau);
        x[e] = z > 0.0 ? z : 0.0;
    }
    if (tau_out) *tau_out = tau;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Everything the dual evaluation at one lam reports (original units). */
typedef struct {
    double g;          /* dual objective, Eq.(2)                               */
    double cx;         /* c'x                                                  */
    double reg;        /* gamma/2 |D_v x|^2                                    */
    double P;          /* primal objective at the feasible restoration x~     */
    double rel_gap;    /* (P - g)/max(1, |g|)                                  */
    double max_infeas; /* max_j (A x - b)_j^+                                  */
} orc_eval;

/* x*(lam), grad g(lam) = A x* - b and the scalars above. */
int orc_dual_eval(const orc_lp* lp, const double* lam, double gamma,
                  double* x_out /*[n] or NULL*/, double* grad /*[m]*/, orc_eval* out)
{
    if (!lp || !lam || !grad || !(gamma > 0.0)) return ORC_EINVAL;
    const int64_t m = lp->m, n = lp->n;
    double* t = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* w = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* u = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* x = x_out ? x_out : (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* Ax = (double*)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    if (!t || !w || !u || !x || !Ax) {
        free(t); free(w); free(u); if (!x_out) free(x); free(Ax);
        return ORC_ENOMEM;
    }
    /* t = -(A'lam + c), w = 1/(gamma v^2) */
    for (int64_t e = 0; e < n; ++e) {
        double q = lp->c[e];
        for (int64_t k = col_lo(lp, e); k < col_hi(lp, e); ++k) q += lp->val[k] * lam[lp->rowidx[k]];
        t[e] = -q;
        double ve = vv(lp, e);
        w[e] = 1.0 / (gamma * ve * ve);
        u[e] = uu(lp, e);
    }
    /* blockwise projection */
    for (int64_t i = 0; i < lp->nblocks; ++i) {
        int64_t lo = lp->block_off[i], hi = lp->block_off[i + 1];
        int rc = orc_project_block(lp->block_proj[i], hi - lo, t + lo, w + lo, u + lo, x + lo, NULL);
        if (rc) { free(t); free(w); free(u); if (!x_out) free(x); free(Ax); return rc; }
    }
    /* A x, gradient */
    for (int64_t e = 0; e < n; ++e)
        for (int64_t k = col_lo(lp, e); k < col_hi(lp, e); ++k) Ax[lp->rowidx[k]] += lp->val[k] * x[e];
    double lg = 0.0, mi = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        grad[j] = Ax[j] - lp->b[j];
        lg += lam[j] * grad[j];
        if (grad[j] > mi) mi = grad[j];
    }
    double cx = 0.0, reg = 0.0;
    for (int64_t e = 0; e < n; ++e) {
        double ve = vv(lp, e);
        cx += lp->c[e] * x[e];
        reg += ve * ve * x[e] * x[e];
    }
    reg *= 0.5 * gamma;
    /* feasible restoration: scale every variable by its rows' worst ratio */
    double P = 0.0;
    {
        double pc = 0.0, pr = 0.0;
        for (int64_t e = 0; e < n; ++e) {
            double s = 1.0;
            for (int64_t k = col_lo(lp, e); k < col_hi(lp, e); ++k) {
                int32_t j = lp->rowidx[k];
                if (Ax[j] > lp->b[j]) {
                    double sj = lp->b[j] / Ax[j];
                    if (sj < s) s = sj;
                }
            }
            double xt = s * x[e];
            double ve = vv(lp, e);
            pc += lp->c[e] * xt;
            pr += ve * ve * xt * xt;
        }
        P = pc + 0.5 * gamma * pr;
    }
    if (out) {
        out->cx = cx;
        out->reg = reg;
        out->g = cx + reg + lg;
        out->P = P;
        double ag = fabs(out->g);
        out->rel_gap = (P - out->g) / (ag > 1.0 ? ag : 1.0);
        out->max_infeas = mi;
    }
    free(t); free(w); free(u); if (!x_out) free(x); free(Ax);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Setup: primal scale and Jacobi row normalization (Section 5). */

/* v_e = |A_{:,e}|_2 ("column norms of A"), 1 for an empty column. */
int orc_colnorm_scale(const orc_lp* lp, double* v_out)
{
    for (int64_t e = 0; e < lp->n; ++e) {
        double s = 0.0;
        for (int64_t k = col_lo(lp, e); k < col_hi(lp, e); ++k) s += lp->val[k] * lp->val[k];
        v_out[e] = s > 0.0 ? sqrt(s) : 1.0;
    }
    return ORC_OK;
}

/* D_j = 1/|(A D_v^{-1})_j*|_2, 1 for a zero row. */
int orc_row_scale(const orc_lp* lp, double* D_out)
{
    for (int64_t j = 0; j < lp->m; ++j) D_out[j] = 0.0;
    for (int64_t e = 0; e < lp->n; ++e) {
        double ve = vv(lp, e);
        for (int64_t k = col_lo(lp, e); k < col_hi(lp, e); ++k) {
            double z = lp->val[k] / ve;
            D_out[lp->rowidx[k]] += z * z;
        }
    }
    for (int64_t j = 0; j < lp->m; ++j) D_out[j] = D_out[j] > 0.0 ? 1.0 / sqrt(D_out[j]) : 1.0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Accelerated dual ascent with gamma continuation. */

typedef struct {
    double gamma0, gamma_final;
    int32_t n_stages;          /* gamma_s = gamma0 (gamma_final/gamma0)^(s/(n_stages-1)) */
    int32_t row_normalize;     /* 1: iterate in lam' = D^{-1} lam on A' = D A        */
    int64_t stage_iters;       /* advance after this many iterations (0 = never)     */
    double stage_tol;          /* or when rel_gap <= stage_tol at a check (0 = never)*/
    double tol_rel_gap;        /* stop in the last stage when rel_gap <= tol         */
    int64_t max_iters;
    int64_t check_every;       /* gap evaluated every k iterations and at the last  */
                               /* one (0 = never)                                   */
    double max_step, init_step;/* step cap and first step at gamma0 (lam' units)     */
    int32_t momentum;          /* 1 accelerated, 0 plain projected gradient          */
    int32_t adaptive;          /* 1 secant Lipschitz estimate, 0 fixed step max_step */
} orc_solve_opts;

typedef struct {
    int64_t iters;             /* gradient evaluations done                         */
    int32_t converged, stage;
    double gamma, g, P, rel_gap, max_infeas;
} orc_solve_result;

/* trace rows (if trace != NULL), one per iteration k, ORC_TRACE_W doubles:
 *   g(y_k), rel_gap(y_k) (NaN off-check), eta used for the step, gamma, stage,
 *   |G'|_2 */
#define ORC_TRACE_W 6

int orc_solve(const orc_lp* lp_in, const orc_solve_opts* o, double* lam_inout,
              orc_solve_result* res, double* trace)
{
    if (!lp_in || !o || !lam_inout || !res) return ORC_EINVAL;
    if (!(o->gamma0 > 0.0) || o->n_stages < 1 || o->max_iters < 0) return ORC_EINVAL;
    const int64_t m = lp_in->m, n = lp_in->n;
    int64_t nnz = lp_in->colptr ? lp_in->colptr[n] : n;
    size_t M = (size_t)(m > 0 ? m : 1);

    /* row-scaled copy A' = D A, b' = D b (Section 5, Jacobi preconditioning) */
    double* D = (double*)malloc(sizeof(double) * M);
    double* val2 = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double* b2 = (double*)malloc(sizeof(double) * M);
    double* lam = (double*)malloc(sizeof(double) * M);
    double* y = (double*)malloc(sizeof(double) * M);
    double* yp = (double*)malloc(sizeof(double) * M);
    double* G = (double*)malloc(sizeof(double) * M);
    double* Gp = (double*)malloc(sizeof(double) * M);
    double* ln = (double*)malloc(sizeof(double) * M);
    if (!D || !val2 || !b2 || !lam || !y || !yp || !G || !Gp || !ln) {
        free(D); free(val2); free(b2); free(lam); free(y); free(yp); free(G); free(Gp); free(ln);
        return ORC_ENOMEM;
    }
    if (o->row_normalize) orc_row_scale(lp_in, D);
    else for (int64_t j = 0; j < m; ++j) D[j] = 1.0;
    orc_lp lp = *lp_in;
    for (int64_t e = 0; e < n; ++e)
        for (int64_t k = col_lo(lp_in, e); k < col_hi(lp_in, e); ++k)
            val2[k] = D[lp_in->rowidx[k]] * lp_in->val[k];
    for (int64_t j = 0; j < m; ++j) b2[j] = D[j] * lp_in->b[j];
    lp.val = val2;
    lp.b = b2;

    /* lam' = D^{-1} lam, projected to lam' >= 0 */
    for (int64_t j = 0; j < m; ++j) {
        double z = lam_inout[j] / D[j];
        lam[j] = z > 0.0 ? z : 0.0;
        y[j] = lam[j];
    }
    double gamma = o->gamma0;
    int32_t stage = 0;
    double eta_cap = o->max_step;
    double eta = o->init_step;
    double tm = 1.0;
    int64_t ks = 0;
    orc_eval ev;
    memset(&ev, 0, sizeof ev);
    memset(res, 0, sizeof *res);
    res->rel_gap = NAN;
    int rc = ORC_OK;
    int64_t k = 0;
    for (; k < o->max_iters; ++k) {
        int check = o->check_every > 0 &&
                    ((k + 1) % o->check_every == 0 || k + 1 == o->max_iters);
        rc = orc_dual_eval(&lp, y, gamma, NULL, G, &ev);
        if (rc) break;
        if (!isfinite(ev.g)) { rc = ORC_ENUMERIC; break; }
        /* step size from the secant Lipschitz estimate, capped */
        if (o->adaptive) {
            if (ks > 0) {
                double dy = 0.0, dg = 0.0;
                for (int64_t j = 0; j < m; ++j) {
                    double a1 = y[j] - yp[j], a2 = G[j] - Gp[j];
                    dy += a1 * a1;
                    dg += a2 * a2;
                }
                if (dy > 0.0) {
                    double Lh = sqrt(dg) / sqrt(dy);
                    eta = (Lh > 0.0 && 1.0 / Lh < eta_cap) ? 1.0 / Lh : eta_cap;
                }
            }
        } else {
            eta = eta_cap;
        }
        double gn = 0.0;
        for (int64_t j = 0; j < m; ++j) gn += G[j] * G[j];
        if (trace) {
            double* r = trace + (size_t)k * ORC_TRACE_W;
            r[0] = ev.g;
            r[1] = check ? ev.rel_gap : NAN;
            r[2] = eta;
            r[3] = gamma;
            r[4] = (double)stage;
            r[5] = sqrt(gn);
        }
        res->g = ev.g;
        res->max_infeas = ev.max_infeas;
        res->gamma = gamma;
        res->stage = stage;
        if (check) { res->P = ev.P; res->rel_gap = ev.rel_gap; }
        int last = stage == o->n_stages - 1;
        if (check && last && ev.rel_gap <= o->tol_rel_gap) { res->converged = 1; ++k; break; }
        /* projected ascent step and momentum */
        double tn = o->momentum ? 0.5 * (1.0 + sqrt(1.0 + 4.0 * tm * tm)) : 1.0;
        double beta = o->momentum ? (tm - 1.0) / tn : 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double z = y[j] + eta * G[j];
            ln[j] = z > 0.0 ? z : 0.0;
        }
        int advance = 0;
        if (!last) {
            if (o->stage_iters > 0 && ks + 1 >= o->stage_iters) advance = 1;
            if (check && o->stage_tol > 0.0 && ev.rel_gap <= o->stage_tol) advance = 1;
        }
        for (int64_t j = 0; j < m; ++j) {
            yp[j] = y[j];
            Gp[j] = G[j];
        }
        if (advance) {
            double gnew = o->gamma0 * pow(o->gamma_final / o->gamma0,
                                          (double)(stage + 1) / (double)(o->n_stages - 1));
            eta = eta * gnew / gamma;
            eta_cap = o->max_step * gnew / o->gamma0;
            gamma = gnew;
            ++stage;
            for (int64_t j = 0; j < m; ++j) { lam[j] = ln[j]; y[j] = ln[j]; }
            tm = 1.0;
            ks = 0;
        } else {
            for (int64_t j = 0; j < m; ++j) {
                double z = ln[j] + beta * (ln[j] - lam[j]);
                y[j] = z > 0.0 ? z : 0.0;
                lam[j] = ln[j];
            }
            tm = tn;
            ++ks;
        }
    }
    /* the reported point is the last one evaluated, y_k (its g and gap are known) */
    if (rc == ORC_OK) {
        for (int64_t j = 0; j < m; ++j) lam_inout[j] = D[j] * (res->converged || k == 0 ? y[j] : yp[j]);
    }
    res->iters = k;
    if (k == 0) { res->gamma = gamma; res->stage = stage; }
    free(D); free(val2); free(b2); free(lam); free(y); free(yp); free(G); free(Gp); free(ln);
    return rc;
}
