/*
 * Multi-core CPU baseline of the dual gradient of a matching LP (DuaLip-GPU
 * report, arXiv 2603.04621, Section 3.1 and Eq.(2)-(5)).
 *
 * BENCHMARK CONTEXT, NOT THE ORACLE.  The benchmark times it on all host
 * cores beside the single-threaded oracle, to state what a parallel CPU
 * implementation of the same iteration reaches on the machine that hosts the
 * GPU.  The tests check it against the oracle.  It shares no code with the GPU
 * library and the GPU library never calls it.
 *
 * One evaluation at lam, for columns with exactly one nonzero (a_e in row
 * j(e)), v = 1:
 *   t_e = -(c_e + a_e lam_j(e))
 *   x_B = Pi_C(t_B / gamma) per block B: box blocks clamp to [0, u_e];
 *         simplex blocks {x >= 0, sum x <= 1} use the threshold tau >= 0 with
 *         x_e = max(0, t_e - tau) / gamma, found by the fixed point
 *         tau <- (sum_{t > tau} t - gamma) / |{t > tau}| from
 *         tau_0 = max(0, max t - gamma) (exact once the set stops shrinking)
 *   grad_j = sum_{e -> j} a_e x_e - b_j
 *   g = c'x + gamma/2 |x|^2 + lam'grad
 * Blocks are split over OpenMP threads; each thread sums A x into its own
 * m-vector, the vectors are added at the end.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double simplex_tau(const double* t, int64_t d, double gamma)
{
    double sp = 0.0, mt = -INFINITY;
    for (int64_t k = 0; k < d; ++k) {
        if (t[k] > 0.0) sp += t[k];
        if (t[k] > mt) mt = t[k];
    }
    if (!(sp > gamma)) return 0.0;
    double tau = mt - gamma > 0.0 ? mt - gamma : 0.0;
    int64_t n = 0;
    double st = 0.0;
    for (int64_t k = 0; k < d; ++k)
        if (t[k] > tau) { st += t[k]; ++n; }
    for (int64_t rep = 0; rep < 2 * d + 4 && n > 0; ++rep) {
        const double tn = (st - gamma) / (double)n;
        double st2 = 0.0;
        int64_t n2 = 0;
        for (int64_t k = 0; k < d; ++k)
            if (t[k] > tn) { st2 += t[k]; ++n2; }
        tau = tn;
        if (n2 >= n || n2 == 0) break;
        st = st2;
        n = n2;
    }
    return tau;
}

/* returns 0, or -1 on bad arguments / -2 when memory runs out */
int cpb_dual_grad(int64_t m, int64_t nblocks, const int64_t* block_off, const uint8_t* block_proj,
                  const int32_t* dst, const double* a, const double* c, const double* upper,
                  const double* b, const double* lam, double gamma, double* grad, double* g_out,
                  int* threads_out)
{
    if (m < 0 || nblocks < 0 || !(gamma > 0.0) || !block_off || !grad || !g_out) return -1;
    int nt = omp_get_max_threads();
    if (nt < 1) nt = 1;
    double* part = (double*)calloc((size_t)nt * (size_t)(m > 0 ? m : 1), sizeof(double));
    if (!part) return -2;
    double obj = 0.0;
    int failed = 0;
#pragma omp parallel num_threads(nt) reduction(+ : obj)
    {
        const int me = omp_get_thread_num();
        double* ax = part + (size_t)me * (size_t)m;
        int64_t cap = 64;
        double* t = (double*)malloc(sizeof(double) * (size_t)cap);
        if (!t) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < nblocks; ++i) {
            if (!t) continue;
            const int64_t lo = block_off[i], d = block_off[i + 1] - lo;
            if (d > cap) {
                double* nt2 = (double*)realloc(t, sizeof(double) * (size_t)d);
                if (!nt2) {
#pragma omp atomic write
                    failed = 1;
                    continue;
                }
                t = nt2;
                cap = d;
            }
            for (int64_t k = 0; k < d; ++k) t[k] = -(c[lo + k] + a[lo + k] * lam[dst[lo + k]]);
            const int box = block_proj[i] == 1;
            const double tau = box ? 0.0 : simplex_tau(t, d, gamma);
            for (int64_t k = 0; k < d; ++k) {
                double x = (t[k] - tau) / gamma;
                if (box) {
                    const double u = upper ? upper[lo + k] : 1.0;
                    x = t[k] / gamma;
                    x = x > 0.0 ? (x < u ? x : u) : 0.0;
                } else if (!(x > 0.0)) {
                    x = 0.0;
                }
                if (x != 0.0) {
                    ax[dst[lo + k]] += a[lo + k] * x;
                    obj += c[lo + k] * x + 0.5 * gamma * x * x;
                }
            }
        }
        free(t);
    }
    if (failed) {
        free(part);
        return -2;
    }
    double lg = 0.0;
#pragma omp parallel for num_threads(nt) reduction(+ : lg) schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        double s = 0.0;
        for (int q = 0; q < nt; ++q) s += part[(size_t)q * (size_t)m + (size_t)j];
        grad[j] = s - b[j];
        lg += lam[j] * grad[j];
    }
    free(part);
    *g_out = obj + lg;
    if (threads_out) *threads_out = nt;
    return 0;
}
