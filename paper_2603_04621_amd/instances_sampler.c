/* Combinatorial helper of the seeded instance generator (instances.py).
 *
 * Draws, for every source, a set of distinct destination ranks: successive
 * inverse-CDF draws from a caller-supplied stream of uniforms, a draw equal
 * to an earlier rank of the same source being discarded.  This is the
 * without-replacement law of the rank distribution.  Holds no solver
 * arithmetic.
 */
#include <stdint.h>

/* rank = number of cdf entries <= x, clipped to J-1 (numpy searchsorted 'right').
 * guide[g] (g = 0..G-1) is the first index whose cdf exceeds g/G (Chen and
 * Asau's guide table), so the scan starts at most a few entries short. */
static int64_t inv_cdf(const double* cdf, int64_t J, const int32_t* guide, int64_t G, double x)
{
    int64_t g = (int64_t)(x * (double)G);
    if (g >= G) g = G - 1;
    int64_t r = guide[g];
    while (r < J && cdf[r] <= x) ++r;
    return r < J ? r : J - 1;
}

/* deg[I] (each <= J), cdf[J] nondecreasing with cdf[J-1] = 1, u[nu] uniforms in [0,1).
 * Writes out_rank[sum deg] source by source; mark[5J] is scratch.
 * A source that has not completed after 64*d+1024 draws takes its missing
 * ranks from the most probable unused ones (never hit by the shipped recipes).
 * Returns the number of uniforms consumed, or -1 if the stream ran out, or -2
 * on bad arguments. */
int64_t dl_gen_distinct(int64_t I, const int64_t* deg, int64_t J, const double* cdf,
                        const double* u, int64_t nu, int32_t* out_rank, int32_t* mark,
                        int64_t* n_fallback)
{
    if (I < 0 || J <= 0 || I >= (int64_t)1 << 31) return -2;
    for (int64_t j = 0; j < J; ++j) mark[j] = -1;
    /* guide table over G = 4J buckets, kept in the upper part of mark[] */
    int64_t G = 4 * J;
    int32_t* guide = mark + J;
    {
        int64_t r = 0;
        for (int64_t g = 0; g < G; ++g) {
            double lo = (double)g / (double)G;
            while (r < J && cdf[r] <= lo) ++r;
            guide[g] = (int32_t)(r < J ? r : J - 1);
        }
    }
    int64_t k = 0, e = 0, fb = 0;
    for (int64_t i = 0; i < I; ++i) {
        int64_t d = deg[i];
        if (d < 0 || d > J) return -2;
        int64_t got = 0, tries = 0, cap = 64 * d + 1024;
        while (got < d) {
            if (tries >= cap) {
                for (int64_t r = 0; r < J && got < d; ++r)
                    if (mark[r] != (int32_t)i) { mark[r] = (int32_t)i; out_rank[e + got++] = (int32_t)r; }
                ++fb;
                break;
            }
            if (k >= nu) return -1;
            int64_t r = inv_cdf(cdf, J, guide, G, u[k++]);
            ++tries;
            if (mark[r] == (int32_t)i) continue;
            mark[r] = (int32_t)i;
            out_rank[e + got++] = (int32_t)r;
        }
        e += d;
    }
    if (n_fallback) *n_fallback = fb;
    return k;
}

/* Stable counting order: out[k] lists the positions q (0..n-1) with key[q] = 0
 * first, then key 1, ..., each group in increasing q.  count[nkeys + 1] is
 * scratch.  Returns 0, or -2 on a key outside [0, nkeys). */
int64_t dl_counting_order(int64_t n, const int64_t* key, int64_t nkeys, int64_t* count, int64_t* out)
{
    for (int64_t k = 0; k <= nkeys; ++k) count[k] = 0;
    for (int64_t q = 0; q < n; ++q) {
        if (key[q] < 0 || key[q] >= nkeys) return -2;
        ++count[key[q] + 1];
    }
    for (int64_t k = 0; k < nkeys; ++k) count[k + 1] += count[k];
    for (int64_t q = 0; q < n; ++q) out[count[key[q]]++] = q;
    return 0;
}
