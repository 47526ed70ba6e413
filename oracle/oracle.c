/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct CPU
 * computation of exact Jaccard similarity, used to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never does.
 *
 * It follows the definitions, not the paper's algorithm: no row batches, no
 * zero-row filter, no bitmasks, no popcount.
 *
 *   X_i is a set of integers (Sec. II-A: each data sample is a set), so an
 *   input list is normalised by sorting and dropping repeats.
 *   |X_i cap X_j| and |X_i cup X_j| are counted by walking the two sorted
 *   lists together (Sec. II-A, Eq. (1)).
 *   J(X_i, X_j) = |X_i cap X_j| / |X_i cup X_j|, and J = 1 when both sets are
 *   empty (Sec. II-A).  The quotient of the two exact integer counts is taken
 *   in IEEE-754 binary64 with round-to-nearest (the paper fixes no precision
 *   for S; both counts are < 2^53, so they convert exactly and the quotient is
 *   the correctly rounded value of the rational).
 *
 * Inputs are CSR collections: ids[offsets[i] .. offsets[i+1]) are the entries
 * of sample i, in any order, repeats allowed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Sort one sample's entries and drop repeats; returns the set size. */
static uint64_t make_set(const uint64_t *src, uint64_t len, uint64_t *dst)
{
    if (len == 0) return 0;
    memcpy(dst, src, len * sizeof(uint64_t));
    qsort(dst, len, sizeof(uint64_t), cmp_u64);
    uint64_t k = 1;
    for (uint64_t t = 1; t < len; ++t)
        if (dst[t] != dst[k - 1]) dst[k++] = dst[t];
    return k;
}

/* Normalise a collection: out_ids gets each set sorted without repeats,
 * out_offsets[0..n] its CSR pointers.  out_ids needs offsets[n] entries. */
int oracle_normalize(const uint64_t *ids, const uint64_t *offsets, int32_t n, uint64_t *out_ids,
                     uint64_t *out_offsets)
{
    if (n < 0) return -1;
    for (int32_t i = 0; i < n; ++i)
        if (offsets[i + 1] < offsets[i]) return -1;
    uint64_t *size = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    if (!size) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < n; ++i)
        size[i] = make_set(ids + offsets[i], offsets[i + 1] - offsets[i], out_ids + offsets[i]);
    /* pack the sets back to back */
    uint64_t w = 0;
    out_offsets[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (w != offsets[i]) memmove(out_ids + w, out_ids + offsets[i], size[i] * sizeof(uint64_t));
        w += size[i];
        out_offsets[i + 1] = w;
    }
    free(size);
    return 0;
}

/* |X cap Y| and |X cup Y| of two sorted, repeat-free lists, counted in one
 * walk over both: each step takes the smaller of the two heads (both heads
 * when they are equal, which is then an element of the intersection), so
 * every step takes exactly one element of the union; whatever remains of
 * either list after the other is exhausted belongs to the union only. */
void oracle_counts(const uint64_t *x, uint64_t nx, const uint64_t *y, uint64_t ny, uint64_t *inter, uint64_t *uni)
{
    uint64_t a = 0, b = 0, c = 0, u = 0;
    while (a < nx && b < ny) {
        const uint64_t p = x[a], q = y[b];
        c += p == q;
        a += p <= q;
        b += q <= p;
        ++u;
    }
    *inter = c;
    *uni = u + (nx - a) + (ny - b);
}

/* J from the two counts (Sec. II-A, including J(empty, empty) = 1). */
double oracle_jaccard(uint64_t inter, uint64_t uni)
{
    if (uni == 0) return 1.0;
    return (double)inter / (double)uni;
}

/* Selected pairs between collection Q (sets q) and collection X (sets x),
 * both already normalised.  For k < npairs: inter[k] = |Q_qi[k] cap X_xi[k]|,
 * uni[k] = |Q_qi[k] cup X_xi[k]|, jac[k] = J.  Any output may be NULL. */
int oracle_pairs(const uint64_t *q, const uint64_t *qoff, int32_t nq, const uint64_t *x, const uint64_t *xoff,
                 int32_t nx, int64_t npairs, const int32_t *qi, const int32_t *xi, int64_t *inter, int64_t *uni,
                 double *jac)
{
    for (int64_t k = 0; k < npairs; ++k)
        if (qi[k] < 0 || qi[k] >= nq || xi[k] < 0 || xi[k] >= nx) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npairs; ++k) {
        const uint64_t *a = q + qoff[qi[k]], *b = x + xoff[xi[k]];
        const uint64_t na = qoff[qi[k] + 1] - qoff[qi[k]], nb = xoff[xi[k] + 1] - xoff[xi[k]];
        uint64_t c, u;
        oracle_counts(a, na, b, nb, &c, &u);
        if (inter) inter[k] = (int64_t)c;
        if (uni) uni[k] = (int64_t)u;
        if (jac) jac[k] = oracle_jaccard(c, u);
    }
    return 0;
}

/* Every pair (i, j) of Q x X, row-major [nq][nx].  Normalised inputs. */
int oracle_cross(const uint64_t *q, const uint64_t *qoff, int32_t nq, const uint64_t *x, const uint64_t *xoff,
                 int32_t nx, int64_t *inter, int64_t *uni, double *jac)
{
    if (nq < 0 || nx < 0) return -1;
    const int64_t total = (int64_t)nq * (int64_t)nx;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        const int32_t i = (int32_t)(k / nx), j = (int32_t)(k % nx);
        const uint64_t *a = q + qoff[i], *b = x + xoff[j];
        const uint64_t na = qoff[i + 1] - qoff[i], nb = xoff[j + 1] - xoff[j];
        uint64_t c, u;
        oracle_counts(a, na, b, nb, &c, &u);
        if (inter) inter[k] = (int64_t)c;
        if (uni) uni[k] = (int64_t)u;
        if (jac) jac[k] = oracle_jaccard(c, u);
    }
    return 0;
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the parallel loops above use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
