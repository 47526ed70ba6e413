/*
 * synth.c -- seeded, counter-based generator of synthetic set collections.
 *
 * This module only draws inputs: n sets of hashed 64-bit IDs stored as CSR
 * (ids[], offsets[n+1]).  It holds none of the similarity arithmetic and is
 * shared, as an input source only, by the CPU oracle and by the GPU path.
 *
 * Workload model (stand-in for the k-mer sets of genome samples, paper
 * Sec. V-A2, whose datasets are not available): every sample i gets
 *   - a target size s_i (log-uniform or clipped log-normal),
 *   - a share f_i in [share_lo, share_hi] and a cluster c_i (uniform),
 *   - k_i = min(round(f_i * s_i), |P_{c_i}|) IDs drawn WITHOUT replacement
 *     from the cluster pool P_{c_i} (a random permutation of the pool, cut),
 *   - s_i - k_i IDs drawn uniformly from the universe [0, 2^U),
 *   - optionally round(dup_rate * s_i) repeats of its own earlier entries.
 * Pools are ranges [pool_start, pool_start + pool_size) of a global pool
 * index space; pool index g maps to the ID perm_U(g), a keyed bijection on
 * U-bit integers, so pool IDs are distinct and spread over the universe.
 *
 * Bernoulli collections (size_kind 2) follow the paper's synthetic indicator
 * matrices (Sec. V-A3): each of `rows` row indices is in each set
 * independently with probability `density`.  A set is drawn by geometric skips
 * (the gap to the next present row is 1 + floor(ln(1-u) / ln(1-p)) for
 * uniform u; Devroye, "Non-Uniform Random Variate Generation", 1986, Ch. X),
 * so its cost is its size, not `rows`; its IDs come out in increasing order
 * and its size is known only once it is drawn.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used in counter mode: the k-th value of
 * stream `key` is mix(key + (k+1) * gamma).  Every element is a pure function
 * of (seeds, sample, position), so any subset of samples can be regenerated
 * on its own and generation parallelises over elements.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm_at(uint64_t key, uint64_t k)
{
    return sm_mix(key + (k + 1) * SM_GAMMA);
}

/* stream key for (seed, tag, sample) */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t sample)
{
    return sm_mix(sm_mix(seed ^ (tag * 0xd1b54a32d192ed03ULL)) + (sample + 1) * SM_GAMMA);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

static inline uint64_t low_mask(uint32_t b) { return b >= 64 ? ~0ULL : ((1ULL << b) - 1ULL); }

/* Keyed bijection on [0, 2^b): each step (add, multiply by an odd constant
 * mod 2^b, xor with a right shift) is invertible on b-bit integers. */
static inline uint64_t perm_bits(uint64_t x, uint32_t b, uint64_t k0, uint64_t k1)
{
    const uint64_t m = low_mask(b);
    const uint32_t h = (b + 1) / 2;
    x = (x + k0) & m;
    x = (x * (k1 | 1ULL)) & m;
    x ^= x >> h;
    x = (x * SM_GAMMA) & m;
    x ^= x >> h;
    x = (x * 0xbf58476d1ce4e5b9ULL) & m;
    x ^= x >> h;
    x = (x + k1) & m;
    x = (x * 0x94d049bb133111ebULL) & m;
    x ^= x >> h;
    return x;
}

static inline uint32_t ceil_log2(uint64_t v)
{
    uint32_t b = 0;
    while (b < 64 && (1ULL << b) < v) ++b;
    return b;
}

/* Bijection on [0, size) by cycle walking a bijection on [0, 2^b), b = ceil(log2 size). */
static inline uint64_t perm_range(uint64_t x, uint64_t size, uint32_t b, uint64_t k0, uint64_t k1)
{
    if (b == 0) return 0;
    uint64_t y = perm_bits(x, b, k0, k1);
    while (y >= size) y = perm_bits(y, b, k0, k1);
    return y;
}

typedef struct {
    uint64_t pool_seed;    /* defines pool IDs (shared by a database and its queries) */
    uint64_t sample_seed;  /* defines every per-sample draw */
    uint32_t universe_bits;
    int32_t n;
    int32_t size_kind;     /* 0: log-uniform [size_a, size_b]; 1: log-normal(median size_a, sigma size_b) clipped to [size_lo, size_hi] */
    int32_t n_pools;
    double size_a, size_b, size_lo, size_hi;
    double share_lo, share_hi;
    double dup_rate;
    const uint64_t *pool_start; /* n_pools entries */
    const uint64_t *pool_size;  /* n_pools entries */
    double density;        /* size_kind 2: probability that a row is in a set */
    uint64_t rows;         /* size_kind 2: row indices 0 .. rows-1 */
} synth_spec;

enum { TAG_PARAM = 1, TAG_POOLPERM = 2, TAG_PRIVATE = 3, TAG_DUP = 4, TAG_IDPERM = 5, TAG_BERNOULLI = 6 };

enum { KIND_LOG_UNIFORM = 0, KIND_LOG_NORMAL = 1, KIND_BERNOULLI = 2 };

/* Bernoulli set of sample i: writes its rows to dst (if not NULL) in
 * increasing order and returns how many there are. */
static uint64_t bernoulli_walk(const synth_spec *sp, int32_t i, uint64_t *dst)
{
    const uint64_t m = sp->rows;
    const double p = sp->density;
    if (!(p > 0.0) || m == 0) return 0;
    if (p >= 1.0) {
        if (dst)
            for (uint64_t r = 0; r < m; ++r) dst[r] = r;
        return m;
    }
    const uint64_t key = stream_key(sp->sample_seed, TAG_BERNOULLI, (uint64_t)i);
    const double inv = 1.0 / log1p(-p); /* negative */
    uint64_t count = 0, next = 0;       /* next: first row not yet passed */
    for (uint64_t t = 0;; ++t) {
        const double skip = floor(log1p(-u01(sm_at(key, t))) * inv); /* rows left out before the next one */
        if (skip >= (double)(m - next)) break;
        const uint64_t r = next + (uint64_t)skip;
        if (dst) dst[count] = r;
        ++count;
        next = r + 1;
        if (next >= m) break;
    }
    return count;
}

typedef struct {
    uint64_t size, pool_part, dups;
    int32_t cluster;
} sample_plan;

static sample_plan plan_sample(const synth_spec *sp, int32_t i)
{
    sample_plan p;
    if (sp->size_kind == KIND_BERNOULLI) {
        p.size = bernoulli_walk(sp, i, NULL);
        p.pool_part = p.dups = 0;
        p.cluster = -1;
        return p;
    }
    const uint64_t key = stream_key(sp->sample_seed, TAG_PARAM, (uint64_t)i);
    const double u0 = u01(sm_at(key, 0)), u1 = u01(sm_at(key, 1));
    const double u2 = u01(sm_at(key, 2)), u3 = u01(sm_at(key, 3));
    double s;
    if (sp->size_kind == KIND_LOG_UNIFORM) {
        s = exp(log(sp->size_a) + u0 * (log(sp->size_b) - log(sp->size_a)));
    } else {
        /* Box-Muller normal from (u0, u1) */
        const double z = sqrt(-2.0 * log(1.0 - u0)) * cos(6.283185307179586 * u1);
        s = exp(log(sp->size_a) + sp->size_b * z);
        if (s < sp->size_lo) s = sp->size_lo;
        if (s > sp->size_hi) s = sp->size_hi;
    }
    p.size = (uint64_t)llround(s);
    const double f = sp->share_lo + u2 * (sp->share_hi - sp->share_lo);
    p.cluster = sp->n_pools > 0 ? (int32_t)(u3 * sp->n_pools) : -1;
    if (p.cluster >= sp->n_pools) p.cluster = sp->n_pools - 1;
    uint64_t k = (uint64_t)llround(f * (double)p.size);
    if (k > p.size) k = p.size;
    if (p.cluster >= 0 && k > sp->pool_size[p.cluster]) k = sp->pool_size[p.cluster];
    if (p.cluster < 0) k = 0;
    p.pool_part = k;
    p.dups = (uint64_t)llround(sp->dup_rate * (double)p.size);
    return p;
}

/* offsets[0..n]: CSR row pointers of the generated collection.  Returns 0. */
int synth_offsets(const synth_spec *sp, uint64_t *offsets)
{
    offsets[0] = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < sp->n; ++i) {
        const sample_plan p = plan_sample(sp, i);
        offsets[i + 1] = p.size + p.dups;
    }
    for (int32_t i = 0; i < sp->n; ++i) offsets[i + 1] += offsets[i];
    return 0;
}

/* Per-sample plan (size, pool part, dups, cluster) for reporting. */
int synth_plan(const synth_spec *sp, int32_t i, uint64_t *out4)
{
    const sample_plan p = plan_sample(sp, i);
    out4[0] = p.size;
    out4[1] = p.pool_part;
    out4[2] = p.dups;
    out4[3] = (uint64_t)(int64_t)p.cluster;
    return 0;
}

static void fill_one(const synth_spec *sp, int32_t i, uint64_t *dst)
{
    if (sp->size_kind == KIND_BERNOULLI) {
        bernoulli_walk(sp, i, dst);
        return;
    }
    const sample_plan p = plan_sample(sp, i);
    const uint32_t U = sp->universe_bits;
    const uint64_t mU = low_mask(U);
    const uint64_t idk0 = stream_key(sp->pool_seed, TAG_IDPERM, 0);
    const uint64_t idk1 = stream_key(sp->pool_seed, TAG_IDPERM, 1);
    if (p.pool_part) {
        const uint64_t start = sp->pool_start[p.cluster], size = sp->pool_size[p.cluster];
        const uint64_t k0 = stream_key(sp->sample_seed, TAG_POOLPERM, 2 * (uint64_t)i);
        const uint64_t k1 = stream_key(sp->sample_seed, TAG_POOLPERM, 2 * (uint64_t)i + 1);
        const uint32_t b = ceil_log2(size);
        for (uint64_t t = 0; t < p.pool_part; ++t) {
            const uint64_t g = start + perm_range(t, size, b, k0, k1);
            dst[t] = perm_bits(g, U, idk0, idk1);
        }
    }
    const uint64_t kp = stream_key(sp->sample_seed, TAG_PRIVATE, (uint64_t)i);
    for (uint64_t t = p.pool_part; t < p.size; ++t) dst[t] = sm_at(kp, t) & mU;
    if (p.dups && p.size) {
        const uint64_t kd = stream_key(sp->sample_seed, TAG_DUP, (uint64_t)i);
        for (uint64_t t = 0; t < p.dups; ++t) {
            const uint64_t src = sm_at(kd, t) % p.size;
            dst[p.size + t] = dst[src];
        }
    }
}

/* Fill samples [i0, i1) into ids; ids[0] is the first entry of sample i0. */
int synth_fill(const synth_spec *sp, int32_t i0, int32_t i1, const uint64_t *offsets, uint64_t *ids)
{
    if (i0 < 0 || i1 > sp->n || i0 > i1) return -1;
    const uint64_t base = offsets[i0];
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = i0; i < i1; ++i) fill_one(sp, i, ids + (offsets[i] - base));
    return 0;
}

/* Fill an arbitrary list of samples, packed back to back in list order
 * (dst_offsets[k] .. dst_offsets[k+1] holds sample idx[k]). */
int synth_fill_list(const synth_spec *sp, int32_t count, const int32_t *idx, const uint64_t *dst_offsets,
                    uint64_t *ids)
{
    for (int32_t k = 0; k < count; ++k)
        if (idx[k] < 0 || idx[k] >= sp->n) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < count; ++k) fill_one(sp, idx[k], ids + dst_offsets[k]);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Power-law graphs for vertex similarity (the neighbourhood Jaccard of paper
 * Sec. II-F, with the adjacency matrix as A, Sec. III-A).  R-MAT (Chakrabarti,
 * Zhan, Faloutsos, "R-MAT: A Recursive Model for Graph Mining", SDM 2004):
 * each of edge_factor * 2^scale draws picks one of the four quadrants of the
 * adjacency matrix with probabilities (a, b, c, 1 - a - b - c) at each of the
 * `scale` levels.  Vertex labels are scrambled by a keyed bijection so that
 * the heavy vertices are spread over the ID range.  The graph is undirected:
 * a draw (u, v) with u != v puts v in N(u) and u in N(v).  Output: the
 * neighbourhoods N(0) .. N(2^scale - 1) in CSR, each ascending, repeats
 * removed.  ids must hold 2 * edge_factor * 2^scale entries; returns the
 * number written, or -1 for bad arguments.
 */
static int cmp_u64(const void *x, const void *y)
{
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : a > b;
}

static void rmat_edge(uint64_t key, uint64_t e, uint32_t scale, double a, double b, double c, uint64_t *u,
                      uint64_t *v)
{
    uint64_t r = 0, s = 0;
    for (uint32_t l = 0; l < scale; ++l) {
        const double x = u01(sm_at(key, e * scale + l));
        const uint64_t bit = 1ULL << (scale - 1 - l);
        if (x < a) {
        } else if (x < a + b) {
            s |= bit;
        } else if (x < a + b + c) {
            r |= bit;
        } else {
            r |= bit;
            s |= bit;
        }
    }
    *u = r;
    *v = s;
}

int64_t synth_rmat(uint32_t scale, uint64_t edge_factor, uint64_t seed, double a, double b, double c,
                   uint64_t *offsets, uint64_t *ids)
{
    if (scale < 1 || scale > 30 || !(a >= 0 && b >= 0 && c >= 0 && a + b + c <= 1.0)) return -1;
    const uint64_t nv = 1ULL << scale, E = edge_factor * nv;
    const uint64_t key = stream_key(seed, TAG_PARAM, 0xE);
    const uint64_t k0 = stream_key(seed, TAG_IDPERM, 0xE0), k1 = stream_key(seed, TAG_IDPERM, 0xE1);
    uint64_t *cnt = (uint64_t *)calloc(nv + 1, sizeof(uint64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(static)
    for (uint64_t e = 0; e < E; ++e) {
        uint64_t u, v;
        rmat_edge(key, e, scale, a, b, c, &u, &v);
        if (u == v) continue;
        u = perm_bits(u, scale, k0, k1);
        v = perm_bits(v, scale, k0, k1);
        __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    }
    /* raw CSR (with repeats) in offsets, cursors in cnt */
    offsets[0] = 0;
    for (uint64_t i = 0; i < nv; ++i) offsets[i + 1] = offsets[i] + cnt[i];
    for (uint64_t i = 0; i < nv; ++i) cnt[i] = offsets[i];
#pragma omp parallel for schedule(static)
    for (uint64_t e = 0; e < E; ++e) {
        uint64_t u, v;
        rmat_edge(key, e, scale, a, b, c, &u, &v);
        if (u == v) continue;
        u = perm_bits(u, scale, k0, k1);
        v = perm_bits(v, scale, k0, k1);
        ids[__atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED)] = v;
        ids[__atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED)] = u;
    }
    /* sort each neighbourhood (the fill order above is not deterministic),
     * drop repeats, and close the gaps */
#pragma omp parallel for schedule(dynamic, 64)
    for (uint64_t i = 0; i < nv; ++i) {
        uint64_t *x = ids + offsets[i];
        const uint64_t len = offsets[i + 1] - offsets[i];
        qsort(x, len, sizeof(uint64_t), cmp_u64);
        uint64_t w = 0;
        for (uint64_t t = 0; t < len; ++t)
            if (w == 0 || x[t] != x[w - 1]) x[w++] = x[t];
        cnt[i] = w;
    }
    uint64_t pos = 0;
    for (uint64_t i = 0; i < nv; ++i) {
        const uint64_t src = offsets[i], len = cnt[i];
        memmove(ids + pos, ids + src, len * sizeof(uint64_t));
        offsets[i] = pos;
        pos += len;
    }
    offsets[nv] = pos;
    free(cnt);
    return (int64_t)pos;
}
