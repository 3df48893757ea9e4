/*
 * Seeded synthetic graph generators (input side only).
 *
 * These functions produce undirected edge lists as int32 (src, dst) pairs in
 * the orientation and order in which the edges were drawn.  They hold none of
 * the triangle-counting arithmetic: no canonicalisation, ordering, orientation
 * or counting happens here.  Loops and repeated pairs are left in the output
 * where the generative model draws them (R-MAT, Chung-Lu); the models that are
 * defined over distinct pairs (G(n,m), preferential attachment with distinct
 * targets) reject repeats while drawing.
 *
 * Randomness: every draw comes from Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), keyed by the
 * seed and addressed by a counter, so output never depends on thread count.
 *
 * Workload shapes follow the paper's power-law inputs: preferential
 * attachment (Section II, datasets paragraph) and R-MAT / Chung-Lu graphs
 * with skewed degrees standing in for its social and web graphs.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

typedef struct { uint32_t v[4]; } ph4;

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Ten rounds of the Philox 4x32 bijection with the published multipliers and
 * Weyl key increments. */
static ph4 philox4x32_10(ph4 ctr, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, ctr.v[0], &hi0, &lo0);
        mulhilo32(M1, ctr.v[2], &hi1, &lo1);
        ph4 n;
        n.v[0] = hi1 ^ ctr.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ ctr.v[3] ^ k1;
        n.v[3] = lo0;
        ctr = n;
        k0 += W0;
        k1 += W1;
    }
    return ctr;
}

/* Stream identifiers keep the generators' counter spaces apart. */
enum { STREAM_ER = 1, STREAM_PA = 2, STREAM_RMAT = 3, STREAM_CL = 4, STREAM_PERM = 5, STREAM_MISC = 6 };

static inline ph4 draw(uint64_t seed, uint32_t stream, uint64_t a, uint32_t b) {
    ph4 c;
    c.v[0] = (uint32_t)a;
    c.v[1] = (uint32_t)(a >> 32);
    c.v[2] = b;
    c.v[3] = stream;
    return philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
}

/* Uniform integer in [0, bound) from a 32-bit word (multiply-high). */
static inline uint64_t below32(uint32_t x, uint64_t bound) { return ((uint64_t)x * bound) >> 32; }

/* Uniform integer in [0, bound) from two 32-bit words, for bounds >= 2^32. */
static inline uint64_t below64(uint32_t hi, uint32_t lo, uint64_t bound) {
    unsigned __int128 w = ((unsigned __int128)(((uint64_t)hi << 32) | lo)) * bound;
    return (uint64_t)(w >> 64);
}

static inline double unit53(uint32_t hi, uint32_t lo) {
    uint64_t w = (((uint64_t)hi << 32) | lo) >> 11;
    return (double)w * (1.0 / 9007199254740992.0);
}

/* --------------------------------------------------------- thread helper */

typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi);

typedef struct { range_fn fn; void *ctx; int64_t lo, hi; } range_job;

static void *range_run(void *p) {
    range_job *j = (range_job *)p;
    j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

static void parallel_for(int64_t total, int nthreads, range_fn fn, void *ctx) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (total < 65536 || nthreads == 1) {
        fn(ctx, 0, total);
        return;
    }
    pthread_t th[256];
    range_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].lo = total * t / nthreads;
        jobs[t].hi = total * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, range_run, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* -------------------------------------------------- open-addressing set */

typedef struct { uint64_t *slot; uint64_t mask; } u64set;

static int set_init(u64set *s, uint64_t expect) {
    uint64_t cap = 16;
    while (cap < 2 * expect + 16) cap <<= 1;
    s->slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!s->slot) return -1;
    memset(s->slot, 0xff, cap * sizeof(uint64_t));
    s->mask = cap - 1;
    return 0;
}

static inline uint64_t mix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

/* Returns 1 when the key was new. */
static inline int set_insert(u64set *s, uint64_t key) {
    uint64_t i = mix64(key) & s->mask;
    for (;;) {
        if (s->slot[i] == key) return 0;
        if (s->slot[i] == ~0ULL) {
            s->slot[i] = key;
            return 1;
        }
        i = (i + 1) & s->mask;
    }
}

/* -------------------------------------------------------- permutations */

/* Fisher-Yates shuffle of 0..n-1 driven by the counter stream. */
int gg_random_permutation(int64_t n, uint64_t seed, int32_t *perm) {
    if (n < 0 || (n > 0 && !perm)) return -1;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        ph4 r = draw(seed, STREAM_PERM, (uint64_t)i, 0);
        int64_t j = (int64_t)below64(r.v[0], r.v[1], (uint64_t)(i + 1));
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

typedef struct { int32_t *src, *dst; const int32_t *perm; } relabel_ctx;

static void relabel_range(void *p, int64_t lo, int64_t hi) {
    relabel_ctx *c = (relabel_ctx *)p;
    for (int64_t e = lo; e < hi; ++e) {
        c->src[e] = c->perm[c->src[e]];
        c->dst[e] = c->perm[c->dst[e]];
    }
}

static int relabel(int64_t n, int64_t m, int32_t *src, int32_t *dst, uint64_t seed, int nthreads) {
    int32_t *perm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!perm) return -2;
    gg_random_permutation(n, seed ^ 0x5eed5eedULL, perm);
    relabel_ctx c = {src, dst, perm};
    parallel_for(m, nthreads, relabel_range, &c);
    free(perm);
    return 0;
}

/* ------------------------------------------------------ Erdos-Renyi G(n,m) */

/* m distinct unordered pairs {u,v}, u != v, each uniform over the C(n,2)
 * pairs, drawn sequentially and rejected when already present.  Stored as
 * drawn (u, v). */
int gg_erdos_renyi(int32_t n, int64_t m, uint64_t seed, int32_t *src, int32_t *dst) {
    if (n < 0 || m < 0) return -1;
    if (m == 0) return 0;
    if (n < 2 || (double)m > 0.5 * (double)n * (double)(n - 1)) return -1;
    u64set set;
    if (set_init(&set, (uint64_t)m)) return -2;
    int64_t have = 0;
    uint64_t attempt = 0;
    while (have < m) {
        ph4 r = draw(seed, STREAM_ER, attempt++, 0);
        int32_t u = (int32_t)below32(r.v[0], (uint64_t)n);
        int32_t v = (int32_t)below32(r.v[1], (uint64_t)n);
        if (u == v) continue;
        uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
        if (!set_insert(&set, (lo << 32) | hi)) continue;
        src[have] = u;
        dst[have] = v;
        ++have;
    }
    free(set.slot);
    return 0;
}

/* ------------------------------------------------ preferential attachment */

/* Number of edges gg_preferential_attachment emits. */
int64_t gg_pa_edge_count(int32_t n, int32_t d) {
    if (d < 1 || n <= d) return -1;
    return (int64_t)d * (d - 1) / 2 + (int64_t)(n - d) * d;
}

/* Seed graph: the complete graph on nodes 0..d-1.  Every later node t
 * attaches to d distinct earlier nodes, each picked with probability
 * proportional to its current degree: a uniform pick from the endpoint list
 * of all edges present before t arrived; repeats of a target already chosen
 * by t are redrawn.  Ids are then relabelled by a seeded permutation so that
 * id order carries no arrival-time information.  Output edge e is (t, target). */
int gg_preferential_attachment(int32_t n, int32_t d, uint64_t seed, int32_t *src, int32_t *dst, int nthreads) {
    int64_t m = gg_pa_edge_count(n, d);
    if (m < 0) return -1;
    int32_t *stub = (int32_t *)malloc((size_t)(2 * m) * sizeof(int32_t));
    int32_t *chosen = (int32_t *)malloc((size_t)d * sizeof(int32_t));
    if (!stub || !chosen) {
        free(stub);
        free(chosen);
        return -2;
    }
    int64_t e = 0;
    for (int32_t i = 0; i < d; ++i)
        for (int32_t j = i + 1; j < d; ++j) {
            src[e] = i;
            dst[e] = j;
            stub[2 * e] = i;
            stub[2 * e + 1] = j;
            ++e;
        }
    for (int32_t t = d; t < n; ++t) {
        uint64_t stubs_before = (uint64_t)(2 * e);
        uint32_t attempt = 0;
        for (int32_t j = 0; j < d; ++j) {
            int32_t cand;
            for (;;) {
                ph4 r = draw(seed, STREAM_PA, (uint64_t)t, attempt++);
                cand = stub[below64(r.v[0], r.v[1], stubs_before)];
                int dup = 0;
                for (int32_t q = 0; q < j; ++q)
                    if (chosen[q] == cand) {
                        dup = 1;
                        break;
                    }
                if (!dup) break;
            }
            chosen[j] = cand;
        }
        for (int32_t j = 0; j < d; ++j) {
            src[e] = t;
            dst[e] = chosen[j];
            stub[2 * e] = t;
            stub[2 * e + 1] = chosen[j];
            ++e;
        }
    }
    free(stub);
    free(chosen);
    return relabel(n, m, src, dst, seed, nthreads);
}

/* ----------------------------------------------------------------- R-MAT */

typedef struct {
    int scale;
    uint32_t ta, tab, tabc; /* cumulative quadrant thresholds in 2^-32 units */
    uint64_t seed;
    int32_t *src, *dst;
} rmat_ctx;

static void rmat_range(void *p, int64_t lo, int64_t hi) {
    rmat_ctx *c = (rmat_ctx *)p;
    for (int64_t e = lo; e < hi; ++e) {
        uint32_t u = 0, v = 0;
        int level = 0;
        for (uint32_t blk = 0; level < c->scale; ++blk) {
            ph4 r = draw(c->seed, STREAM_RMAT, (uint64_t)e, blk);
            for (int w = 0; w < 4 && level < c->scale; ++w, ++level) {
                uint32_t x = r.v[w];
                uint32_t row = 0, col = 0;
                if (x < c->ta) {
                } else if (x < c->tab) {
                    col = 1;
                } else if (x < c->tabc) {
                    row = 1;
                } else {
                    row = 1;
                    col = 1;
                }
                u = (u << 1) | row;
                v = (v << 1) | col;
            }
        }
        c->src[e] = (int32_t)u;
        c->dst[e] = (int32_t)v;
    }
}

/* 2^scale nodes, ef * 2^scale draws; each draw descends scale levels of the
 * recursive 2x2 partition choosing quadrant (a, b, c, 1-a-b-c).  No noise.
 * Loops and repeated pairs are kept.  Ids are relabelled by a seeded
 * permutation. */
int gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, int32_t *src,
            int32_t *dst, int nthreads) {
    if (scale < 1 || scale > 30 || edge_factor < 0 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    int64_t m = edge_factor << scale;
    rmat_ctx ctx;
    ctx.scale = scale;
    ctx.ta = (uint32_t)fmin(4294967295.0, a * 4294967296.0);
    ctx.tab = (uint32_t)fmin(4294967295.0, (a + b) * 4294967296.0);
    ctx.tabc = (uint32_t)fmin(4294967295.0, (a + b + c) * 4294967296.0);
    ctx.seed = seed;
    ctx.src = src;
    ctx.dst = dst;
    parallel_for(m, nthreads, rmat_range, &ctx);
    return relabel((int64_t)1 << scale, m, src, dst, seed, nthreads);
}

/* --------------------------------------------------------------- Chung-Lu */

typedef struct {
    const double *cdf;
    int32_t n;
    uint64_t seed;
    int32_t *src, *dst;
} cl_ctx;

static inline int32_t cdf_pick(const double *cdf, int32_t n, double x) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > x)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

static void cl_range(void *p, int64_t lo, int64_t hi) {
    cl_ctx *c = (cl_ctx *)p;
    for (int64_t e = lo; e < hi; ++e) {
        ph4 r = draw(c->seed, STREAM_CL, (uint64_t)e, 0);
        c->src[e] = cdf_pick(c->cdf, c->n, unit53(r.v[0], r.v[1]));
        c->dst[e] = cdf_pick(c->cdf, c->n, unit53(r.v[2], r.v[3]));
    }
}

/* Node i has weight (i+1)^(-1/(beta-1)); each of the m pairs draws both
 * endpoints independently with probability proportional to weight.  Loops and
 * repeated pairs are kept.  Ids are relabelled by a seeded permutation. */
int gg_chung_lu(int32_t n, int64_t m, double beta, uint64_t seed, int32_t *src, int32_t *dst, int nthreads) {
    if (n < 1 || m < 0 || beta <= 1.0) return -1;
    double *cdf = (double *)malloc((size_t)n * sizeof(double));
    if (!cdf) return -2;
    double acc = 0.0, ex = -1.0 / (beta - 1.0);
    for (int32_t i = 0; i < n; ++i) {
        acc += pow((double)(i + 1), ex);
        cdf[i] = acc;
    }
    for (int32_t i = 0; i < n; ++i) cdf[i] /= acc;
    cdf[n - 1] = 1.0;
    cl_ctx ctx = {cdf, n, seed, src, dst};
    parallel_for(m, nthreads, cl_range, &ctx);
    free(cdf);
    return relabel(n, m, src, dst, seed, nthreads);
}

/* ------------------------------------------------------- misc draws */

/* k uniform doubles in [0,1) from the counter stream, for workload recipes
 * (batch sizes, request sizes, arrival gaps) that need seeded draws. */
int gg_uniforms(uint64_t seed, uint64_t stream_tag, int64_t k, double *out) {
    if (k < 0 || (k > 0 && !out)) return -1;
    for (int64_t i = 0; i < k; ++i) {
        ph4 r = draw(seed ^ (stream_tag * 0x9E3779B97F4A7C15ULL), STREAM_MISC, (uint64_t)i, 0);
        out[i] = unit53(r.v[0], r.v[1]);
    }
    return 0;
}

/* Raw Philox4x32-10 output for counter (c0..c3) and key (k0,k1); exposed so
 * tests can check the generator against the published known-answer vectors. */
void gg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    ph4 c;
    memcpy(c.v, ctr, sizeof(c.v));
    ph4 r = philox4x32_10(c, key[0], key[1]);
    memcpy(out, r.v, sizeof(r.v));
}
