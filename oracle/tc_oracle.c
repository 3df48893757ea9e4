/*
 * TEST INFRASTRUCTURE -- the CPU oracle for exact triangle counting.
 *
 * Only the test-suite, the smoke check and the bench's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library: it has its own
 * canonicalisation, ordering, orientation, sorting and counting, written as
 * plainly as possible so that a reader can check each step against the paper
 * (Arifuzzaman, Khan, Marathe, "Parallel Algorithms for Counting Triangles in
 * Networks with Large Degrees").  All counts are int64.
 *
 * Steps and where they come from:
 *   - graph model, neighbour sets, T and T_v ........ Section II, basic definitions
 *   - degree order (ties by node id) ................. Section III-A
 *   - orientation N_v, effective degree ............... Section III-A; Fig. 1 (first loop)
 *   - per-row ascending sort .......................... Fig. 1 (second loop)
 *   - node iterator with sorted-list intersection ...... Fig. 1 (last loop)
 *   - cost functions f(v) .............................. Sections IV-B, IV-F, V-A
 *   - task schedule (initial half, shrinking tasks) .... Section V-B, Eq. (1) and Eq. (2)
 *   - space-efficient surrogate algorithm .............. Section IV-C, Fig. 2 and Fig. 3
 *   - task-based counting .............................. Section V-C, Fig. 10 and Fig. 11
 *     (also on several host threads, for the CPU baseline's timing only)
 *
 * Readings where the paper is silent (stated once here, used throughout):
 *   - input edges may contain loops and repeated or reversed pairs; loops are
 *     dropped and each unordered pair is kept once before degrees are taken;
 *   - T_v counts every triangle that contains v (Section II), not only those
 *     whose lowest-ordered vertex is v.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ERANGE = 2, ORC_ENOMEM = 3, ORC_EINTERNAL = 4 };

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Canonical undirected edge set: every unordered pair {u, v}, u != v, once,
 * as key (min << 32) | max, sorted ascending.  Section II models the input as
 * a simple undirected graph on ids 0..n-1. */
static int canonical_edges(int32_t n, int64_t m_in, const int32_t *src, const int32_t *dst, uint64_t **keys_out,
                           int64_t *m_out) {
    *keys_out = NULL;
    *m_out = 0;
    if (n < 0 || m_in < 0) return ORC_EINVAL;
    if (m_in > 0 && (!src || !dst)) return ORC_EINVAL;
    for (int64_t e = 0; e < m_in; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORC_ERANGE;
    uint64_t *keys = (uint64_t *)malloc((size_t)(m_in > 0 ? m_in : 1) * sizeof(uint64_t));
    if (!keys) return ORC_ENOMEM;
    int64_t k = 0;
    for (int64_t e = 0; e < m_in; ++e) {
        uint32_t u = (uint32_t)src[e], v = (uint32_t)dst[e];
        if (u == v) continue;
        uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
        keys[k++] = ((uint64_t)lo << 32) | hi;
    }
    qsort(keys, (size_t)k, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    for (int64_t i = 0; i < k; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    *keys_out = keys;
    *m_out = m;
    return ORC_OK;
}

/* u precedes v in the degree order: smaller degree, ties broken by smaller id
 * (Section III-A). */
static int precedes(const int32_t *deg, int32_t u, int32_t v) {
    return deg[u] < deg[v] || (deg[u] == deg[v] && u < v);
}

/* Oriented adjacency of Fig. 1: for each edge (u, v), v goes into N_u when
 * u precedes v, otherwise u goes into N_v; each N_v is then sorted ascending
 * by node id.  Outputs: m (distinct undirected edges), off[n+1], col[m] with
 * col capacity m_in, deg[n] = |neighbour set|.  Any output may be NULL except
 * when a later one needs it internally. */
int orc_orient(int32_t n, int64_t m_in, const int32_t *src, const int32_t *dst, int64_t *m_out, int64_t *off,
               int32_t *col, int32_t *deg) {
    uint64_t *keys;
    int64_t m;
    int rc = canonical_edges(n, m_in, src, dst, &keys, &m);
    if (rc) return rc;
    int32_t *d = deg ? deg : (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *o = off ? off : (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *c = col ? col : (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!d || !o || !c || !fill) {
        rc = ORC_ENOMEM;
        goto done;
    }
    memset(d, 0, (size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < m; ++i) {
        d[keys[i] >> 32]++;
        d[keys[i] & 0xffffffffu]++;
    }
    /* effective degrees: count of the edges stored in each N_v */
    memset(o, 0, (size_t)(n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = (int32_t)(keys[i] >> 32), b = (int32_t)(keys[i] & 0xffffffffu);
        int32_t owner = precedes(d, a, b) ? a : b;
        o[owner + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) o[v + 1] += o[v];
    for (int32_t v = 0; v < n; ++v) fill[v] = o[v];
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = (int32_t)(keys[i] >> 32), b = (int32_t)(keys[i] & 0xffffffffu);
        if (precedes(d, a, b))
            c[fill[a]++] = b;
        else
            c[fill[b]++] = a;
    }
    for (int32_t v = 0; v < n; ++v) qsort(c + o[v], (size_t)(o[v + 1] - o[v]), sizeof(int32_t), cmp_i32);
    if (m_out) *m_out = m;
done:
    free(keys);
    free(fill);
    if (!deg) free(d);
    if (!off) free(o);
    if (!col) free(c);
    return rc;
}

/* Node iterator of Fig. 1 over an oriented adjacency: for every v and every
 * u in N_v, S = N_v intersect N_u by a two-pointer merge of the two sorted
 * lists, T += |S|.  Per-node counts (Section II): the triangle {v, u, w} found
 * here is counted once, so each of v, u and w gains one.  Tv may be NULL. */
int orc_count_oriented(int32_t n, const int64_t *off, const int32_t *col, int64_t *T_out, int64_t *Tv) {
    if (n < 0 || !off || !T_out) return ORC_EINVAL;
    if (Tv) memset(Tv, 0, (size_t)n * sizeof(int64_t));
    int64_t T = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t p = off[v]; p < off[v + 1]; ++p) {
            int32_t u = col[p];
            int64_t i = off[v], iend = off[v + 1];
            int64_t j = off[u], jend = off[u + 1];
            int64_t s = 0;
            while (i < iend && j < jend) {
                if (col[i] < col[j])
                    ++i;
                else if (col[i] > col[j])
                    ++j;
                else {
                    if (Tv) Tv[col[i]] += 1;
                    ++s;
                    ++i;
                    ++j;
                }
            }
            T += s;
            if (Tv) {
                Tv[v] += s;
                Tv[u] += s;
            }
        }
    }
    if (Tv) {
        int64_t sum = 0;
        for (int32_t v = 0; v < n; ++v) sum += Tv[v];
        if (sum != 3 * T) return ORC_EINTERNAL;
    }
    *T_out = T;
    return ORC_OK;
}

/* Whole sequential method of Fig. 1 from an edge list: T and (optionally)
 * T_v for every node.  *m_out (optional) receives the distinct edge count. */
int orc_count(int32_t n, int64_t m_in, const int32_t *src, const int32_t *dst, int64_t *T_out, int64_t *Tv,
              int64_t *m_out) {
    if (n < 0 || m_in < 0 || !T_out) return ORC_EINVAL;
    int64_t *off = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *col = (int32_t *)malloc((size_t)(m_in > 0 ? m_in : 1) * sizeof(int32_t));
    if (!off || !col) {
        free(off);
        free(col);
        return ORC_ENOMEM;
    }
    int64_t m = 0;
    int rc = orc_orient(n, m_in, src, dst, &m, off, col, NULL);
    if (!rc) rc = orc_count_oriented(n, off, col, T_out, Tv);
    if (!rc && m_out) *m_out = m;
    free(off);
    free(col);
    return rc;
}

/* Clustering coefficients, the applications named in Section I, by their
 * textbook definitions over the canonical simple graph: the local coefficient
 * of v is T_v divided by the number of pairs of its neighbours, C(d_v, 2)
 * (0 when d_v < 2); the transitivity is 3T divided by the number of paths of
 * length two, sum over v of C(d_v, 2) (0 when there is none).  Each is one
 * floating-point division of two exact integers. */
int orc_clustering(int32_t n, int64_t m_in, const int32_t *src, const int32_t *dst, double *coeff, double *trans,
                   int64_t *wedges_out) {
    if (n < 0 || m_in < 0 || !trans) return ORC_EINVAL;
    int64_t *off = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *col = (int32_t *)malloc((size_t)(m_in > 0 ? m_in : 1) * sizeof(int32_t));
    int32_t *deg = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *Tv = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!off || !col || !deg || !Tv) {
        free(off);
        free(col);
        free(deg);
        free(Tv);
        return ORC_ENOMEM;
    }
    int64_t m = 0, T = 0;
    int rc = orc_orient(n, m_in, src, dst, &m, off, col, deg);
    if (!rc) rc = orc_count_oriented(n, off, col, &T, Tv);
    if (!rc) {
        int64_t W = 0;
        for (int32_t v = 0; v < n; ++v) {
            const int64_t d = deg[v];
            const int64_t pairs = d * (d - 1) / 2;
            W += pairs;
            if (coeff) coeff[v] = pairs > 0 ? (double)Tv[v] / (double)pairs : 0.0;
        }
        *trans = W > 0 ? (double)(3 * T) / (double)W : 0.0;
        if (wedges_out) *wedges_out = W;
    }
    free(off);
    free(col);
    free(deg);
    free(Tv);
    return rc;
}

/* The degree order written out as a sequence: perm[r] is the node in place r
 * when all nodes are listed from first to last under the order of Section
 * III-A (a stable sort by degree of the id-ordered list). */
typedef struct { int32_t d, v; } dv_pair;

static int cmp_dv(const void *a, const void *b) {
    const dv_pair *x = (const dv_pair *)a, *y = (const dv_pair *)b;
    if (x->d != y->d) return (x->d > y->d) - (x->d < y->d);
    return (x->v > y->v) - (x->v < y->v);
}

int orc_degree_order(int32_t n, const int32_t *deg, int32_t *perm) {
    if (n < 0 || (n > 0 && (!deg || !perm))) return ORC_EINVAL;
    dv_pair *p = (dv_pair *)malloc((size_t)(n > 0 ? n : 1) * sizeof(dv_pair));
    if (!p) return ORC_ENOMEM;
    for (int32_t v = 0; v < n; ++v) {
        p[v].d = deg[v];
        p[v].v = v;
    }
    qsort(p, (size_t)n, sizeof(dv_pair), cmp_dv);
    for (int32_t r = 0; r < n; ++r) perm[r] = p[r].v;
    free(p);
    return ORC_OK;
}

/* Cost functions over the oriented adjacency, one value per node:
 *   kind 0: f(v) = 1                                   (Section V-A)
 *   kind 1: f(v) = d_v                                 (Section V-A)
 *   kind 2: f(v) = sum over u in N_v of (dhat_v + dhat_u)        (Section IV-B, the prior system's best)
 *   kind 3: f(v) = sum over u in Nfull_v - N_v of (dhat_v + dhat_u) (Section IV-F)
 * where dhat_x = |N_x| and Nfull_v - N_v = {u : v in N_u}. */
int orc_costs(int32_t n, const int64_t *off, const int32_t *col, const int32_t *deg, int kind, int64_t *f) {
    if (n < 0 || !off || !f || kind < 0 || kind > 3 || (kind == 1 && !deg)) return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v) {
        int64_t dv = off[v + 1] - off[v];
        if (kind == 0)
            f[v] = 1;
        else if (kind == 1)
            f[v] = deg[v];
        else if (kind == 2) {
            int64_t s = 0;
            for (int64_t p = off[v]; p < off[v + 1]; ++p) s += dv + (off[col[p] + 1] - off[col[p]]);
            f[v] = s;
        } else
            f[v] = 0;
    }
    if (kind == 3) {
        /* u in Nfull_v - N_v  <=>  v in N_u: walk every stored pair (u, v). */
        for (int32_t u = 0; u < n; ++u) {
            int64_t du = off[u + 1] - off[u];
            for (int64_t p = off[u]; p < off[u + 1]; ++p) {
                int32_t v = col[p];
                f[v] += (off[v + 1] - off[v]) + du;
            }
        }
    }
    return ORC_OK;
}

/* Task schedule of Section V-B over costs f[0..n) (tasks are ranges of
 * consecutive positions).  Reading used (Eq. (1) is garbled and Eq. (2) is
 * silent on rounding):
 *   F(x) = f[0] + ... + f[x-1]; total = F(n); H = ceil(total / 2).
 *   Initial tasks (Eq. (1)): W tasks; task k ends at the first x with
 *     F(x) >= ceil((k+1) * H / W).
 *   Later tasks (Eq. (2)): with C the cost target reached so far (C = H after
 *     the initial tasks), the next target is C + max(ceil((total - C) / W),
 *     min_chunk); the task ends at the first x with F(x) >= that target; this
 *     repeats until the target reaches total, and that last task ends at n.
 *     When no later task is needed, one final task ends at n.  The remaining
 *     cost is measured from the last target, not from the node boundary it
 *     fell on (they differ by less than one position's cost); this makes
 *     every boundary an independent search.
 * Boundaries are written to bnd[0..ntasks] (bnd[0] = 0, bnd[ntasks] = n);
 * tasks may be empty when one position's cost spans several targets (the
 * atomic task of Section V-A cannot be split).  Returns ORC_EINVAL when cap
 * is too small; *ntasks receives the count either way. */
static int64_t first_reaching(const int64_t *F, int32_t n, int64_t target) {
    /* smallest x in [0, n] with F[x] >= target, or n when none */
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (F[mid] >= target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

int orc_schedule(int32_t n, const int64_t *f, int32_t W, int64_t min_chunk, int32_t *bnd, int64_t cap,
                 int64_t *ntasks) {
    if (n < 0 || W < 1 || min_chunk < 1 || !ntasks || (n > 0 && !f)) return ORC_EINVAL;
    int64_t *F = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t tcap = (int64_t)W + 64, k = 0;
    int32_t *t = (int32_t *)malloc((size_t)tcap * sizeof(int32_t));
    if (!F || !t) {
        free(F);
        free(t);
        return ORC_ENOMEM;
    }
    F[0] = 0;
    for (int32_t v = 0; v < n; ++v) F[v + 1] = F[v] + f[v];
    int64_t total = F[n];
    int64_t H = (total + 1) / 2;
    t[k++] = 0;
    for (int32_t i = 0; i < W; ++i) t[k++] = (int32_t)first_reaching(F, n, ((int64_t)(i + 1) * H + W - 1) / W);
    int64_t C = H;
    int ended = 0;
    while (C < total) {
        int64_t step = (total - C + W - 1) / W;
        if (step < min_chunk) step = min_chunk;
        C += step;
        if (k == tcap) {
            tcap *= 2;
            int32_t *g = (int32_t *)realloc(t, (size_t)tcap * sizeof(int32_t));
            if (!g) {
                free(F);
                free(t);
                return ORC_ENOMEM;
            }
            t = g;
        }
        if (C >= total) {
            t[k++] = n; /* the target that reaches the total ends the last task at n */
            ended = 1;
        } else {
            t[k++] = (int32_t)first_reaching(F, n, C);
        }
    }
    if (!ended) {
        if (k == tcap) {
            int32_t *g = (int32_t *)realloc(t, (size_t)(tcap + 1) * sizeof(int32_t));
            if (!g) {
                free(F);
                free(t);
                return ORC_ENOMEM;
            }
            t = g;
        }
        t[k++] = n; /* no later task: one final task ends at n */
    }
    *ntasks = k - 1;
    int rc = ORC_OK;
    if (bnd && cap >= k)
        memcpy(bnd, t, (size_t)k * sizeof(int32_t));
    else if (bnd)
        rc = ORC_EINVAL;
    free(F);
    free(t);
    return rc;
}

/* CountTriangles of Fig. 10 for the task of positions [lo, hi) of an
 * oriented adjacency: the node iterator restricted to those v.  Adds to
 * *T and (if non-NULL) to Tv. */
static void count_task(const int64_t *off, const int32_t *col, int32_t lo, int32_t hi, int64_t *T, int64_t *Tv) {
    for (int32_t v = lo; v < hi; ++v)
        for (int64_t p = off[v]; p < off[v + 1]; ++p) {
            int32_t u = col[p];
            int64_t i = off[v], j = off[u], s = 0;
            while (i < off[v + 1] && j < off[u + 1]) {
                if (col[i] < col[j])
                    ++i;
                else if (col[i] > col[j])
                    ++j;
                else {
                    if (Tv) Tv[col[i]]++;
                    ++s;
                    ++i;
                    ++j;
                }
            }
            *T += s;
            if (Tv) {
                Tv[v] += s;
                Tv[u] += s;
            }
        }
}

/* Fig. 11 with the workers run one after another: each task of the schedule
 * is counted by CountTriangles and the partial counts are summed (the
 * barrier-and-reduce step).  The order in which tasks are handed out does not
 * matter for the result (Section V-D). */
int orc_dynamic_count(int32_t n, const int64_t *off, const int32_t *col, const int32_t *bnd, int64_t ntasks,
                      int64_t *T_out, int64_t *Tv) {
    if (n < 0 || !off || !bnd || ntasks < 0 || !T_out) return ORC_EINVAL;
    if (Tv) memset(Tv, 0, (size_t)n * sizeof(int64_t));
    int64_t T = 0;
    for (int64_t k = 0; k < ntasks; ++k) {
        int64_t Tk = 0;
        count_task(off, col, bnd[k], bnd[k + 1], &Tk, Tv);
        T += Tk;
    }
    *T_out = T;
    return ORC_OK;
}

/* Fig. 10/11 with `threads` workers on the host's cores: the same tasks and
 * the same per-task node iterator as orc_dynamic_count, handed out in order
 * by an atomic counter (the coordinator of Fig. 11), each worker adding its
 * triangles into a private total and private per-node counts that are summed
 * at the end.  For timing the CPU baseline only; its results equal those of
 * orc_dynamic_count. */
typedef struct {
    const int64_t *off;
    const int32_t *col;
    const int32_t *bnd;
    int64_t ntasks;
    int32_t n;
    atomic_llong *next;
    int64_t T;
    int64_t *Tv;
} orc_worker;

static void *orc_worker_run(void *arg) {
    orc_worker *w = (orc_worker *)arg;
    for (;;) {
        const int64_t k = atomic_fetch_add(w->next, 1);
        if (k >= w->ntasks) break;
        int64_t Tk = 0;
        count_task(w->off, w->col, w->bnd[k], w->bnd[k + 1], &Tk, w->Tv);
        w->T += Tk;
    }
    return NULL;
}

int orc_dynamic_count_threaded(int32_t n, const int64_t *off, const int32_t *col, const int32_t *bnd,
                               int64_t ntasks, int32_t threads, int64_t *T_out, int64_t *Tv) {
    if (n < 0 || !off || !bnd || ntasks < 0 || !T_out || threads < 1 || threads > 1024) return ORC_EINVAL;
    orc_worker *ws = (orc_worker *)calloc((size_t)threads, sizeof(orc_worker));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    atomic_llong next;
    atomic_init(&next, 0);
    int rc = ws && tid ? ORC_OK : ORC_ENOMEM;
    for (int32_t i = 0; i < threads && rc == ORC_OK; ++i) {
        ws[i] = (orc_worker){off, col, bnd, ntasks, n, &next, 0, NULL};
        if (Tv) {
            ws[i].Tv = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
            if (!ws[i].Tv) rc = ORC_ENOMEM;
        }
    }
    int32_t started = 0;
    for (int32_t i = 0; i < threads && rc == ORC_OK; ++i, ++started)
        if (pthread_create(&tid[i], NULL, orc_worker_run, &ws[i]) != 0) rc = ORC_ENOMEM;
    for (int32_t i = 0; i < started; ++i) pthread_join(tid[i], NULL);
    if (rc == ORC_OK) {
        int64_t T = 0;
        if (Tv) memset(Tv, 0, (size_t)n * sizeof(int64_t));
        for (int32_t i = 0; i < threads; ++i) {
            T += ws[i].T;
            if (Tv)
                for (int32_t v = 0; v < n; ++v) Tv[v] += ws[i].Tv[v];
        }
        *T_out = T;
    }
    for (int32_t i = 0; ws && i < threads; ++i) free(ws[i].Tv);
    free(ws);
    free(tid);
    return rc;
}

/* Space-efficient algorithm of Fig. 3, with P processors simulated one after
 * another.  Processor i owns the consecutive node ids [part[i], part[i+1])
 * (Definition 1) and stores N_v of its own nodes.  For v it owns and u in
 * N_v: when u is also its own, it intersects N_v and N_u; otherwise it sends
 * N_v to the owner of u, at most once per destination (the LastProc rule of
 * Section IV-C: consecutive ranges and sorted lists make the nodes of one
 * owner contiguous in N_v).  Each receiver runs SurrogateCount (Fig. 2) on
 * the received list X: for every u in X that it owns, T += |N_u intersect X|.
 * Messages are delivered after all senders ran (the completion protocol only
 * decides when a processor may stop, not what it counts).  Per-node counts
 * add one to each vertex of every triangle found.  *messages and
 * *message_ids (optional) receive the number of lists sent and their total
 * length. */
int orc_surrogate_count(int32_t n, const int64_t *off, const int32_t *col, int32_t P, const int32_t *part,
                        int64_t *T_out, int64_t *Tv, int64_t *messages, int64_t *message_ids) {
    if (n < 0 || P < 1 || !off || !part || !T_out || part[0] != 0 || part[P] != n) return ORC_EINVAL;
    for (int32_t i = 0; i < P; ++i)
        if (part[i] > part[i + 1]) return ORC_EINVAL;
    int32_t *owner = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    /* message queue: (destination, sender node v) pairs */
    int64_t qcap = 1024, qlen = 0;
    int32_t *qdst = (int32_t *)malloc((size_t)qcap * sizeof(int32_t));
    int32_t *qv = (int32_t *)malloc((size_t)qcap * sizeof(int32_t));
    if (!owner || !qdst || !qv) {
        free(owner);
        free(qdst);
        free(qv);
        return ORC_ENOMEM;
    }
    for (int32_t i = 0; i < P; ++i)
        for (int32_t v = part[i]; v < part[i + 1]; ++v) owner[v] = i;
    if (Tv) memset(Tv, 0, (size_t)n * sizeof(int64_t));
    int64_t T = 0, nmsg = 0, nids = 0;
    /* local work and sends (Fig. 3, first loop) */
    for (int32_t i = 0; i < P; ++i) {
        for (int32_t v = part[i]; v < part[i + 1]; ++v) {
            int32_t last_proc = -1;
            for (int64_t p = off[v]; p < off[v + 1]; ++p) {
                int32_t u = col[p];
                int32_t j = owner[u];
                if (j == i) {
                    int64_t a = off[v], b = off[u];
                    while (a < off[v + 1] && b < off[u + 1]) {
                        if (col[a] < col[b])
                            ++a;
                        else if (col[a] > col[b])
                            ++b;
                        else {
                            ++T;
                            if (Tv) {
                                Tv[v]++;
                                Tv[u]++;
                                Tv[col[a]]++;
                            }
                            ++a;
                            ++b;
                        }
                    }
                } else if (j != last_proc) {
                    if (qlen == qcap) {
                        qcap *= 2;
                        int32_t *a1 = (int32_t *)realloc(qdst, (size_t)qcap * sizeof(int32_t));
                        int32_t *a2 = (int32_t *)realloc(qv, (size_t)qcap * sizeof(int32_t));
                        if (!a1 || !a2) {
                            free(a1 ? a1 : qdst);
                            free(a2 ? a2 : qv);
                            free(owner);
                            return ORC_ENOMEM;
                        }
                        qdst = a1;
                        qv = a2;
                    }
                    qdst[qlen] = j;
                    qv[qlen] = v;
                    ++qlen;
                    ++nmsg;
                    nids += off[v + 1] - off[v];
                    last_proc = j;
                }
            }
        }
    }
    /* message handling: SurrogateCount(X, j) with X = N_v (Fig. 2) */
    for (int64_t q = 0; q < qlen; ++q) {
        int32_t j = qdst[q], v = qv[q];
        const int32_t *X = col + off[v];
        int64_t xl = off[v + 1] - off[v];
        for (int64_t x = 0; x < xl; ++x) {
            int32_t u = X[x];
            if (owner[u] != j) continue;
            int64_t a = 0, b = off[u];
            while (a < xl && b < off[u + 1]) {
                if (X[a] < col[b])
                    ++a;
                else if (X[a] > col[b])
                    ++b;
                else {
                    ++T;
                    if (Tv) {
                        Tv[v]++;
                        Tv[u]++;
                        Tv[X[a]]++;
                    }
                    ++a;
                    ++b;
                }
            }
        }
    }
    free(owner);
    free(qdst);
    free(qv);
    *T_out = T;
    if (messages) *messages = nmsg;
    if (message_ids) *message_ids = nids;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Per-node counts straight from the definition of Section II, for checking
 * sampled nodes of graphs too large for the full oracle run:
 * T_v = number of edges (u, w) with both u and w neighbours of v.
 * An undirected sorted adjacency is built once, then queried per node.   */
typedef struct {
    int32_t n;
    int64_t *off;
    int32_t *adj;
} orc_adj;

void *orc_adj_build(int32_t n, int64_t m_in, const int32_t *src, const int32_t *dst) {
    uint64_t *keys;
    int64_t m;
    if (canonical_edges(n, m_in, src, dst, &keys, &m)) return NULL;
    orc_adj *g = (orc_adj *)calloc(1, sizeof(orc_adj));
    if (!g) {
        free(keys);
        return NULL;
    }
    g->n = n;
    g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->off || !g->adj || !fill) {
        free(keys);
        free(fill);
        free(g->off);
        free(g->adj);
        free(g);
        return NULL;
    }
    for (int64_t i = 0; i < m; ++i) {
        g->off[(keys[i] >> 32) + 1]++;
        g->off[(keys[i] & 0xffffffffu) + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) g->off[v + 1] += g->off[v];
    for (int32_t v = 0; v < n; ++v) fill[v] = g->off[v];
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = (int32_t)(keys[i] >> 32), b = (int32_t)(keys[i] & 0xffffffffu);
        g->adj[fill[a]++] = b;
        g->adj[fill[b]++] = a;
    }
    for (int32_t v = 0; v < n; ++v)
        qsort(g->adj + g->off[v], (size_t)(g->off[v + 1] - g->off[v]), sizeof(int32_t), cmp_i32);
    free(fill);
    free(keys);
    return g;
}

void orc_adj_free(void *h) {
    orc_adj *g = (orc_adj *)h;
    if (!g) return;
    free(g->off);
    free(g->adj);
    free(g);
}

int64_t orc_adj_edges(void *h) {
    orc_adj *g = (orc_adj *)h;
    return g ? g->off[g->n] / 2 : -1;
}

int orc_adj_degree(void *h, int64_t k, const int32_t *vs, int32_t *out) {
    orc_adj *g = (orc_adj *)h;
    if (!g || k < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < k; ++i) {
        if (vs[i] < 0 || vs[i] >= g->n) return ORC_ERANGE;
        out[i] = (int32_t)(g->off[vs[i] + 1] - g->off[vs[i]]);
    }
    return ORC_OK;
}

/* For each queried v: sum over neighbours u of |Nfull_u intersect Nfull_v|,
 * which counts every edge among the neighbours of v twice. */
int orc_adj_tv(void *h, int64_t k, const int32_t *vs, int64_t *out) {
    orc_adj *g = (orc_adj *)h;
    if (!g || k < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < k; ++i) {
        int32_t v = vs[i];
        if (v < 0 || v >= g->n) return ORC_ERANGE;
        int64_t twice = 0;
        for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) {
            int32_t u = g->adj[p];
            int64_t a = g->off[v], b = g->off[u];
            while (a < g->off[v + 1] && b < g->off[u + 1]) {
                if (g->adj[a] < g->adj[b])
                    ++a;
                else if (g->adj[a] > g->adj[b])
                    ++b;
                else {
                    ++twice;
                    ++a;
                    ++b;
                }
            }
        }
        out[i] = twice / 2;
    }
    return ORC_OK;
}
