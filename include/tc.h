/*
 * tc.h -- exact triangle counting over a degree-ordered oriented graph on one
 * AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * Method (Arifuzzaman, Khan, Marathe, "Parallel Algorithms for Counting
 * Triangles in Networks with Large Degrees"):
 *   - the input is an undirected graph G(V, E) on ids 0..n-1 (Section II);
 *   - nodes are ordered by degree, ties broken by id (Section III-A);
 *   - each edge is stored once, in the list N_v of its lower-ordered endpoint,
 *     and every list is sorted (Fig. 1, first two loops);
 *   - the total T is the sum over stored edges (v, u) of |N_v intersect N_u|
 *     (Fig. 1, last loop); the per-node count T_v is the number of triangles
 *     that contain v (Section II);
 *   - work is handed out as node-range tasks whose sizes follow Eq. (1) and
 *     Eq. (2) of Section V-B, pulled by persistent GPU workers from an atomic
 *     queue in place of the coordinator of Fig. 11;
 *   - graphs larger than a device-memory budget are counted in non-overlapping
 *     node-range partitions (Definition 1) whose lists N_v are streamed to the
 *     partition that needs them, once per partition (Section IV-C, Fig. 2/3).
 *
 * Conventions for every entry point:
 *   - the return value is a tc_status; outputs are written only on TC_OK;
 *   - nothing aborts, exits or throws across this interface;
 *   - work is ordered on the stream named in tc_options (NULL: the null stream);
 *   - a call whose outputs are host pointers returns once they are written;
 *     a call whose outputs are device pointers returns after enqueuing work;
 *   - tc_last_error() gives a thread-local text for the last failure.
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TC_OK = 0,
    TC_ERR_INVALID_ARG = 1,   /* NULL where data is required, negative sizes, bad option values */
    TC_ERR_ID_RANGE = 2,      /* an endpoint outside 0..n-1 (Section II labels nodes 0..n-1) */
    TC_ERR_TOO_LARGE = 3,     /* sizes beyond the int32 node-id space of one handle */
    TC_ERR_OUT_OF_MEMORY = 4, /* device allocation failed, or the budget cannot hold one partition */
    TC_ERR_DEVICE = 5         /* a HIP runtime call failed */
} tc_status;

/* One undirected input graph (Section II).  src[e], dst[e] are the endpoints
 * of edge e, int32 node ids in 0..n-1.  Loops are dropped and repeated or
 * reversed pairs are merged before degrees are taken.  Host or device memory
 * according to tc_options.inputs_on_device; read only, owned by the caller. */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t *src;
    const int32_t *dst;
} tc_edges;

/* Cost functions for the task schedule (Sections IV-B, IV-F and V-A). */
enum {
    TC_COST_ONE = 0,    /* f(v) = 1 */
    TC_COST_DEGREE = 1, /* f(v) = d_v */
    TC_COST_PRIOR = 2,  /* f(v) = sum over u in N_v of (|N_v| + |N_u|) */
    TC_COST_NEW = 3     /* f(v) = sum over u with v in N_u of (|N_v| + |N_u|) */
};

typedef struct {
    void *stream;               /* hipStream_t; NULL = null stream */
    int32_t inputs_on_device;   /* tc_edges.src/dst are device pointers */
    int32_t outputs_on_device;  /* count outputs are device pointers */
    uint64_t hbm_budget_bytes;  /* 0: no budget.  Otherwise every device allocation a
                                   build or count makes for the handle stays below it:
                                   a graph whose resident form does not fit is built
                                   and counted in node-range partitions (see below);
                                   TC_ERR_OUT_OF_MEMORY when even one partition does
                                   not fit.  Set at build time. */
    /* Device allocator; both NULL = hipMallocAsync / hipFreeAsync on the stream.
     * alloc returns NULL on failure. */
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, size_t bytes, void *stream, void *ctx);
    void *alloc_ctx;
    int32_t workers;    /* persistent waves pulling tasks; 0 = as many as fit on the device at once;
                           launches never exceed that resident capacity */
    int32_t cost_fn;    /* TC_COST_*; used when the schedule is built */
    int64_t min_chunk;  /* floor on a task's cost target (Eq. (2)); 0 = automatic */
    int32_t small_max;  /* lists up to this length are handled by one wave, longer ones by a
                           whole workgroup; 0 = automatic (128, also the maximum) */
    int32_t lds_list_max; /* longest list a workgroup stages in LDS; longer lists are probed by
                             binary search in device memory; 0 = automatic (1920, the maximum) */
    int32_t time_kernels; /* 1: record device events around the counting kernels of each count
                             call; the elapsed time is reported by tc_graph_info.  2: also record
                             when each worker starts and stops (tc_worker_times) */
    int32_t partitions;   /* build time: > 0 forces the partitioned form with at least this many
                             node-range partitions (one graph per handle); 0 = only when the
                             budget requires it */
    int32_t rounds;       /* schedule: the first half of the cost is cut into workers * rounds
                             tasks (Eq. (1) with W = workers * rounds), so the tasks in flight
                             cover 1 / (2 rounds) of the nodes at a time; 0 = automatic (1 for
                             one graph, more for large packed batches) */
    int32_t direct;       /* partitioned form, build time: 1 streams the list of v once per stored
                             edge (v, u) (the direct scheme of Section IV-C) instead of once per
                             partition (the surrogate scheme); same results, for comparison */
    int32_t static_chunks; /* schedule: 1 = W tasks of equal cost instead of the shrinking tasks of
                              Eq. (1)/(2); same results, for comparison */
    int32_t intersect;    /* how a list counted by one wave (small_max entries at most; Fig. 1:
                             S = N_v intersect N_u for each u in N_v) meets the list N_u of each
                             of its entries u:
                             TC_INTERSECT_AUTO: N_u is walked against a hash of N_v, unless N_u
                             holds 256 entries or more and is longer than search_ratio times the
                             entries of N_v after u (the only candidates), which are then looked
                             up in N_u by binary search;
                             TC_INTERSECT_WALK: always walked; TC_INTERSECT_SEARCH: always
                             searched.  Same results either way.  Set at build or reschedule
                             time; a count call with a non-zero intersect or search_ratio uses
                             its own for that call */
    int32_t search_ratio; /* R of TC_INTERSECT_AUTO, 1 .. 2^20; 0 = automatic (64) */
    int32_t hash;         /* the table of N_v in on-chip memory that each entry of N_u is looked up
                             in (Fig. 1: the test w in S):
                             TC_HASH_AUTO: two-choice (cuckoo) table, every lookup two reads; a
                             list whose insertion fails falls back to linear probing;
                             TC_HASH_LINEAR: linear probing for every list.  Same results either
                             way.  Set at build or reschedule time; a count call with a non-zero
                             hash uses its own for that call */
    int32_t bitmap_ratio; /* dense core (Fig. 1: the test w in N_u, turned around): a one-graph
                             handle built without a budget keeps the rows of its last nodes in
                             the degree order (those of highest degree, whose rows fill a good
                             share of the few labels above them) as bitmaps too, when one of
                             those rows holds 128 entries or more.  With
                             TC_INTERSECT_AUTO, a target row of the core holding 64 entries or
                             more that is longer than bitmap_ratio times the entries of N_v
                             after u (the only candidates) is not read: each candidate is tested
                             against one word of its bitmap instead.  Same results either way.
                             0 = automatic (2); -1 = never (at build time: no core is kept);
                             at most 2^20.  Set at build or reschedule time; a count call with a
                             non-zero bitmap_ratio uses its own for that call */
} tc_options;

enum { TC_INTERSECT_AUTO = 0, TC_INTERSECT_WALK = 1, TC_INTERSECT_SEARCH = 2 };
enum { TC_HASH_AUTO = 0, TC_HASH_LINEAR = 1 };

/* Fills *opt with the defaults (all zero except cost_fn = TC_COST_PRIOR). */
void tc_options_default(tc_options *opt);

/* Opaque handle: the oriented adjacency (in degree-order labels), the map back
 * to caller labels and the task schedule, for k graphs packed together.  Owns
 * its device memory until tc_graph_free. */
typedef struct tc_graph tc_graph;

/* Builds the oriented, sorted adjacency of Fig. 1 for k graphs (k >= 1) in one
 * pass on the device: canonical edge set, degrees, degree order (Section
 * III-A), orientation and row sort, the per-node cost f (Section V-A), and the
 * task table of Eq. (1)/(2).  graphs[i] may have n = 0 or m = 0.  Device
 * inputs laid out back to back (graph i's arrays at graphs[0].src/dst plus the
 * sum of the earlier m) are read in place; others are first copied into that
 * layout.  With a budget, or partitions > 0, a single graph may be built in the
 * partitioned form, its oriented adjacency kept in pinned host memory.
 * Errors: TC_ERR_INVALID_ARG (NULL graphs/out, k < 1, negative n or m, NULL
 * src/dst with m > 0), TC_ERR_ID_RANGE, TC_ERR_TOO_LARGE (sum of n >= 2^31,
 * or 2^32 - 1 or more distinct edges in one resident handle),
 * TC_ERR_OUT_OF_MEMORY, TC_ERR_DEVICE.  *out is written only on TC_OK. */
tc_status tc_build_oriented(const tc_edges *graphs, int32_t k, const tc_options *opt, tc_graph **out);

/* Rebuilds the task table of an existing handle with the schedule options of
 * opt (workers, cost_fn, min_chunk, small_max, rounds, static_chunks; and the
 * count settings intersect, search_ratio, lds_list_max; 0 = automatic, as in
 * tc_build_oriented) without touching the adjacency: per-node costs f
 * (Sections IV-B, IV-F, V-A), the split between lists counted by one wave and
 * by a whole workgroup, and the tasks of Eq. (1)/(2).  Counts are unchanged
 * by construction (Section V-D); only their speed changes.  Errors:
 * TC_ERR_INVALID_ARG, TC_ERR_OUT_OF_MEMORY, TC_ERR_DEVICE. */
tc_status tc_graph_reschedule(tc_graph *g, const tc_options *opt);

/* Total triangle count of each graph in the handle (Fig. 1; Fig. 10/11 task
 * by task): totals[k], int64, host or device per opt->outputs_on_device.
 * Counting one handle concurrently on two streams is not supported. */
tc_status tc_count_total(tc_graph *g, const tc_options *opt, int64_t *totals);

/* Per-node counts T_v (Section II: triangles containing v) in the caller's
 * labels, packed graph after graph: per_node[sum of n_i].  totals (may be
 * NULL) receives the k totals.  Host or device per opt->outputs_on_device. */
tc_status tc_count_per_node(tc_graph *g, const tc_options *opt, int64_t *per_node, int64_t *totals);

/* Counts ng handles in one persistent launch: all their tasks share one
 * queue.  totals receives, handle after handle, each handle's k totals
 * (sum of k entries).  per_node may be NULL; otherwise per_node[i] is NULL or
 * the per-node output of handle i.  Results equal those of separate calls. */
tc_status tc_count_batch(tc_graph *const *gs, int32_t ng, const tc_options *opt, int64_t *totals,
                         int64_t *const *per_node);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count of
 * tc_count_batch with the same arguments and results, whose scratch (queue
 * heads, totals, per-node accumulators, handle descriptors) lives in a fixed
 * device array of TC_STATIC_SCRATCH_BYTES per GPU, held by the library until
 * the process ends, instead of memory allocated per call.  It calls no device
 * allocator.  Outputs must be device pointers (opt->outputs_on_device = 1,
 * else TC_ERR_INVALID_ARG).  The scratch needed is 256 + 8 * (sum of k) +
 * 8 * (sum of n over the handles, when any per-node output is asked for),
 * rounded up to 256, + 200 * ng bytes; a batch that needs more returns
 * TC_ERR_TOO_LARGE before any launch.  Every call on one GPU uses the same
 * array and clears what it reads before the count: calls that overlap on one
 * GPU (two streams, two threads) race and must be serialised by the caller. */
#define TC_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
tc_status tc_count_batch_static(tc_graph *const *gs, int32_t ng, const tc_options *opt, int64_t *totals,
                                int64_t *const *per_node);

/* A count of ng handles captured once as a HIP graph and replayed as one graph
 * launch (Fig. 11: the worker loop of one count, with its queue resets and
 * reductions, as a unit the host launches).  tc_count_capture records on a
 * private stream the work tc_count_batch(gs, ng, opt, totals, per_node) would
 * enqueue: clearing its scratch, the persistent count kernels, the per-node
 * scatter and the copy of the totals.  The scratch is allocated once, through
 * opt's allocator, before the capture.  Outputs must be device pointers
 * (outputs_on_device = 1); every replay rewrites them.  The handles and the
 * outputs must outlive the captured count; a handle rescheduled or freed
 * after the capture must not be replayed.  Errors as tc_count_batch, and
 * TC_ERR_DEVICE if the runtime refuses the capture. */
typedef struct tc_count_graph tc_count_graph;
tc_status tc_count_capture(tc_graph *const *gs, int32_t ng, const tc_options *opt, int64_t *totals,
                           int64_t *const *per_node, tc_count_graph **out);
/* Launches the captured count on opt->stream (NULL opt: the null stream);
 * returns after enqueuing it. */
tc_status tc_count_replay(tc_count_graph *c, const tc_options *opt);
/* Waits for the last replay, then releases the captured count and its
 * scratch.  NULL is a no-op. */
void tc_count_graph_free(tc_count_graph *c);

/* Clustering coefficients from the per-node counts (Section I names them as
 * applications; textbook definitions): coeff[v] = T_v / C(d_v, 2), 0 when
 * d_v < 2, in the caller's labels, packed graph after graph (sum of n_i
 * entries); transitivity[g] = 3 T_g / (sum over v of C(d_v, 2)), 0 when graph g
 * has no path of length two (k entries).  Each value is one fp64 division of
 * two exact integers.  coeff, transitivity and totals (k triangle counts) may
 * each be NULL; host or device per opt->outputs_on_device.  Resident handles
 * only (TC_ERR_INVALID_ARG for a partitioned one). */
tc_status tc_clustering(tc_graph *g, const tc_options *opt, double *coeff, double *transitivity, int64_t *totals);

typedef struct {
    int32_t k;              /* graphs in the handle */
    int64_t n;              /* sum of node counts */
    int64_t m;              /* distinct undirected edges = stored oriented edges */
    int64_t m_input;        /* input edges, loops and repeats included */
    int32_t max_out_degree; /* max |N_v| */
    int64_t tasks;          /* entries of the task table */
    int64_t total_cost;     /* sum of f over all nodes */
    int64_t wide_nodes;     /* nodes whose list is longer than small_max */
    uint64_t device_bytes;  /* device memory held by the handle */
    int32_t partitions;     /* node-range partitions used for counting (1 = resident) */
    int32_t workers;        /* W of the task table (workers it was built for) */
    double last_count_ms;   /* device time of the counting kernels of the last count call made
                               with time_kernels = 1 (waits for it); -1 when none */
    int32_t small_max;      /* longest list counted by one wave in the current task table */
    int32_t cost_fn;        /* cost function of the current task table */
    int64_t streamed_bytes; /* partitioned form: host-to-device bytes moved by the last count */
    uint64_t peak_device_bytes; /* largest device footprint of the handle so far (build included) */
    int32_t rounds;         /* rounds of the current task table (see tc_options.rounds) */
    int32_t search_ratio;   /* intersection of later counts (one-wave lists): -1 = every row
                               searched,
                               0 = every row walked, R > 0 = rows longer than R times their
                               candidates searched (see tc_options.intersect) */
    int32_t hash;           /* TC_HASH_* of later counts (see tc_options.hash) */
    int32_t bitmap_ratio;   /* core tests of later counts: 0 = none (no core, or switched off),
                               B > 0 = core rows longer than B times their candidates tested
                               (see tc_options.bitmap_ratio) */
    int64_t core_rows;      /* rows kept as bitmaps (the last core_rows labels); 0 = no core */
    uint64_t core_bytes;    /* device bytes of those bitmaps */
} tc_graph_info_t;

tc_status tc_graph_info(const tc_graph *g, tc_graph_info_t *info);

/* Copies the oriented adjacency to host arrays for inspection: off[n+1] row
 * offsets and col[m] entries in degree-order labels (rows ascending), and
 * perm[n], the caller label of each degree-order position (Section III-A
 * order; for k graphs, packed labels graph after graph).  Any pointer may be
 * NULL.  Synchronises the stream. */
tc_status tc_export_csr(const tc_graph *g, const tc_options *opt, int64_t *off, int32_t *col, int32_t *perm);

/* Copies the task table: bnd[0..tasks] node boundaries in degree-order labels
 * and, if gid is not NULL, gid[0..tasks-1] the graph of each task.  cap is the
 * capacity of bnd; *tasks receives the number of tasks. */
tc_status tc_export_schedule(const tc_graph *g, const tc_options *opt, int32_t *bnd, int32_t *gid, int64_t cap,
                             int64_t *tasks);

/* Worker timeline of the last count of g made with time_kernels = 2 (resident
 * handles): for each persistent worker i, times[3i] and times[3i+1] receive when
 * it started and when it stopped, in nanoseconds from the earliest start, and
 * times[3i+2] its kind: 0 = a wave taking node-range tasks (Eq. (1)/(2)),
 * 1 = a workgroup taking lists of up to 768 entries, 2 = a workgroup taking
 * longer lists.  cap is the number of workers times can hold; *nworkers
 * receives the number of workers (0 if no such count).  Synchronises the
 * stream.  Errors: TC_ERR_INVALID_ARG (NULL g or nworkers, cap below
 * *nworkers with times non-NULL), TC_ERR_DEVICE. */
tc_status tc_worker_times(const tc_graph *g, const tc_options *opt, int64_t *times, int64_t cap,
                          int64_t *nworkers);

/* Releases the handle and its device memory.  NULL is a no-op. */
void tc_graph_free(tc_graph *g);

const char *tc_status_str(tc_status s);
const char *tc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
