// Internal interfaces between the translation units of the library.
#pragma once

#include <vector>

#include "common.h"

namespace tc {

// scan.hip -- exclusive prefix sums; with write_total, out[n] = sum (out has n+1 slots)
void exclusive_scan(const uint32_t *in, int64_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s);
void exclusive_scan(const int32_t *in, int64_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s);
void exclusive_scan(const int64_t *in, int64_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s);
void exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s);

// sort.hip -- LSD radix sort by bits [begin_bit, end_bit); returns the buffer holding the result
uint64_t *radix_sort_u64(uint64_t *keys, uint64_t *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al,
                         hipStream_t s);
uint32_t *radix_sort_u32(uint32_t *keys, uint32_t *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al,
                         hipStream_t s);
uint32_t *radix_sort_u32_from(const uint32_t *first, uint32_t *keys, uint32_t *tmp, int64_t n, int begin_bit,
                              int end_bit, Allocator &al, hipStream_t s);
// Tiles of the radix passes: kRadixTile keys each, tile t taken by workgroup b
// with xcd_tile(b, tiles) == t, keys t * kRadixTile + w * 1024 + r * 64 + lane
// (w = wave of 4, r = round of 16).  A pass's digit table is digit-major:
// hist[d * tiles + t] = keys of tile t whose digit is d.
constexpr int kRadixTile = 4096;
// The same as radix_sort_u64, with the first pass's digit table (256 * tiles
// words) computed by the caller while it wrote the keys.
uint64_t *radix_sort_u64_hist(uint64_t *keys, uint64_t *tmp, int64_t n, int begin_bit, int end_bit,
                              const uint32_t *first_hist, Allocator &al, hipStream_t s);

// build.hip -------------------------------------------------------------

// Node and edge layout of the k graphs packed into one handle.
struct Packing {
    int32_t k = 0;
    std::vector<int64_t> node_base;  // k+1, host
    std::vector<int64_t> edge_base;  // k+1, host
    int64_t N = 0;                   // sum of n
    int64_t M_in = 0;                // sum of input edges
    int32_t max_n = 0;
};

struct BuildParams {
    int32_t workers = 0;
    int32_t cost_fn = TC_COST_PRIOR;
    int64_t min_chunk = 0;
    int32_t small_max = 128;
    int32_t rounds = 0;  // Eq. (1) with W = workers * rounds; 0 = automatic
    int32_t direct = 0;  // partitioned form: one streamed range per stored edge
    int32_t static_chunks = 0;  // W equal-cost tasks instead of Eq. (1)/(2)
    int32_t core = 1;           // keep the dense core's rows as bitmaps too (Oriented::bm)
};

// Automatic rounds: one for a single graph; for k packed graphs, enough that
// the tasks in flight (1 / (2 rounds) of the edges) hold about 64 MiB of rows.
int32_t auto_rounds(int32_t k, int64_t M);

// Device-side product of a build (all in degree-order labels).
struct Oriented {
    DevBuf<int64_t> off;        // N+1
    DevBuf<int32_t> col;        // M
    DevBuf<int32_t> perm;       // N: packed caller label of each position
    DevBuf<int32_t> deg;        // N: degree (distinct neighbours) of each position
    DevBuf<int64_t> node_base;  // k+1 (device copy)
    DevBuf<int32_t> bnd;        // tasks+1
    DevBuf<int32_t> gid;        // tasks (k > 1 only)
    DevBuf<int32_t> start;      // tasks: where each task's scan begins (see Schedule::start)
    DevBuf<int32_t> big;        // long lists, handled by whole workgroups: medium ones first
    int64_t M = 0;
    int64_t tasks = 0;
    int64_t total_cost = 0;
    int64_t nbig = 0;
    int64_t nmed = 0;  // lists in big[0, nmed) have at most max_medium_list() entries
    int32_t max_dhat = 0;
    int32_t rounds = 1;  // rounds of the task table
    DevBuf<int32_t> samp;  // ceil(M / kSampleStride): col[j * kSampleStride]
    // Dense core (one graph only): the core's adjacency as bitmaps, see CoreLayout
    DevBuf<uint32_t> bm;
    struct CoreLayout {
        int32_t lo = 0;   // first core label; N = no core
        int32_t wl = 0;   // (N - 1) >> 5: the last word of a row
        int32_t kw = 0;   // words per row: wl - (lo >> 5) + 1
        int64_t words = 0;
    } core;
};

// Layout of the core bitmaps: one row of kw words per core label u, rows in
// label order from core.lo, word j of a row covering the labels
// 32 * ((lo >> 5) + j) .. + 31; bit x & 31 of the word of x is set in row u
// when u and x are adjacent (both in the core).  Over labels above u a row is
// N_u (every member of N_u lies above u by the degree order); below u it holds
// the core nodes whose lists contain u.  core_origin(u) + (x >> 5) is the word
// of x in row u.
__host__ __device__ __forceinline__ int64_t core_origin(int64_t u, int64_t lo, int64_t kw) {
    return (u - lo) * kw - (lo >> 5);
}

// src/dst: packed input edges on the device (edge e of graph g at edge_base[g] + i).
void build_oriented_device(const int32_t *src, const int32_t *dst, const Packing &pk, const BuildParams &bp,
                           Allocator &al, hipStream_t s, Oriented &out);

// Recomputes the per-node costs, the wide-list bucket and the task table of
// an existing build with new parameters (the adjacency is unchanged).
void reschedule_device(const Packing &pk, const BuildParams &bp, Allocator &al, hipStream_t s, Oriented &out);

// Fill helpers usable inside captured streams (no memset nodes).
void fill_zero(void *p, size_t bytes, hipStream_t s);

// Task table of an arbitrary set of N sources: f[i] = cost of source i (0 for
// lists handled by workgroups), wmed / wlarge flag the workgroup lists.
struct Schedule {
    DevBuf<int32_t> bnd;  // tasks+1
    DevBuf<int32_t> gid;  // tasks (k > 1 only)
    // tasks, only when schedule_sources is given the degrees: the first node of
    // task c of degree 2 or more (bnd[c+1] if none), where its scan begins
    DevBuf<int32_t> start;
    DevBuf<int32_t> big;  // medium lists first, then large ones
    int64_t tasks = 0;
    int64_t total_cost = 0;
    int64_t nmed = 0;
    int64_t nbig = 0;
};
// Eq. (1)/(2) cost targets of a schedule (bp.rounds resolved) for a total cost.
std::vector<int64_t> schedule_targets(int64_t total, const BuildParams &bp);
// Targets computed ahead (on the host, while the device works) for a total
// cost; schedule_sources takes them when its total is the same.
struct PresetTargets {
    int64_t total = -1;
    std::vector<int64_t> targets;
};
// Device words copied to the host together with the schedule's totals, so
// that one synchronisation serves both.
struct Piggyback {
    const uint32_t *dev[2] = {nullptr, nullptr};
    uint32_t host[2] = {0, 0};
};
void schedule_sources(const int64_t *f, const uint32_t *wmed, const uint32_t *wlarge, int64_t N, int k,
                      const int64_t *node_base, const BuildParams &bp, Allocator &al, Allocator &tmp, hipStream_t s,
                      Schedule &out, const int32_t *maxd_dev = nullptr, int32_t *maxd_host = nullptr,
                      PresetTargets *pre = nullptr, const int32_t *deg_sorted = nullptr,
                      Piggyback *pb = nullptr);
std::vector<int64_t> task_targets(int64_t total, int32_t W, int64_t min_chunk, bool static_chunks = false);
// bnd[0] = 0, bnd[j+1] = first x in [0, N] with F[x] >= targets[j] (targets < 0: N)
void task_bounds(const int64_t *F, int64_t N, const std::vector<int64_t> &targets, int32_t *bnd, Allocator &tmp,
                 hipStream_t s);
// Build steps shared by the resident and the partitioned builds.
// Distinct valid keys of sorted[0..n), in order.  *res is set to where they
// are: sorted itself when all n keys are distinct and valid (nothing is
// copied), else out.  Synchronises; returns their number.
int64_t unique_sorted_keys(uint64_t *sorted, int64_t n, uint64_t *out, uint64_t **res, Allocator &tmp,
                           hipStream_t s);
// deg[x] += number of distinct neighbours of x in the sorted, distinct pair
// keys (x_lo << gb) | x_hi; deg has N entries, every label is below N.
void add_degrees(const uint64_t *ukeys, int64_t M, int gb, int32_t *deg, int64_t N, uint32_t *spare /* 2 M words */,
                 Allocator &tmp, hipStream_t s);
void degree_rank(const int32_t *deg, int64_t N, const int64_t *node_base, int k, int32_t max_n, int32_t *perm,
                 int32_t *rank, Allocator &tmp, hipStream_t s);

// partition.hip ----------------------------------------------------------

// A graph counted in P consecutive node ranges ("slices") of the degree order
// (Definition 1), with its oriented adjacency in page-locked host memory.
// For slice j = [cut[j], cut[j+1]), the streamed ranges are records
// rbase[j] .. rbase[j+1]: node rv, entries hcol[rpos .. rpos + rlen) (the part
// of N_rv from its first entry at or after cut[j]), whose first rtc entries
// lie inside the slice.
struct Partitioned {
    int64_t N = 0;
    int64_t M = 0;
    int32_t P = 0;
    int32_t max_dhat = 0;
    std::vector<int64_t> cut;   // P+1
    std::vector<int64_t> ecut;  // P+1: off[cut[j]]
    HostBuf<int64_t> off;       // N+1
    HostBuf<int32_t> col;       // M
    HostBuf<int32_t> rv, rtc, rlen;
    HostBuf<int64_t> rpos;
    std::vector<int64_t> rbase;  // P+1
    std::vector<int64_t> batch;  // record batches: [batch[b], batch[b+1]) never spans two slices
    DevBuf<int32_t> perm;        // N, device: caller label of each position
    int64_t rows_max = 0;        // largest slice (rows, entries)
    int64_t entries_max = 0;
    int64_t msg_cap = 0;  // largest streamed ids / records of one batch
    int64_t rec_cap = 0;
    int64_t streamed_bytes = 0;  // host-to-device bytes of the last count
    bool direct = false;         // records follow the direct scheme
};

// Builds the partitioned form of one graph.  src/dst: host arrays, or device
// arrays when on_device.  Every device allocation goes through `al`, whose
// budget (if any) bounds the peak.  partitions: at least this many slices.
void build_partitioned(const int32_t *src, const int32_t *dst, bool on_device, const Packing &pk,
                       const BuildParams &bp, int32_t partitions, Allocator &al, hipStream_t s, Partitioned &out);

// Counts a partitioned graph slice by slice; totals (1 entry) and tv (N
// entries, degree-order labels, may be NULL) are device arrays, zeroed here.
// search: the one-wave intersection choice of the descriptors (CountDesc).
void count_partitioned(Partitioned &pg, const BuildParams &bp, int32_t lds_max, int32_t search,
                       int32_t cuckoo_rounds, Allocator &al,
                       hipStream_t s, int64_t *totals, int64_t *tv, uint32_t *heads);

// count.hip --------------------------------------------------------------

struct CountDesc {
    const int64_t *off;  // target rows: row of label t is off[t - row_lo] .. off[t - row_lo + 1] in col
    const int32_t *col;
    const int32_t *bnd;
    const int32_t *start;      // tasks, or NULL: task c scans nodes start[c] .. bnd[c+1]
    const int32_t *gid;        // NULL when k == 1
    const int64_t *node_base;  // k+1
    const int32_t *big;  // long lists: [0, nmed) up to 1024 entries, [nmed, nbig) longer
    int64_t *totals;  // k
    int64_t *tv;      // N (degree-order labels) or NULL
    int64_t m;  // entries of col (bounds every row read)
    int64_t nmed;
    int64_t nbig;
    int64_t task_base;
    int64_t med_base;
    int64_t large_base;
    int32_t k;
    int32_t small_max;  // lists up to this length were scheduled for single waves
    // Slice launches only (CountLaunch::slice): source i hashes the list
    // scol[soff[i] .. soff[i+1]), is labelled sid[i], and its first
    // min(tcnt[i], a - 1) entries are the targets whose rows are resident.
    const int64_t *soff;
    const int32_t *scol;
    const int32_t *sid;
    const int32_t *tcnt;
    int32_t row_lo;
    // one-wave lists: a target row longer than search_ratio times the list
    // entries after the target is binary-searched instead of walked; -1 =
    // every row, 0 = none
    int32_t search_ratio;
    // every kSampleStride-th entry of col (samp[j] = col[j * kSampleStride]),
    // the first level of those searches; NULL: search col directly
    const int32_t *samp;
    // Dense core (Oriented::bm): a target row u >= core_lo of at least
    // kCoreMinProbe entries that is longer than bitmap_ratio times the list
    // entries after u is not walked; those entries are tested against its
    // bitmap instead.  bm NULL or bitmap_ratio 0: none.
    const uint32_t *bm;
    int32_t core_lo;
    int32_t core_wl;
    int32_t core_kw;
    int32_t bitmap_ratio;
};
constexpr int kCoreMinProbe = 64;
// The core starts at a row that fills at least 1 / kCoreDensity of the labels
// above it.  A source of the core meets its list by bitmap AND when its own
// list fills at least 1 / kAndDensity of them (total only; per node, where
// every entry's whole row is AND-ed, 2 / kAndDensity): a list of a entries
// among the d labels above the source otherwise costs about a * a / 2 tests
// of single words, against a * d / 64 words AND-ed (a * d / 32 per node).
constexpr int kCoreDensity = 128;
constexpr int kAndDensity = 32;
constexpr int kSampleShift = 5;
constexpr int64_t kSampleStride = (int64_t)1 << kSampleShift;  // entries per sample (one 128-byte line)

// Moves a two-choice insertion may make before the list falls back to linear
// probing.
constexpr int32_t kCuckooRounds = 96;

struct CountLaunch {
    const CountDesc *descs;  // device array
    int32_t ndesc;
    int64_t total_tasks;
    int64_t total_med;
    int64_t total_large;
    uint32_t *heads;  // 3 counters, zeroed before launch
    int64_t max_m;    // largest adjacency (entries of col) among the descriptors
    int32_t workers;  // persistent waves for the small-list kernel
    int32_t lds_max;     // longest list kept in LDS by the workgroup kernels
    int32_t cuckoo_rounds;  // two-choice table eviction limit; 0 = linear probing
    bool per_node;
    bool slice;  // descriptors are slice launches (32-bit row addressing)
    bool core = false;  // some descriptor has a core and asks for its bit tests
    // optional per-worker (start, finish) timestamps, wall-clock ticks: small-list
    // waves first, then the workgroups of each tier; capacity in pairs
    unsigned long long *times = nullptr;
    int64_t times_cap = 0;
    int64_t times_used = 0;  // set by count_launch: workers that wrote a pair
    int64_t times_tier[3] = {0, 0, 0};  // set by count_launch: workers of each kernel
};

void count_launch(CountLaunch &L, hipStream_t s);
int64_t max_timed_workers();  // upper bound on the workers of one count_launch

// coeff[perm[i]] = tv[i] / C(deg[i], 2); trans[g] = 3 totals[g] / (sum of C(deg, 2)
// over graph g); wedges: k scratch words.  coeff or trans may be NULL.
void clustering_epilogue(const int64_t *tv, const int32_t *deg, const int32_t *perm, int64_t N,
                         const int64_t *node_base, int k, const int64_t *totals, double *coeff, double *trans,
                         unsigned long long *wedges, hipStream_t s);

// out[perm[i]] = tv[i] for i < n
void scatter_per_node(const int64_t *tv, const int32_t *perm, int64_t n, int64_t *out, hipStream_t s);

int device_cu_count();
int max_small_list();
int max_medium_list();
int small_kernel_waves_per_cu(bool per_node);  // resident waves per CU
int max_lds_list();

}  // namespace tc
