// C ABI of the library (declared in include/tc.h).  Host orchestration only:
// argument checks, packing of input graphs, allocation, and kernel launches.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>

#include "internal.h"

struct tc_graph {
    tc::Allocator al;  // allocator of the handle's own memory (stream = last stream used)
    tc::Packing pk;
    tc::Oriented o;
    std::unique_ptr<tc::Partitioned> part;  // set when counted in node-range partitions
    int64_t min_chunk = 0;
    int64_t max_graph_m = 0;  // entries of the largest graph's rows (bounds graph-relative row addressing)
    int32_t rounds = 0;       // as asked (0 = automatic)
    int32_t workers = 0;
    int32_t small_max = 128;
    int32_t lds_max = 1920;  // as tc::max_lds_list(); set at build
    int32_t cost_fn = TC_COST_PRIOR;
    int32_t search = 64;  // one-wave lists: search ratio of the descriptors (-1 every row, 0 none)
    int32_t hash = TC_HASH_AUTO;  // LDS table of the lists: two-choice or linear probing
    int32_t bitmap = 2;  // core rows: bitmap ratio of the descriptors (0 none)
    // persistent count scratch: queue heads, totals, per-node accumulators
    tc::DevBuf<uint32_t> heads;
    tc::DevBuf<int64_t> totals;
    tc::DevBuf<int64_t> tv;
    tc::DevBuf<tc::CountDesc> desc;  // one descriptor pointing at the buffers above
    bool desc_has_tv = false;
    int32_t desc_search = 0;  // search ratio written into desc
    int32_t desc_bitmap = 0;  // bitmap ratio written into desc
    // optional device timing of the counting kernels
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool timed = false;
    // per-worker (start, stop) wall-clock ticks of the last count with time_kernels = 2
    tc::DevBuf<unsigned long long> times;
    int64_t times_used = 0;
    int64_t times_tier[3] = {0, 0, 0};
    int32_t static_chunks = 0;
    ~tc_graph() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// A count captured as a HIP graph (tc_count_capture): its own scratch and the
// instantiated graph; the handles it counts are referenced, not owned.
struct tc_count_graph {
    tc::Allocator al;
    tc::DevBuf<uint8_t> scratch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;  // stream of the last replay
    ~tc_count_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

thread_local std::string g_last_error;

tc_status fail(tc_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

template <class F>
tc_status guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return TC_OK;
    } catch (const tc::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(TC_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(TC_ERR_DEVICE, e.what());
    }
}

tc::Allocator make_allocator(const tc_options *opt) {
    tc::Allocator a;
    if (opt) {
        a.fn_alloc = opt->alloc;
        a.fn_free = opt->free;
        a.ctx = opt->alloc_ctx;
        a.stream = (hipStream_t)opt->stream;
        a.budget = opt->hbm_budget_bytes;
    }
    return a;
}

void check_options(const tc_options *opt) {
    if (!opt) return;
    if ((opt->alloc == nullptr) != (opt->free == nullptr))
        throw tc::Error(TC_ERR_INVALID_ARG, "alloc and free callbacks must be given together");
    if (opt->workers < 0 || opt->min_chunk < 0 || opt->small_max < 0 || opt->lds_list_max < 0 || opt->rounds < 0 ||
        opt->partitions < 0 || opt->direct < 0)
        throw tc::Error(TC_ERR_INVALID_ARG, "negative option value");
    if (opt->cost_fn < TC_COST_ONE || opt->cost_fn > TC_COST_NEW)
        throw tc::Error(TC_ERR_INVALID_ARG, "unknown cost function");
    if (opt->intersect < TC_INTERSECT_AUTO || opt->intersect > TC_INTERSECT_SEARCH)
        throw tc::Error(TC_ERR_INVALID_ARG, "unknown intersection variant");
    if (opt->search_ratio < 0 || opt->search_ratio > (1 << 20))
        throw tc::Error(TC_ERR_INVALID_ARG, "search_ratio outside 0 .. 2^20");
    if (opt->hash < TC_HASH_AUTO || opt->hash > TC_HASH_LINEAR)
        throw tc::Error(TC_ERR_INVALID_ARG, "unknown hash table kind");
    if (opt->bitmap_ratio < -1 || opt->bitmap_ratio > (1 << 20))
        throw tc::Error(TC_ERR_INVALID_ARG, "bitmap_ratio outside -1 .. 2^20");
}

constexpr int32_t kDefaultSearchRatio = 64;

// Descriptor encoding of the intersection choice: -1 = search every row,
// 0 = walk every row, R > 0 = search rows longer than R times their candidates.
int32_t resolve_search(int32_t intersect, int32_t ratio) {
    if (intersect == TC_INTERSECT_WALK) return 0;
    if (intersect == TC_INTERSECT_SEARCH) return -1;
    return ratio > 0 ? ratio : kDefaultSearchRatio;
}

constexpr int32_t kDefaultBitmapRatio = 2;

// Descriptor encoding of the core tests: 0 = none, B > 0 = core rows longer
// than B times their candidates are tested against their bitmaps.  Only the
// automatic intersection uses them.
int32_t resolve_bitmap(int32_t intersect, int32_t ratio) {
    if (intersect != TC_INTERSECT_AUTO || ratio < 0) return 0;
    return ratio > 0 ? ratio : kDefaultBitmapRatio;
}

// The core-test setting of a count call: its own when it names one, else the handle's.
int32_t count_bitmap(const tc_graph *g, const tc_options *opt) {
    if (opt && (opt->intersect != TC_INTERSECT_AUTO || opt->bitmap_ratio != 0))
        return resolve_bitmap(opt->intersect, opt->bitmap_ratio);
    return g->bitmap;
}

// Eviction limit of the two-choice table for a count call (0 = linear
// probing): the call's table kind when it names one, else the handle's.
int32_t count_rounds(const tc_graph *g, const tc_options *opt) {
    const int32_t h = opt && opt->hash != TC_HASH_AUTO ? opt->hash : g->hash;
    return h == TC_HASH_LINEAR ? 0 : tc::kCuckooRounds;
}

// The search setting of a count call: its own when it names one, else the handle's.
int32_t count_search(const tc_graph *g, const tc_options *opt) {
    if (opt && (opt->intersect != TC_INTERSECT_AUTO || opt->search_ratio != 0))
        return resolve_search(opt->intersect, opt->search_ratio);
    return g->search;
}

// Stores a descriptor passed by value (kernel arguments need no host copy).
__global__ void k_store_desc(tc::CountDesc d, tc::CountDesc *out) {
    if (threadIdx.x == 0) *out = d;
}

// Zeroes the queue heads (4 words), the totals (k) and, when tv is given, the
// per-node counters (n): one launch for what a count starts from.
__global__ void k_count_reset(uint32_t *heads, int64_t *totals, int64_t k, int64_t *tv, int64_t n) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    if (i0 < 4) heads[i0] = 0u;
    for (int64_t i = i0; i < k; i += st) totals[i] = 0;
    if (tv)
        for (int64_t i = i0; i < n; i += st) tv[i] = 0;
}

// The core fields of a descriptor (none when the handle has no core).
void set_core(tc::CountDesc &d, const tc_graph *g, int32_t bitmap) {
    d.bm = g->o.bm.p;
    d.core_lo = g->o.core.lo;
    d.core_wl = g->o.core.wl;
    d.core_kw = g->o.core.kw;
    d.bitmap_ratio = g->o.bm.p ? bitmap : 0;
}

// Per-handle descriptor used by single-handle counts (kept on the device).
void ensure_scratch(tc_graph *g, bool per_node, int32_t search, int32_t bitmap, hipStream_t s) {
    g->al.stream = s;
    if (!g->heads.p) g->heads = tc::DevBuf<uint32_t>(g->al, 4);  // 3 queue heads
    if (!g->totals.p) g->totals = tc::DevBuf<int64_t>(g->al, (size_t)std::max(g->pk.k, 1));
    if (per_node && !g->tv.p) g->tv = tc::DevBuf<int64_t>(g->al, (size_t)std::max<int64_t>(g->pk.N, 1));
    if (!g->part && (!g->desc.p || (per_node && !g->desc_has_tv) || g->desc_search != search ||
                     g->desc_bitmap != bitmap)) {
        tc::CountDesc d{};
        d.off = g->o.off.p;
        d.col = g->o.col.p;
        d.bnd = g->o.bnd.p;
        d.start = g->o.start.p;
        d.gid = g->pk.k > 1 ? g->o.gid.p : nullptr;
        d.node_base = g->o.node_base.p;
        d.big = g->o.big.p;
        d.m = g->o.M;
        d.totals = g->totals.p;
        d.tv = g->tv.p;
        d.nmed = g->o.nmed;
        d.nbig = g->o.nbig;
        d.task_base = 0;
        d.med_base = 0;
        d.large_base = 0;
        d.k = g->pk.k;
        d.small_max = g->small_max;
        d.search_ratio = search;
        d.samp = g->o.samp.p;
        set_core(d, g, bitmap);
        if (!g->desc.p) g->desc = tc::DevBuf<tc::CountDesc>(g->al, 1);
        k_store_desc<<<1, 64, 0, s>>>(d, g->desc.p);
        TC_LAUNCH_CHECK();
        g->desc_has_tv = g->tv.p != nullptr;
        g->desc_search = search;
        g->desc_bitmap = bitmap;
    }
}

void copy_out(void *dst, const void *src, size_t bytes, bool dst_on_device, hipStream_t s) {
    if (bytes == 0) return;
    TC_HIP(hipMemcpyAsync(dst, src, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
}

tc_status check_batch_args(tc_graph *const *gs, int32_t ng, const int64_t *totals) {
    if (!gs || ng < 1 || !totals) return fail(TC_ERR_INVALID_ARG, "graphs, ng >= 1 and totals are required");
    for (int32_t i = 0; i < ng; ++i) {
        if (!gs[i]) return fail(TC_ERR_INVALID_ARG, "NULL graph in batch");
        if (gs[i]->part) return fail(TC_ERR_INVALID_ARG, "a partitioned handle cannot join a batch");
    }
    return TC_OK;
}

// Scratch of one batch count, at byte offsets from its base: the queue heads,
// the totals of every graph, the per-node accumulators (degree-order labels,
// handle after handle) and the count descriptors of the handles.
struct BatchLayout {
    std::vector<int64_t> kbase, nbase;  // ng+1: first total / accumulator of each handle
    bool want_tv = false;
    size_t tot_off = 0, tv_off = 0, zero_bytes = 0, desc_off = 0, bytes = 0;
};

BatchLayout batch_layout(tc_graph *const *gs, int32_t ng, int64_t *const *per_node) {
    BatchLayout b;
    b.kbase.assign((size_t)ng + 1, 0);
    b.nbase.assign((size_t)ng + 1, 0);
    if (per_node)
        for (int32_t i = 0; i < ng; ++i) b.want_tv = b.want_tv || (per_node[i] != nullptr && gs[i]->pk.N > 0);
    for (int32_t i = 0; i < ng; ++i) {
        b.kbase[i + 1] = b.kbase[i] + gs[i]->pk.k;
        b.nbase[i + 1] = b.nbase[i] + (b.want_tv ? gs[i]->pk.N : 0);
    }
    b.tot_off = 256;
    b.tv_off = b.tot_off + (size_t)b.kbase[ng] * 8;
    b.zero_bytes = b.tv_off + (size_t)b.nbase[ng] * 8;
    b.desc_off = (b.zero_bytes + 255) & ~(size_t)255;
    b.bytes = b.desc_off + (size_t)ng * sizeof(tc::CountDesc);
    return b;
}

// Descriptors stored by kernels whose arguments carry them: no host buffer
// has to outlive the call, so the upload can be captured in a graph.
constexpr int kDescPack = 15;
struct DescPack {
    tc::CountDesc d[kDescPack];
};
static_assert(sizeof(DescPack) <= 3072, "descriptor pack must fit the kernel argument space");
static_assert(sizeof(tc::CountDesc) == 200, "tc.h states the scratch of tc_count_batch_static with 200-byte descriptors");

__global__ void k_store_descs(DescPack p, int n, tc::CountDesc *out) {
    const int i = (int)threadIdx.x;
    if (i < n) out[i] = p.d[i];
}

// Zeroes the heads, totals and accumulators in `base`, stores the handles'
// descriptors and launches the persistent count over all of their tasks.
void launch_batch(tc_graph *const *gs, int32_t ng, const tc_options *opt, const BatchLayout &lay, uint8_t *base,
                  bool descs_by_kernel, hipStream_t s) {
    tc::fill_zero(base, lay.zero_bytes, s);
    uint32_t *heads = (uint32_t *)base;
    int64_t *tot = (int64_t *)(base + lay.tot_off);
    int64_t *tv = (int64_t *)(base + lay.tv_off);
    tc::CountDesc *ddesc = (tc::CountDesc *)(base + lay.desc_off);
    std::vector<tc::CountDesc> hd((size_t)ng);
    int64_t task_base = 0, med_base = 0, large_base = 0;
    int32_t workers = 0, lds_max = tc::max_lds_list(), rounds = tc::kCuckooRounds;
    bool core = false;
    for (int32_t i = 0; i < ng; ++i) {
        const tc_graph *g = gs[i];
        tc::CountDesc &d = hd[i];
        d = tc::CountDesc{};
        d.off = g->o.off.p;
        d.col = g->o.col.p;
        d.bnd = g->o.bnd.p;
        d.start = g->o.start.p;
        d.gid = g->pk.k > 1 ? g->o.gid.p : nullptr;
        d.node_base = g->o.node_base.p;
        d.big = g->o.big.p;
        d.m = g->o.M;
        d.totals = tot + lay.kbase[i];
        d.tv = lay.want_tv ? tv + lay.nbase[i] : nullptr;
        d.nmed = g->o.nmed;
        d.nbig = g->o.nbig;
        d.task_base = task_base;
        d.med_base = med_base;
        d.large_base = large_base;
        d.k = g->pk.k;
        d.small_max = g->small_max;
        d.search_ratio = count_search(g, opt);
        d.samp = g->o.samp.p;
        set_core(d, g, count_bitmap(g, opt));
        task_base += g->o.tasks;
        med_base += g->o.nmed;
        large_base += g->o.nbig - g->o.nmed;
        workers = std::max(workers, g->workers);
        lds_max = std::min(lds_max, g->lds_max);
        core = core || d.bitmap_ratio > 0;
        rounds = std::min(rounds, count_rounds(g, opt));
    }
    if (descs_by_kernel) {
        for (int32_t b = 0; b < ng; b += kDescPack) {
            DescPack p;
            const int c = std::min<int32_t>(kDescPack, ng - b);
            std::memcpy(p.d, hd.data() + b, (size_t)c * sizeof(tc::CountDesc));
            k_store_descs<<<1, 64, 0, s>>>(p, c, ddesc + b);
            TC_LAUNCH_CHECK();
        }
    } else {
        TC_HIP(hipMemcpyAsync(ddesc, hd.data(), ng * sizeof(tc::CountDesc), hipMemcpyHostToDevice, s));
    }
    tc::CountLaunch L{};
    L.descs = ddesc;
    L.ndesc = ng;
    L.total_tasks = task_base;
    L.total_med = med_base;
    L.total_large = large_base;
    L.max_m = 0;
    for (int32_t i = 0; i < ng; ++i) L.max_m = std::max<int64_t>(L.max_m, gs[i]->max_graph_m);
    L.heads = heads;
    L.workers = opt && opt->workers > 0 ? opt->workers : workers;
    L.lds_max = opt && opt->lds_list_max > 0 ? opt->lds_list_max : lds_max;
    L.cuckoo_rounds = rounds;
    L.per_node = lay.want_tv;
    L.core = core;
    tc::count_launch(L, s);
}

// Device outputs of a batch count: per-node counts scattered to caller
// labels, totals copied out.
void write_device_outputs(tc_graph *const *gs, int32_t ng, const BatchLayout &lay, const uint8_t *base,
                          int64_t *totals, int64_t *const *per_node, hipStream_t s) {
    const int64_t *tv = (const int64_t *)(base + lay.tv_off);
    for (int32_t i = 0; i < ng && per_node; ++i)
        if (per_node[i] && gs[i]->pk.N > 0)
            tc::scatter_per_node(tv + lay.nbase[i], gs[i]->o.perm.p, gs[i]->pk.N, per_node[i], s);
    copy_out(totals, base + lay.tot_off, (size_t)lay.kbase[ng] * 8, true, s);
}

// Scratch of tc_count_batch_static: one array per GPU, held until the process
// ends.  Host code reaches it only through the device address that
// hipGetSymbolAddress gives for the current device (the symbol's host-side
// name is not a device address).
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];
std::mutex g_static_mu;
std::vector<void *> g_static_ptr;  // per device ordinal

void *static_scratch(int dev) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_ptr.empty()) {
        int count = 0;
        TC_HIP(hipGetDeviceCount(&count));
        g_static_ptr.assign((size_t)std::max(count, 1), nullptr);
    }
    if (dev < 0 || dev >= (int)g_static_ptr.size()) throw tc::Error(TC_ERR_DEVICE, "current device out of range");
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw tc::Error(TC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_static_ptr[dev] = p;
    }
    return g_static_ptr[dev];
}

}  // namespace

extern "C" {

void tc_options_default(tc_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->cost_fn = TC_COST_PRIOR;
}

const char *tc_status_str(tc_status s) {
    switch (s) {
        case TC_OK: return "ok";
        case TC_ERR_INVALID_ARG: return "invalid argument";
        case TC_ERR_ID_RANGE: return "node id out of range";
        case TC_ERR_TOO_LARGE: return "too large";
        case TC_ERR_OUT_OF_MEMORY: return "out of device memory";
        case TC_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

const char *tc_last_error(void) { return g_last_error.c_str(); }

tc_status tc_build_oriented(const tc_edges *graphs, int32_t k, const tc_options *opt, tc_graph **out) {
    if (!graphs || !out || k < 1) return fail(TC_ERR_INVALID_ARG, "graphs and out must be non-NULL and k >= 1");
    std::unique_ptr<tc_graph> g(new (std::nothrow) tc_graph());
    if (!g) return fail(TC_ERR_OUT_OF_MEMORY, "host allocation failed");
    tc_status st = guarded([&] {
        check_options(opt);
        tc_options o;
        if (opt)
            o = *opt;
        else
            tc_options_default(&o);
        hipStream_t s = (hipStream_t)o.stream;
        tc::Packing &pk = g->pk;
        pk.k = k;
        pk.node_base.assign((size_t)k + 1, 0);
        pk.edge_base.assign((size_t)k + 1, 0);
        for (int32_t i = 0; i < k; ++i) {
            const tc_edges &e = graphs[i];
            if (e.n < 0 || e.m < 0) throw tc::Error(TC_ERR_INVALID_ARG, "negative n or m");
            if (e.m > 0 && (!e.src || !e.dst)) throw tc::Error(TC_ERR_INVALID_ARG, "NULL edge arrays with m > 0");
            pk.node_base[i + 1] = pk.node_base[i] + e.n;
            pk.edge_base[i + 1] = pk.edge_base[i] + e.m;
            pk.max_n = std::max(pk.max_n, e.n);
        }
        pk.N = pk.node_base[k];
        pk.M_in = pk.edge_base[k];
        if (pk.N >= ((int64_t)1 << 31) - 1) throw tc::Error(TC_ERR_TOO_LARGE, "sum of n must stay below 2^31 - 1");

        g->al = make_allocator(&o);
        const int cus = tc::device_cu_count();
        g->workers = o.workers > 0 ? o.workers : tc::small_kernel_waves_per_cu(true) * cus;
        g->small_max = o.small_max > 0 ? std::min(o.small_max, tc::max_small_list()) : tc::max_small_list();
        g->lds_max = o.lds_list_max > 0 ? std::max(2, std::min(o.lds_list_max, tc::max_lds_list())) : tc::max_lds_list();
        g->cost_fn = o.cost_fn;
        g->min_chunk = o.min_chunk;
        g->rounds = o.rounds;
        g->search = resolve_search(o.intersect, o.search_ratio);
        g->hash = o.hash;
        g->bitmap = resolve_bitmap(o.intersect, o.bitmap_ratio);
        tc::BuildParams bp;
        bp.workers = g->workers;
        bp.cost_fn = o.cost_fn;
        bp.min_chunk = o.min_chunk;
        bp.small_max = g->small_max;
        bp.rounds = o.rounds;
        bp.direct = o.direct;
        bp.static_chunks = o.static_chunks;
        bp.core = o.bitmap_ratio >= 0;  // -1 at build time: no core at all
        g->static_chunks = o.static_chunks;

        // Resident unless forced or over the budget: the resident build holds
        // the input (when copied in), its scratch, the adjacency and the count
        // buffers at once.
        const uint64_t budget = o.hbm_budget_bytes;
        const bool copy_in = !o.inputs_on_device;
        const uint64_t resident_need = (uint64_t)pk.M_in * (31 + (copy_in ? 8 : 0)) + (uint64_t)pk.N * 108 +
                                       (uint64_t)g->workers * 160 + ((uint64_t)32 << 20);
        const bool part = pk.N > 0 && (o.partitions > 0 || (budget > 0 && resident_need > budget));
        if (part) {
            if (k != 1) {
                if (o.partitions > 0)
                    throw tc::Error(TC_ERR_INVALID_ARG, "the partitioned form holds one graph per handle");
                throw tc::Error(TC_ERR_OUT_OF_MEMORY, "graphs do not fit the device budget together");
            }
            g->part.reset(new tc::Partitioned());
            tc::build_partitioned(graphs[0].src, graphs[0].dst, o.inputs_on_device != 0, pk, bp, o.partitions, g->al,
                                  s, *g->part);
            return;
        }

        // packed input edges on the device
        tc::DevBuf<int32_t> psrc, pdst;
        const int32_t *dsrc = nullptr, *ddst = nullptr;
        // device inputs already laid out graph after graph (edge e of graph i
        // at src[edge_base[i] + e]) are read in place
        bool in_place = o.inputs_on_device != 0;
        for (int32_t i = 0; i < k && in_place && k > 1; ++i)
            if (graphs[i].m > 0)
                in_place = (uintptr_t)graphs[i].src == (uintptr_t)graphs[0].src + 4 * (uintptr_t)pk.edge_base[i] &&
                           (uintptr_t)graphs[i].dst == (uintptr_t)graphs[0].dst + 4 * (uintptr_t)pk.edge_base[i];
        if (in_place) {
            dsrc = graphs[0].src;
            ddst = graphs[0].dst;
        } else if (pk.M_in > 0) {
            psrc = tc::DevBuf<int32_t>(g->al, (size_t)pk.M_in);
            pdst = tc::DevBuf<int32_t>(g->al, (size_t)pk.M_in);
            const hipMemcpyKind kind = o.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            for (int32_t i = 0; i < k; ++i) {
                const size_t bytes = (size_t)graphs[i].m * sizeof(int32_t);
                if (!bytes) continue;
                TC_HIP(hipMemcpyAsync(psrc.p + pk.edge_base[i], graphs[i].src, bytes, kind, s));
                TC_HIP(hipMemcpyAsync(pdst.p + pk.edge_base[i], graphs[i].dst, bytes, kind, s));
            }
            dsrc = psrc.p;
            ddst = pdst.p;
        }
        if (budget > 0 && k == 1) {
            // the estimate above is an upper bound in practice; should the
            // resident build still run out of budget, build partitioned
            try {
                tc::build_oriented_device(dsrc, ddst, pk, bp, g->al, s, g->o);
            } catch (const tc::Error &e) {
                if (e.code != TC_ERR_OUT_OF_MEMORY) throw;
                g->o = tc::Oriented();
                psrc.release();
                pdst.release();
                g->part.reset(new tc::Partitioned());
                tc::build_partitioned(graphs[0].src, graphs[0].dst, o.inputs_on_device != 0, pk, bp, 0, g->al, s,
                                      *g->part);
            }
        } else {
            tc::build_oriented_device(dsrc, ddst, pk, bp, g->al, s, g->o);
        }
        // canonical rows of one graph never exceed its input edges
        g->max_graph_m = g->o.M;
        if (k > 1) {
            g->max_graph_m = 0;
            for (int32_t i = 0; i < k; ++i) g->max_graph_m = std::max<int64_t>(g->max_graph_m, graphs[i].m);
            g->max_graph_m = std::min<int64_t>(g->max_graph_m, g->o.M);
        }
    });
    if (st != TC_OK) return st;
    *out = g.release();
    return TC_OK;
}

tc_status tc_graph_reschedule(tc_graph *g, const tc_options *opt) {
    if (!g) return fail(TC_ERR_INVALID_ARG, "graph must be non-NULL");
    return guarded([&] {
        check_options(opt);
        tc_options o;
        if (opt)
            o = *opt;
        else
            tc_options_default(&o);
        hipStream_t s = (hipStream_t)o.stream;
        g->al.stream = s;
        const int cus = tc::device_cu_count();
        tc::BuildParams bp;
        bp.workers = o.workers > 0 ? o.workers : tc::small_kernel_waves_per_cu(true) * cus;
        bp.cost_fn = o.cost_fn;
        bp.min_chunk = o.min_chunk;
        bp.rounds = o.rounds;
        bp.static_chunks = o.static_chunks;
        bp.small_max = o.small_max > 0 ? std::min(o.small_max, tc::max_small_list()) : tc::max_small_list();
        // a partitioned handle builds its task tables at count time
        if (!g->part) tc::reschedule_device(g->pk, bp, g->al, s, g->o);
        g->min_chunk = bp.min_chunk;
        g->rounds = bp.rounds;
        g->static_chunks = bp.static_chunks;
        g->workers = bp.workers;
        g->small_max = bp.small_max;
        g->cost_fn = bp.cost_fn;
        g->search = resolve_search(o.intersect, o.search_ratio);
        g->hash = o.hash;
        g->bitmap = resolve_bitmap(o.intersect, o.bitmap_ratio);
        g->lds_max = o.lds_list_max > 0 ? std::max(2, std::min(o.lds_list_max, tc::max_lds_list())) : tc::max_lds_list();
        // the per-handle count descriptor caches the wide list and small_max
        g->desc.release();
        g->desc_has_tv = false;
    });
}

static tc_status count_one(tc_graph *g, const tc_options *opt, int64_t *per_node, int64_t *totals) {
    return guarded([&] {
        check_options(opt);
        const bool on_dev = opt && opt->outputs_on_device;
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        const bool want_tv = per_node != nullptr;
        const int32_t search = count_search(g, opt);
        ensure_scratch(g, want_tv, search, count_bitmap(g, opt), s);
        const size_t k = (size_t)g->pk.k;
        const bool timing = opt && opt->time_kernels;
        if (timing) {
            for (hipEvent_t &e : g->ev)
                if (!e) TC_HIP(hipEventCreate(&e));
        }
        if (g->part) {
            tc::BuildParams bp;
            bp.workers = opt && opt->workers > 0 ? opt->workers : g->workers;
            bp.cost_fn = g->cost_fn;
            bp.min_chunk = g->min_chunk;
            bp.small_max = g->small_max;
            bp.rounds = g->rounds > 0 ? g->rounds : 1;
            bp.static_chunks = g->static_chunks;
            const int32_t lds = opt && opt->lds_list_max > 0 ? opt->lds_list_max : g->lds_max;
            if (timing) TC_HIP(hipEventRecord(g->ev[0], s));
            tc::count_partitioned(*g->part, bp, lds, search, count_rounds(g, opt), g->al, s, g->totals.p, want_tv ? g->tv.p : nullptr,
                                  g->heads.p);
            if (timing) {
                TC_HIP(hipEventRecord(g->ev[1], s));
                g->timed = true;
            }
        } else {
            {
                const int64_t n = want_tv ? g->pk.N : 0;
                const int64_t words = std::max<int64_t>({n, (int64_t)k, 4});
                const unsigned blocks = (unsigned)std::min<int64_t>((words + 1023) / 1024, 2048);
                k_count_reset<<<blocks, 256, 0, s>>>(g->heads.p, g->totals.p, k, want_tv ? g->tv.p : nullptr, n);
                TC_LAUNCH_CHECK();
            }
            tc::CountLaunch L{};
            L.descs = g->desc.p;
            L.ndesc = 1;
            L.total_tasks = g->o.tasks;
            L.total_med = g->o.nmed;
            L.total_large = g->o.nbig - g->o.nmed;
            L.max_m = g->max_graph_m;
            L.heads = g->heads.p;
            L.workers = opt && opt->workers > 0 ? opt->workers : g->workers;
            L.lds_max = opt && opt->lds_list_max > 0 ? opt->lds_list_max : g->lds_max;
            L.cuckoo_rounds = count_rounds(g, opt);
            L.per_node = want_tv;
            L.core = g->o.bm.p && count_bitmap(g, opt) > 0;
            g->times_used = 0;
            if (opt && opt->time_kernels == 2) {
                const int64_t cap = tc::max_timed_workers();
                if (!g->times.p) g->times = tc::DevBuf<unsigned long long>(g->al, (size_t)(2 * cap));
                tc::fill_zero(g->times.p, g->times.bytes(), s);
                L.times = g->times.p;
                L.times_cap = cap;
            }
            if (timing) TC_HIP(hipEventRecord(g->ev[0], s));
            tc::count_launch(L, s);
            g->times_used = L.times_used;
            for (int t = 0; t < 3; ++t) g->times_tier[t] = L.times_tier[t];
            if (timing) {
                TC_HIP(hipEventRecord(g->ev[1], s));
                g->timed = true;
            }
        }
        const int32_t *perm = g->part ? g->part->perm.p : g->o.perm.p;
        if (want_tv) {
            if (on_dev) {
                tc::scatter_per_node(g->tv.p, perm, g->pk.N, per_node, s);
            } else {
                tc::DevBuf<int64_t> stage(g->al, (size_t)std::max<int64_t>(g->pk.N, 1));
                tc::scatter_per_node(g->tv.p, perm, g->pk.N, stage.p, s);
                copy_out(per_node, stage.p, (size_t)g->pk.N * sizeof(int64_t), false, s);
                TC_HIP(hipStreamSynchronize(s));
            }
        }
        if (totals) copy_out(totals, g->totals.p, k * sizeof(int64_t), on_dev, s);
        if (!on_dev) TC_HIP(hipStreamSynchronize(s));
    });
}

tc_status tc_count_total(tc_graph *g, const tc_options *opt, int64_t *totals) {
    if (!g || !totals) return fail(TC_ERR_INVALID_ARG, "graph and totals must be non-NULL");
    return count_one(g, opt, nullptr, totals);
}

tc_status tc_count_per_node(tc_graph *g, const tc_options *opt, int64_t *per_node, int64_t *totals) {
    if (!g || (!per_node && g->pk.N > 0)) return fail(TC_ERR_INVALID_ARG, "graph and per_node must be non-NULL");
    if (g->pk.N == 0) return count_one(g, opt, nullptr, totals ? totals : nullptr);
    return count_one(g, opt, per_node, totals);
}

tc_status tc_count_batch(tc_graph *const *gs, int32_t ng, const tc_options *opt, int64_t *totals,
                         int64_t *const *per_node) {
    const tc_status bad = check_batch_args(gs, ng, totals);
    if (bad != TC_OK) return bad;
    return guarded([&] {
        check_options(opt);
        const bool on_dev = opt && opt->outputs_on_device;
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        tc::Allocator al = make_allocator(opt);
        al.budget = 0;
        const BatchLayout lay = batch_layout(gs, ng, per_node);
        tc::DevBuf<uint8_t> buf(al, lay.bytes);
        launch_batch(gs, ng, opt, lay, buf.p, false, s);
        const int64_t *tot = (const int64_t *)(buf.p + lay.tot_off);
        const int64_t *tv = (const int64_t *)(buf.p + lay.tv_off);
        for (int32_t i = 0; i < ng && per_node; ++i) {
            if (!per_node[i] || gs[i]->pk.N == 0) continue;
            const int64_t n = gs[i]->pk.N;
            if (on_dev) {
                tc::scatter_per_node(tv + lay.nbase[i], gs[i]->o.perm.p, n, per_node[i], s);
            } else {
                tc::DevBuf<int64_t> stage(al, (size_t)n);
                tc::scatter_per_node(tv + lay.nbase[i], gs[i]->o.perm.p, n, stage.p, s);
                copy_out(per_node[i], stage.p, (size_t)n * 8, false, s);
                TC_HIP(hipStreamSynchronize(s));
            }
        }
        copy_out(totals, tot, (size_t)lay.kbase[ng] * 8, on_dev, s);
        if (!on_dev) TC_HIP(hipStreamSynchronize(s));
        // device descriptors and scratch are released in stream order here
    });
}

tc_status tc_count_batch_static(tc_graph *const *gs, int32_t ng, const tc_options *opt, int64_t *totals,
                                int64_t *const *per_node) {
    const tc_status bad = check_batch_args(gs, ng, totals);
    if (bad != TC_OK) return bad;
    if (!opt || !opt->outputs_on_device)
        return fail(TC_ERR_INVALID_ARG, "tc_count_batch_static writes device outputs only (outputs_on_device = 1)");
    return guarded([&] {
        check_options(opt);
        hipStream_t s = (hipStream_t)opt->stream;
        const BatchLayout lay = batch_layout(gs, ng, per_node);
        if (lay.bytes > kStaticScratchBytes)
            throw tc::Error(TC_ERR_TOO_LARGE, "batch needs " + std::to_string(lay.bytes) +
                                                  " bytes of scratch; the static array holds " +
                                                  std::to_string(kStaticScratchBytes));
        int dev = 0;
        TC_HIP(hipGetDevice(&dev));
        uint8_t *base = (uint8_t *)static_scratch(dev);
        launch_batch(gs, ng, opt, lay, base, true, s);
        write_device_outputs(gs, ng, lay, base, totals, per_node, s);
    });
}

tc_status tc_count_capture(tc_graph *const *gs, int32_t ng, const tc_options *opt, int64_t *totals,
                           int64_t *const *per_node, tc_count_graph **out) {
    const tc_status bad = check_batch_args(gs, ng, totals);
    if (bad != TC_OK) return bad;
    if (!out) return fail(TC_ERR_INVALID_ARG, "out must be non-NULL");
    if (!opt || !opt->outputs_on_device)
        return fail(TC_ERR_INVALID_ARG, "a captured count writes device outputs only (outputs_on_device = 1)");
    std::unique_ptr<tc_count_graph> c(new (std::nothrow) tc_count_graph());
    if (!c) return fail(TC_ERR_OUT_OF_MEMORY, "host allocation failed");
    const tc_status st = guarded([&] {
        check_options(opt);
        hipStream_t s = (hipStream_t)opt->stream;
        c->al = make_allocator(opt);
        c->al.budget = 0;
        c->last = s;
        const BatchLayout lay = batch_layout(gs, ng, per_node);
        c->scratch = tc::DevBuf<uint8_t>(c->al, lay.bytes);
        // the scratch must exist before any replay, on whatever stream
        TC_HIP(hipStreamSynchronize(s));
        hipStream_t cs = nullptr;
        TC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        struct StreamGuard {
            hipStream_t s;
            ~StreamGuard() { (void)hipStreamDestroy(s); }
        } guard{cs};
        TC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            launch_batch(gs, ng, opt, lay, c->scratch.p, true, cs);
            write_device_outputs(gs, ng, lay, c->scratch.p, totals, per_node, cs);
        } catch (...) {
            hipGraph_t partial = nullptr;
            (void)hipStreamEndCapture(cs, &partial);
            if (partial) (void)hipGraphDestroy(partial);
            (void)hipGetLastError();
            throw;
        }
        TC_HIP(hipStreamEndCapture(cs, &c->graph));
        TC_HIP(hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
    });
    if (st != TC_OK) return st;
    *out = c.release();
    return TC_OK;
}

tc_status tc_count_replay(tc_count_graph *c, const tc_options *opt) {
    if (!c || !c->exec) return fail(TC_ERR_INVALID_ARG, "captured count must be non-NULL");
    return guarded([&] {
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        TC_HIP(hipGraphLaunch(c->exec, s));
        c->last = s;
        c->al.stream = s;
    });
}

void tc_count_graph_free(tc_count_graph *c) {
    if (!c) return;
    // the last replay may still read the scratch
    if (c->exec) (void)hipStreamSynchronize(c->last);
    delete c;
}

tc_status tc_graph_info(const tc_graph *g, tc_graph_info_t *info) {
    if (!g || !info) return fail(TC_ERR_INVALID_ARG, "graph and info must be non-NULL");
    std::memset(info, 0, sizeof(*info));
    info->k = g->pk.k;
    info->n = g->pk.N;
    info->m = g->part ? g->part->M : g->o.M;
    info->m_input = g->pk.M_in;
    info->max_out_degree = g->part ? g->part->max_dhat : g->o.max_dhat;
    info->tasks = g->o.tasks;
    info->total_cost = g->o.total_cost;
    info->wide_nodes = g->o.nbig;
    info->device_bytes = g->al.live;
    info->peak_device_bytes = g->al.peak;
    info->partitions = g->part ? g->part->P : 1;
    info->rounds = g->part ? (g->rounds > 0 ? g->rounds : 1) : g->o.rounds;
    info->streamed_bytes = g->part ? g->part->streamed_bytes : 0;
    info->workers = g->workers;
    info->small_max = g->small_max;
    info->cost_fn = g->cost_fn;
    info->search_ratio = g->search;
    info->hash = g->hash;
    info->bitmap_ratio = g->o.bm.p ? g->bitmap : 0;
    info->core_rows = g->o.bm.p ? g->pk.N - g->o.core.lo : 0;
    info->core_bytes = (uint64_t)g->o.core.words * 4;
    info->last_count_ms = -1.0;
    if (g->timed) {
        float ms = 0.f;
        if (hipEventSynchronize(g->ev[1]) == hipSuccess && hipEventElapsedTime(&ms, g->ev[0], g->ev[1]) == hipSuccess)
            info->last_count_ms = ms;
    }
    return TC_OK;
}

tc_status tc_export_csr(const tc_graph *g, const tc_options *opt, int64_t *off, int32_t *col, int32_t *perm) {
    if (!g) return fail(TC_ERR_INVALID_ARG, "graph must be non-NULL");
    return guarded([&] {
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        if (g->part) {
            // the adjacency is in host memory already
            if (off) std::memcpy(off, g->part->off.p, (size_t)(g->pk.N + 1) * 8);
            if (col && g->part->M) std::memcpy(col, g->part->col.p, (size_t)g->part->M * 4);
            if (perm && g->pk.N) copy_out(perm, g->part->perm.p, (size_t)g->pk.N * 4, false, s);
            TC_HIP(hipStreamSynchronize(s));
            return;
        }
        if (off) copy_out(off, g->o.off.p, (size_t)(g->pk.N + 1) * 8, false, s);
        if (col && g->o.M) copy_out(col, g->o.col.p, (size_t)g->o.M * 4, false, s);
        if (perm && g->pk.N) copy_out(perm, g->o.perm.p, (size_t)g->pk.N * 4, false, s);
        TC_HIP(hipStreamSynchronize(s));
    });
}

tc_status tc_export_schedule(const tc_graph *g, const tc_options *opt, int32_t *bnd, int32_t *gid, int64_t cap,
                             int64_t *tasks) {
    if (!g || !tasks) return fail(TC_ERR_INVALID_ARG, "graph and tasks must be non-NULL");
    if (g->part) return fail(TC_ERR_INVALID_ARG, "a partitioned handle builds one task table per streamed batch");
    *tasks = g->o.tasks;
    if (!bnd) return TC_OK;
    if (cap < g->o.tasks + 1) return fail(TC_ERR_INVALID_ARG, "bnd capacity below tasks + 1");
    return guarded([&] {
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        copy_out(bnd, g->o.bnd.p, (size_t)(g->o.tasks + 1) * 4, false, s);
        if (gid && g->pk.k > 1) copy_out(gid, g->o.gid.p, (size_t)g->o.tasks * 4, false, s);
        if (gid && g->pk.k == 1) std::fill(gid, gid + g->o.tasks, 0);
        TC_HIP(hipStreamSynchronize(s));
    });
}

tc_status tc_clustering(tc_graph *g, const tc_options *opt, double *coeff, double *transitivity, int64_t *totals) {
    if (!g) return fail(TC_ERR_INVALID_ARG, "graph must be non-NULL");
    if (g->part) return fail(TC_ERR_INVALID_ARG, "clustering needs a resident handle");
    const int64_t N = g->pk.N;
    const int k = g->pk.k;
    return guarded([&] {
        check_options(opt);
        const bool on_dev = opt && opt->outputs_on_device;
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        // per-node counts into the handle's accumulators (degree-order labels)
        tc::DevBuf<int64_t> caller_tv(g->al, (size_t)std::max<int64_t>(N, 1));
        tc_options o;
        if (opt)
            o = *opt;
        else
            tc_options_default(&o);
        o.outputs_on_device = 1;
        const tc_status st = N > 0 ? count_one(g, &o, caller_tv.p, nullptr) : count_one(g, &o, nullptr, nullptr);
        if (st != TC_OK) throw tc::Error(st, g_last_error);
        tc::DevBuf<unsigned long long> wedges(g->al, (size_t)std::max(k, 1));
        tc::DevBuf<double> dcoeff, dtrans;
        double *c = coeff, *t = transitivity;
        if (!on_dev) {
            if (coeff && N > 0) dcoeff = tc::DevBuf<double>(g->al, (size_t)N);
            if (transitivity) dtrans = tc::DevBuf<double>(g->al, (size_t)k);
            c = coeff ? dcoeff.p : nullptr;
            t = transitivity ? dtrans.p : nullptr;
        }
        if (N > 0 || t)
            tc::clustering_epilogue(g->tv.p, g->o.deg.p, g->o.perm.p, N, g->o.node_base.p, k, g->totals.p,
                                    N > 0 ? c : nullptr, t, wedges.p, s);
        if (!on_dev) {
            if (coeff && N > 0) copy_out(coeff, dcoeff.p, (size_t)N * 8, false, s);
            if (transitivity) copy_out(transitivity, dtrans.p, (size_t)k * 8, false, s);
        }
        if (totals) copy_out(totals, g->totals.p, (size_t)k * 8, on_dev, s);
        if (!on_dev) TC_HIP(hipStreamSynchronize(s));
    });
}

tc_status tc_worker_times(const tc_graph *g, const tc_options *opt, int64_t *times, int64_t cap,
                          int64_t *nworkers) {
    if (!g || !nworkers) return fail(TC_ERR_INVALID_ARG, "graph and nworkers must be non-NULL");
    *nworkers = g->times_used;
    if (!times || g->times_used == 0) return TC_OK;
    if (cap < g->times_used) return fail(TC_ERR_INVALID_ARG, "times capacity below the number of workers");
    return guarded([&] {
        hipStream_t s = opt ? (hipStream_t)opt->stream : nullptr;
        std::vector<unsigned long long> h((size_t)(2 * g->times_used));
        TC_HIP(hipMemcpyAsync(h.data(), g->times.p, h.size() * 8, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        int dev = 0, khz = 0;
        TC_HIP(hipGetDevice(&dev));
        TC_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        if (khz <= 0) throw tc::Error(TC_ERR_DEVICE, "no wall-clock rate");
        unsigned long long t0 = ~0ull;
        for (size_t i = 0; i < h.size(); i += 2)
            if (h[i]) t0 = std::min(t0, h[i]);
        int64_t w = 0;
        for (int t = 0; t < 3; ++t)
            for (int64_t i = 0; i < g->times_tier[t]; ++i, ++w)
                for (int c = 0; c < 2; ++c) {
                    const unsigned long long v = h[2 * w + c];
                    times[3 * w + c] = v ? (int64_t)((double)(v - t0) * 1e6 / (double)khz) : -1;
                    times[3 * w + 2] = t;
                }
    });
}

void tc_graph_free(tc_graph *g) {
    if (!g) return;
    // Without callbacks the buffers go back in order on the last stream the
    // handle used.  A caller's allocator may hand them to another stream at
    // once, so wait for the handle's work first.
    if (g->al.fn_free) (void)hipStreamSynchronize(g->al.stream);
    delete g;
}

}  // extern "C"
