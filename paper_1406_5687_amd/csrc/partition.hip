// Partitioned mode: counting a graph whose resident form would not fit the
// device budget, in consecutive node ranges of the degree order (Definition 1)
// with the surrogate scheme of Section IV (Fig. 2 / Fig. 3).
//
// Slices.  The oriented adjacency (rows N_v in degree-order labels, sorted)
// lives in page-locked host memory.  The labels are cut into P consecutive
// ranges V_j = [lo_j, hi_j) whose rows fit on the device next to the count's
// working set.
//
// Count of slice j.  The rows N_u, u in V_j, are copied in.  Every node v
// whose list has an entry in V_j contributes one record: the part of N_v from
// its first entry >= lo_j on.  Because N_v is sorted, that part is one
// contiguous range, and it is streamed once per slice however many of its
// entries lie in V_j (the role of LastProc in Fig. 3).  Its entries inside V_j
// are the targets u; for each, |N_v intersect N_u| is found against the
// resident N_u (SurrogateCount).  Entries of N_v below lo_j are never needed:
// N_u holds only labels above u >= lo_j.  Every oriented edge (v, u) is
// counted once, in the slice of u, so the result equals the resident count
// (Theorem 1).
//
// Build under the budget (every device allocation counts):
//   A. canonical edge set in buckets of the smaller endpoint: one pass counts
//      input edges per node to place bucket bounds; per bucket, the edges are
//      gathered, radix sorted and deduplicated on the device and copied to
//      host memory; degrees accumulate on the device;
//   B. degree order: one device sort of (d_v, v) over all nodes;
//   C. out-degrees in the degree order, offsets (copied to the host), slice
//      bounds by bytes;
//   D. per slice: its oriented pairs are sorted into rows and copied to the
//      host, and the records it sends to every later-or-equal slice are
//      written out in node order.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int per_thread = 1) {
    int64_t b = ceil_div(n, (int64_t)kThreads * per_thread);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)1 << 30));
}

template <class T>
void d2h(T *host, const T *dev, size_t count, hipStream_t s) {
    if (count) TC_HIP(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, s));
}

template <class T>
void h2d(T *dev, const T *host, size_t count, hipStream_t s) {
    if (count) TC_HIP(hipMemcpyAsync(dev, host, count * sizeof(T), hipMemcpyHostToDevice, s));
}

// ------------------------------------------------------------ A. canonical set

// Input edges per smaller endpoint (loops skipped); err bit 0: id out of range.
__global__ void k_min_hist(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m, int32_t n,
                           int32_t *__restrict__ cnt, uint32_t *__restrict__ err) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[e], v = dst[e];
        if (u < 0 || v < 0 || u >= n || v >= n) {
            atomicOr(err, 1u);
        } else if (u != v) {
            atomicAdd(&cnt[u < v ? u : v], 1);
        }
    }
}

// Appends the key (a << gb) | b of every edge {a < b} with lo <= a < hi
// (ids already checked).  One atomic per wave.
__global__ void k_bucket_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m,
                              int32_t lo, int32_t hi, int gb, uint64_t *__restrict__ keys,
                              unsigned long long *__restrict__ count, int64_t cap) {
    const int lane = __lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < m; b0 += stride) {
        const int64_t e = b0 + threadIdx.x;
        int32_t a = 0, b = 0;
        if (e < m) {
            const int32_t u = src[e], v = dst[e];
            a = u < v ? u : v;
            b = u < v ? v : u;
        }
        const bool take = e < m && a != b && a >= lo && a < hi;
        const uint64_t mask = __ballot(take);
        if (!mask) continue;
        const int leader = __ffsll((unsigned long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(count, (unsigned long long)popc64(mask));
        base = (unsigned long long)readlane64((int64_t)base, leader);
        const int64_t at = (int64_t)base + popc64(mask & lanemask_lt());
        if (take && at < cap) keys[at] = ((uint64_t)a << gb) | (uint64_t)b;
    }
}

__global__ void k_max_i32(const int32_t *__restrict__ x, int64_t n, int32_t *__restrict__ out) {
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, x[i]);
    m = wave_reduce_max(m);
    if (__lane_id() == 0) atomicMax(out, m);
}

// --------------------------------------------------------- C. out-degrees

// Edge {a, b} is stored at the lower of its two degree-order labels.
__global__ void k_out_degrees(const uint64_t *__restrict__ ukeys, int64_t m, int gb, const int32_t *__restrict__ rank,
                              int32_t *__restrict__ dh) {
    const uint64_t mask = (1ull << gb) - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = ukeys[e];
        const int32_t ra = rank[k >> gb], rb = rank[k & mask];
        atomicAdd(&dh[ra < rb ? ra : rb], 1);
    }
}

// Slice bounds by bytes: cut[j] = first x with w(x) >= target[j - 1], where
// w(x) = eb * off[x] + nb * x is the device footprint of rows [0, x).
__global__ void k_slice_bounds(const int64_t *__restrict__ off, int64_t N, int64_t eb, int64_t nb,
                               const int64_t *__restrict__ target, int64_t nt, int64_t *__restrict__ cut) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nt; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tg = target[j];
        int64_t lo = 0, hi = N;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (eb * off[mid] + nb * mid >= tg)
                hi = mid;
            else
                lo = mid + 1;
        }
        cut[j] = lo;
    }
}

// ------------------------------------------------------ D. rows of a slice

// Oriented pair (s, t) of every edge with lo <= s < hi, as ((s - lo) << gb) | t.
__global__ void k_slice_keys(const uint64_t *__restrict__ ukeys, int64_t m, int gb, const int32_t *__restrict__ rank,
                             int32_t lo, int32_t hi, uint64_t *__restrict__ keys,
                             unsigned long long *__restrict__ count, int64_t cap) {
    const uint64_t mask = (1ull << gb) - 1;
    const int lane = __lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < m; b0 += stride) {
        const int64_t e = b0 + threadIdx.x;
        int32_t sv = -1, tv = 0;
        if (e < m) {
            const uint64_t k = ukeys[e];
            const int32_t ra = rank[k >> gb], rb = rank[k & mask];
            sv = ra < rb ? ra : rb;
            tv = ra < rb ? rb : ra;
        }
        const bool take = sv >= lo && sv < hi;
        const uint64_t bal = __ballot(take);
        if (!bal) continue;
        const int leader = __ffsll((unsigned long long)bal) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(count, (unsigned long long)popc64(bal));
        base = (unsigned long long)readlane64((int64_t)base, leader);
        const int64_t at = (int64_t)base + popc64(bal & lanemask_lt());
        if (take && at < cap) keys[at] = ((uint64_t)(sv - lo) << gb) | (uint64_t)tv;
    }
}

__global__ void k_low_bits(const uint64_t *__restrict__ keys, int64_t n, int gb, int32_t *__restrict__ col) {
    const uint64_t mask = (1ull << gb) - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        col[i] = (int32_t)(keys[i] & mask);
}

__device__ __forceinline__ int64_t lower_bound_i32(const int32_t *a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// For each row r of the slice [lo_i, lo_i + rows): the part of N_r inside
// [lo_j, hi_j) is one run of the sorted row; flag it and note its start and
// length.  off is the global offset array, col the slice's entries from ebase.
__global__ void k_run_of_slice(const int64_t *__restrict__ off, const int32_t *__restrict__ col, int64_t ebase,
                               int32_t lo_i, int64_t rows, int32_t lo_j, int32_t hi_j, uint32_t *__restrict__ flag,
                               int32_t *__restrict__ first, int32_t *__restrict__ cnt) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < rows; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e0 = off[lo_i + x] - ebase, e1 = off[lo_i + x + 1] - ebase;
        const int64_t p = lower_bound_i32(col, e0, e1, lo_j);
        const int64_t q = lower_bound_i32(col, p, e1, hi_j);
        flag[x] = q > p ? 1u : 0u;
        first[x] = (int32_t)(p - e0);
        cnt[x] = (int32_t)(q - p);
    }
}

__global__ void k_write_records(const int64_t *__restrict__ off, const uint32_t *__restrict__ flag,
                                const int64_t *__restrict__ at, const int32_t *__restrict__ first,
                                const int32_t *__restrict__ cnt, int32_t lo_i, int64_t rows,
                                int32_t *__restrict__ rv, int64_t *__restrict__ rpos, int32_t *__restrict__ rtc,
                                int32_t *__restrict__ rlen) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < rows; x += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[x]) continue;
        const int64_t o = at[x];
        const int64_t start = off[lo_i + x] + first[x];
        rv[o] = lo_i + (int32_t)x;
        rpos[o] = start;
        rtc[o] = cnt[x];
        rlen[o] = (int32_t)(off[lo_i + x + 1] - start);
    }
}

// ------------------------------------------------------------ count of a slice

__global__ void k_rebase(int64_t *__restrict__ off, int64_t n, int64_t base) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        off[i] -= base;
}

// Streams the records' ranges of the host adjacency into one device list
// array: one wave per record, 64 consecutive ids per load.
__global__ void k_gather_ranges(const int32_t *__restrict__ hcol, const int64_t *__restrict__ rpos,
                                const int64_t *__restrict__ moff, int64_t nrec, int32_t *__restrict__ mcol) {
    const int lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < nrec; r += nwaves) {
        const int64_t src = rpos[r], dst = moff[r];
        const int64_t len = moff[r + 1] - dst;
        for (int64_t x = lane; x < len; x += 64) mcol[dst + x] = hcol[src + x];
    }
}

// Cost of each streamed source for the task table: the ids its target rows
// hold plus the list length per target (the prior cost of Section IV-B
// restricted to the resident targets); lists longer than small_max go to
// whole workgroups instead.
__global__ void k_slice_costs(const int64_t *__restrict__ moff, const int32_t *__restrict__ mcol,
                              const int32_t *__restrict__ rtc, int64_t nrec, const int64_t *__restrict__ off,
                              int32_t lo, int small_max, int med_max, int64_t *__restrict__ f,
                              uint32_t *__restrict__ wmed, uint32_t *__restrict__ wlarge) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrec; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r0 = moff[i];
        const int32_t a = (int32_t)(moff[i + 1] - r0);
        const int32_t te = min(rtc[i], a - 1);
        int64_t c = 0;
        const bool wide = a > small_max;
        if (!wide && te > 0) {
            for (int32_t x = 0; x < te; ++x) {
                const int32_t u = mcol[r0 + x] - lo;
                c += (int64_t)a + (off[u + 1] - off[u]);
            }
        }
        f[i] = c;
        wmed[i] = (wide && te > 0 && a <= med_max) ? 1u : 0u;
        wlarge[i] = (wide && te > 0 && a > med_max) ? 1u : 0u;
    }
}

// ------------------------------------------------------------ budget plan

constexpr size_t kSlack = (size_t)16 << 20;  // sort/scan tables of small arrays, descriptors

struct Plan {
    uint64_t B = 0;           // effective budget
    int64_t in_chunk = 0;     // input edges staged per copy (host inputs)
    int64_t u_chunk = 0;      // canonical edges staged per copy
};

uint64_t headroom(const Allocator &al, uint64_t B) { return al.live >= B ? 0 : B - al.live; }

}  // namespace

void build_partitioned(const int32_t *src, const int32_t *dst, bool on_device, const Packing &pk,
                       const BuildParams &bp, int32_t partitions, Allocator &al, hipStream_t s, Partitioned &out) {
    if (pk.k != 1) throw Error(TC_ERR_INVALID_ARG, "partitioned mode counts one graph per handle");
    const int64_t N = pk.N, M_in = pk.M_in;
    const uint64_t B = al.budget ? al.budget : ((uint64_t)1 << 62);
    const int gb = std::max(1, bits_for((uint64_t)std::max<int64_t>(N - 1, 1)));
    out.N = N;
    Plan pl;
    pl.B = B;
    // node arrays: degrees, order keys and sort tables in B (< 29 B / node);
    // later perm, rank and off (16 B / node) next to a slice
    const uint64_t node_need = (uint64_t)N * 29 + kSlack * 2;
    if (node_need > B)
        throw Error(TC_ERR_OUT_OF_MEMORY, "device budget " + std::to_string(B) + " bytes is below the " +
                                              std::to_string(node_need) + " bytes the node arrays of n = " +
                                              std::to_string(N) + " need");
    pl.in_chunk = on_device ? 0 : std::max<int64_t>(1 << 16, std::min<int64_t>((int64_t)(B / 64 / 8), 1 << 25));
    pl.u_chunk = std::max<int64_t>(1 << 16, std::min<int64_t>((int64_t)(B / 64 / 8), 1 << 25));

    DevBuf<int64_t> nb_dev(al, 2);
    {
        const int64_t nbh[2] = {0, N};
        h2d(nb_dev.p, nbh, 2, s);
    }
    DevBuf<uint32_t> err(al, 4);
    fill_zero(err.p, 16, s);

    // staging of host input chunks
    DevBuf<int32_t> sin_src, sin_dst;
    if (!on_device && M_in > 0) {
        sin_src = DevBuf<int32_t>(al, (size_t)std::min(M_in, pl.in_chunk));
        sin_dst = DevBuf<int32_t>(al, (size_t)std::min(M_in, pl.in_chunk));
    }
    // calls fn(src_chunk, dst_chunk, len) for consecutive chunks of the input
    auto for_input_chunks = [&](auto &&fn) {
        if (on_device) {
            if (M_in > 0) fn(src, dst, M_in);
            return;
        }
        for (int64_t e0 = 0; e0 < M_in; e0 += pl.in_chunk) {
            const int64_t len = std::min(pl.in_chunk, M_in - e0);
            h2d(sin_src.p, src + e0, (size_t)len, s);
            h2d(sin_dst.p, dst + e0, (size_t)len, s);
            fn((const int32_t *)sin_src.p, (const int32_t *)sin_dst.p, len);
        }
    };

    // ---- A. canonical edge set, bucketed by the smaller endpoint
    DevBuf<int32_t> deg(al, (size_t)std::max<int64_t>(N, 1));
    fill_zero(deg.p, deg.bytes(), s);
    std::vector<int64_t> bcut;  // bucket bounds (node ids)
    std::vector<int64_t> braw;  // input edges (loops excluded) per bucket
    int64_t raw_total = 0;
    {
        DevBuf<int32_t> cnt(al, (size_t)std::max<int64_t>(N, 1));
        fill_zero(cnt.p, cnt.bytes(), s);
        for_input_chunks([&](const int32_t *cs, const int32_t *cd, int64_t len) {
            k_min_hist<<<grid_for(len, 4), kThreads, 0, s>>>(cs, cd, len, (int32_t)N, cnt.p, err.p);
            TC_LAUNCH_CHECK();
        });
        uint32_t herr = 0;
        d2h(&herr, err.p, 1, s);
        TC_HIP(hipStreamSynchronize(s));
        if (herr & 1u) throw Error(TC_ERR_ID_RANGE, "an edge endpoint is outside 0..n-1");
        DevBuf<int32_t> mx(al, 1);
        fill_zero(mx.p, 4, s);
        if (N > 0) {
            k_max_i32<<<grid_for(N, 8), kThreads, 0, s>>>(cnt.p, N, mx.p);
            TC_LAUNCH_CHECK();
        }
        DevBuf<int64_t> H(al, (size_t)N + 1);
        exclusive_scan(cnt.p, H.p, N, true, al, s);
        int32_t maxcnt = 0;
        d2h(&raw_total, H.p + N, 1, s);
        d2h(&maxcnt, mx.p, 1, s);
        TC_HIP(hipStreamSynchronize(s));
        cnt.release();
        // per bucket: two key buffers, sort tables, unique partials (< 18 B / edge)
        const uint64_t room = headroom(al, B);
        const int64_t cap = room > kSlack * 2 ? (int64_t)((room - kSlack * 2) / 18) : 0;
        if (raw_total > 0 && cap <= (int64_t)maxcnt + 1)
            throw Error(TC_ERR_OUT_OF_MEMORY, "device budget too small for the edges of one node");
        const int64_t nbk = raw_total > 0 ? std::max<int64_t>(1, ceil_div(raw_total, cap - maxcnt)) : 1;
        std::vector<int64_t> tg;
        for (int64_t j = 1; j < nbk; ++j) tg.push_back(ceil_div(j * raw_total, nbk));
        tg.push_back(-1);
        DevBuf<int32_t> bb(al, tg.size() + 1);
        task_bounds(H.p, N, tg, bb.p, al, s);
        std::vector<int32_t> hb(tg.size() + 1);
        d2h(hb.data(), bb.p, hb.size(), s);
        TC_HIP(hipStreamSynchronize(s));
        bcut.assign(hb.begin(), hb.end());
        std::vector<int64_t> hH(bcut.size());
        for (size_t b = 0; b < bcut.size(); ++b) d2h(&hH[b], H.p + bcut[b], 1, s);
        TC_HIP(hipStreamSynchronize(s));
        for (size_t b = 0; b + 1 < bcut.size(); ++b) braw.push_back(hH[b + 1] - hH[b]);
    }
    HostBuf<uint64_t> U((size_t)std::max<int64_t>(raw_total, 1));
    int64_t M = 0;
    {
        DevBuf<unsigned long long> counter(al, 1);
        for (size_t b = 0; b + 1 < bcut.size(); ++b) {
            const int32_t lo = (int32_t)bcut[b], hi = (int32_t)bcut[b + 1];
            const int64_t nraw = braw[b];  // from the histogram pass
            if (lo >= hi || nraw == 0) continue;
            DevBuf<uint64_t> ka(al, (size_t)nraw), kb(al, (size_t)nraw);
            fill_zero(counter.p, 8, s);
            for_input_chunks([&](const int32_t *cs, const int32_t *cd, int64_t len) {
                k_bucket_keys<<<grid_for(len, 4), kThreads, 0, s>>>(cs, cd, len, lo, hi, gb, ka.p, counter.p, nraw);
                TC_LAUNCH_CHECK();
            });
            unsigned long long got = 0;
            d2h(&got, counter.p, 1, s);
            TC_HIP(hipStreamSynchronize(s));
            if ((int64_t)got != nraw) throw Error(TC_ERR_DEVICE, "bucket edge count disagrees with the histogram");
            uint64_t *sorted = radix_sort_u64(ka.p, kb.p, (int64_t)nraw, 0, 2 * gb, al, s);
            uint64_t *other = sorted == ka.p ? kb.p : ka.p;
            uint64_t *uk = nullptr;
            const int64_t mb = unique_sorted_keys(sorted, (int64_t)nraw, other, &uk, al, s);
            uint64_t *spare = uk == sorted ? other : sorted;
            add_degrees(uk, mb, gb, deg.p, N, reinterpret_cast<uint32_t *>(spare), al, s);
            d2h(U.p + M, uk, (size_t)mb, s);
            TC_HIP(hipStreamSynchronize(s));
            M += mb;
        }
    }
    sin_src.release();
    sin_dst.release();
    out.M = M;

    // ---- B. degree order
    out.perm = DevBuf<int32_t>(al, (size_t)std::max<int64_t>(N, 1));
    DevBuf<int32_t> rank(al, (size_t)std::max<int64_t>(N, 1));
    degree_rank(deg.p, N, nb_dev.p, 1, (int32_t)N, out.perm.p, rank.p, al, s);
    deg.release();

    // canonical edges come back from host memory in chunks
    DevBuf<uint64_t> ustage(al, (size_t)std::max<int64_t>(1, std::min(M, pl.u_chunk)));
    auto for_edge_chunks = [&](auto &&fn) {
        for (int64_t e0 = 0; e0 < M; e0 += pl.u_chunk) {
            const int64_t len = std::min(pl.u_chunk, M - e0);
            h2d(ustage.p, U.p + e0, (size_t)len, s);
            fn((const uint64_t *)ustage.p, len);
        }
    };

    // ---- C. out-degrees, offsets, slices
    DevBuf<int64_t> off(al, (size_t)N + 1);
    {
        DevBuf<int32_t> dh(al, (size_t)std::max<int64_t>(N, 1));
        fill_zero(dh.p, dh.bytes(), s);
        for_edge_chunks([&](const uint64_t *uk, int64_t len) {
            k_out_degrees<<<grid_for(len, 4), kThreads, 0, s>>>(uk, len, gb, rank.p, dh.p);
            TC_LAUNCH_CHECK();
        });
        DevBuf<int32_t> mx(al, 1);
        fill_zero(mx.p, 4, s);
        if (N > 0) {
            k_max_i32<<<grid_for(N, 8), kThreads, 0, s>>>(dh.p, N, mx.p);
            TC_LAUNCH_CHECK();
        }
        exclusive_scan(dh.p, off.p, N, true, al, s);
        d2h(&out.max_dhat, mx.p, 1, s);
    }
    out.off.reset((size_t)N + 1);
    d2h(out.off.p, off.p, (size_t)N + 1, s);
    TC_HIP(hipStreamSynchronize(s));

    // Slice footprint per row and per entry.  Build of a slice: two key
    // buffers and sort tables (18 B / entry) plus run records (32 B / row);
    // the count needs less per entry (rows 8 B, entries 4 B) and the rest of
    // the budget for streamed ranges.
    const int64_t eb = 18, nbw = 48;
    {
        const uint64_t room = headroom(al, B);
        const uint64_t slice_room = room > kSlack * 2 ? room - kSlack * 2 : 0;
        const uint64_t total_w = (uint64_t)eb * (uint64_t)M + (uint64_t)nbw * (uint64_t)N;
        // the largest single row must fit
        if ((uint64_t)eb * (uint64_t)out.max_dhat + (uint64_t)nbw > slice_room)
            throw Error(TC_ERR_OUT_OF_MEMORY, "device budget too small for the longest list");
        const uint64_t per = slice_room > (uint64_t)(eb * out.max_dhat + nbw)
                                 ? slice_room - (uint64_t)(eb * out.max_dhat + nbw)
                                 : 1;
        int64_t P = (int64_t)std::max<uint64_t>(1, (total_w + per - 1) / per);
        P = std::max<int64_t>(P, partitions);
        P = std::min<int64_t>(P, std::max<int64_t>(N, 1));
        std::vector<int64_t> tg;
        for (int64_t j = 1; j < P; ++j) tg.push_back((int64_t)(((unsigned __int128)j * total_w + P - 1) / P));
        std::vector<int64_t> c((size_t)P + 1, 0);
        c[P] = N;
        if (!tg.empty()) {
            DevBuf<int64_t> dt(al, tg.size()), dc(al, tg.size());
            h2d(dt.p, tg.data(), tg.size(), s);
            k_slice_bounds<<<grid_for((int64_t)tg.size()), kThreads, 0, s>>>(off.p, N, eb, nbw, dt.p,
                                                                               (int64_t)tg.size(), dc.p);
            TC_LAUNCH_CHECK();
            d2h(c.data() + 1, dc.p, tg.size(), s);
            TC_HIP(hipStreamSynchronize(s));
        }
        out.P = (int32_t)P;
        out.cut = c;
        out.ecut.assign((size_t)P + 1, 0);
        for (int64_t j = 0; j <= P; ++j) out.ecut[j] = out.off.p[c[j]];
        out.rows_max = out.entries_max = 0;
        for (int64_t j = 0; j < P; ++j) {
            out.rows_max = std::max(out.rows_max, c[j + 1] - c[j]);
            out.entries_max = std::max(out.entries_max, out.ecut[j + 1] - out.ecut[j]);
        }
        if (out.entries_max >= ((int64_t)1 << 29)) throw Error(TC_ERR_TOO_LARGE, "slice of 2^29 or more entries");
    }

    // ---- D. rows of each slice, and the records they send
    out.col.reset((size_t)std::max<int64_t>(M, 1));
    const int P = out.P;
    std::vector<std::vector<int32_t>> hv(P), htc(P), hlen(P);
    std::vector<std::vector<int64_t>> hpos(P);
    {
        DevBuf<unsigned long long> counter(al, 1);
        for (int i = 0; i < P; ++i) {
            const int64_t lo = out.cut[i], hi = out.cut[i + 1];
            const int64_t E = out.ecut[i + 1] - out.ecut[i];
            const int64_t rows = hi - lo;
            if (E == 0) continue;
            DevBuf<uint64_t> ka(al, (size_t)E), kb(al, (size_t)E);
            fill_zero(counter.p, 8, s);
            for_edge_chunks([&](const uint64_t *uk, int64_t len) {
                k_slice_keys<<<grid_for(len, 4), kThreads, 0, s>>>(uk, len, gb, rank.p, (int32_t)lo, (int32_t)hi,
                                                                    ka.p, counter.p, E);
                TC_LAUNCH_CHECK();
            });
            const int lb = std::max(1, bits_for((uint64_t)std::max<int64_t>(rows - 1, 1)));
            uint64_t *sorted = radix_sort_u64(ka.p, kb.p, E, 0, gb + lb, al, s);
            int32_t *col_i = reinterpret_cast<int32_t *>(sorted == ka.p ? kb.p : ka.p);
            k_low_bits<<<grid_for(E, 4), kThreads, 0, s>>>(sorted, E, gb, col_i);
            TC_LAUNCH_CHECK();
            unsigned long long got = 0;
            d2h(&got, counter.p, 1, s);
            d2h(out.col.p + out.ecut[i], col_i, (size_t)E, s);
            TC_HIP(hipStreamSynchronize(s));
            if ((int64_t)got != E) throw Error(TC_ERR_DEVICE, "slice pair count disagrees with the offsets");
            // records to slices j >= i, in node order
            DevBuf<uint32_t> flag(al, (size_t)rows);
            DevBuf<int32_t> first(al, (size_t)rows), cnt(al, (size_t)rows);
            DevBuf<int64_t> at(al, (size_t)rows + 1);
            DevBuf<int32_t> rv(al, (size_t)rows), rtc(al, (size_t)rows), rlen(al, (size_t)rows);
            DevBuf<int64_t> rpos(al, (size_t)rows);
            for (int j = i; j < P; ++j) {
                if (out.cut[j + 1] == out.cut[j]) continue;
                k_run_of_slice<<<grid_for(rows), kThreads, 0, s>>>(off.p, col_i, out.ecut[i], (int32_t)lo, rows,
                                                                   (int32_t)out.cut[j], (int32_t)out.cut[j + 1],
                                                                   flag.p, first.p, cnt.p);
                TC_LAUNCH_CHECK();
                exclusive_scan(flag.p, at.p, rows, true, al, s);
                int64_t R = 0;
                d2h(&R, at.p + rows, 1, s);
                TC_HIP(hipStreamSynchronize(s));
                if (R == 0) continue;
                k_write_records<<<grid_for(rows), kThreads, 0, s>>>(off.p, flag.p, at.p, first.p, cnt.p, (int32_t)lo,
                                                                    rows, rv.p, rpos.p, rtc.p, rlen.p);
                TC_LAUNCH_CHECK();
                const size_t old = hv[j].size();
                hv[j].resize(old + R);
                htc[j].resize(old + R);
                hlen[j].resize(old + R);
                hpos[j].resize(old + R);
                d2h(hv[j].data() + old, rv.p, (size_t)R, s);
                d2h(htc[j].data() + old, rtc.p, (size_t)R, s);
                d2h(hlen[j].data() + old, rlen.p, (size_t)R, s);
                d2h(hpos[j].data() + old, rpos.p, (size_t)R, s);
                TC_HIP(hipStreamSynchronize(s));
            }
        }
    }
    U.release();

    // Records grouped by destination slice, then batches that fit the count's
    // room.  The direct scheme (Section IV-C, for comparison) sends a list once
    // per stored edge instead of once per slice: record (v, pos, c, len) becomes
    // c records (v, pos + k, 1, len - k), the part of N_v from its k-th target on.
    int64_t R = 0;
    out.direct = bp.direct != 0;
    out.rbase.assign((size_t)P + 1, 0);
    for (int j = 0; j < P; ++j) {
        out.rbase[j] = R;
        if (out.direct) {
            for (const int32_t c : htc[j]) R += c;
        } else {
            R += (int64_t)hv[j].size();
        }
    }
    out.rbase[P] = R;
    out.rv.reset((size_t)std::max<int64_t>(R, 1));
    out.rtc.reset((size_t)std::max<int64_t>(R, 1));
    out.rlen.reset((size_t)std::max<int64_t>(R, 1));
    out.rpos.reset((size_t)std::max<int64_t>(R, 1));
    for (int j = 0; j < P; ++j) {
        const size_t n = hv[j].size();
        if (!n) continue;
        if (out.direct) {
            int64_t o = out.rbase[j];
            for (size_t r = 0; r < n; ++r)
                for (int32_t k = 0; k < htc[j][r]; ++k, ++o) {
                    out.rv.p[o] = hv[j][r];
                    out.rtc.p[o] = 1;
                    out.rlen.p[o] = hlen[j][r] - k;
                    out.rpos.p[o] = hpos[j][r] + k;
                }
        } else {
            std::memcpy(out.rv.p + out.rbase[j], hv[j].data(), n * 4);
            std::memcpy(out.rtc.p + out.rbase[j], htc[j].data(), n * 4);
            std::memcpy(out.rlen.p + out.rbase[j], hlen[j].data(), n * 4);
            std::memcpy(out.rpos.p + out.rbase[j], hpos[j].data(), n * 8);
        }
        std::vector<int32_t>().swap(hv[j]);
        std::vector<int32_t>().swap(htc[j]);
        std::vector<int32_t>().swap(hlen[j]);
        std::vector<int64_t>().swap(hpos[j]);
    }
    // Count-time room for one batch: the budget minus the persistent arrays
    // (perm, per-node counts and their host staging: 20 B / node), the largest
    // slice and slack.
    {
        const uint64_t fixed = (uint64_t)N * 20 + (uint64_t)out.rows_max * 8 + (uint64_t)out.entries_max * 4 +
                               kSlack * 2 + (uint64_t)bp.workers * 128;
        const uint64_t room = B > fixed ? B - fixed : 0;
        // per record: ids, position, counts, offsets and its task-table share (80 B);
        // per streamed id: 4 B.  Half of the room each.
        out.rec_cap = (int64_t)std::max<uint64_t>(1, room / 2 / 80);
        out.msg_cap = (int64_t)std::max<uint64_t>(1, room / 2 / 4);
        if (out.msg_cap < (int64_t)out.max_dhat)
            throw Error(TC_ERR_OUT_OF_MEMORY, "device budget too small to stream the longest list");
        out.rec_cap = std::min<int64_t>(out.rec_cap, (int64_t)1 << 30);
        out.msg_cap = std::min<int64_t>(out.msg_cap, (int64_t)1 << 31);
    }
    out.batch.clear();
    for (int j = 0; j < P; ++j) {
        int64_t r = out.rbase[j];
        const int64_t r1 = out.rbase[j + 1];
        while (r < r1) {
            out.batch.push_back(r);
            int64_t ids = 0, n = 0;
            while (r < r1 && n < out.rec_cap && ids + out.rlen.p[r] <= out.msg_cap) {
                ids += out.rlen.p[r];
                ++n;
                ++r;
            }
        }
    }
    out.batch.push_back(R);
}

void count_partitioned(Partitioned &pg, const BuildParams &bp, int32_t lds_max, int32_t search,
                       int32_t cuckoo_rounds, Allocator &al,
                       hipStream_t s, int64_t *totals, int64_t *tv, uint32_t *heads) {
    fill_zero(totals, 8, s);
    if (tv) fill_zero(tv, (size_t)std::max<int64_t>(pg.N, 1) * 8, s);
    pg.streamed_bytes = 0;
    if (pg.M == 0) return;
    const int32_t *hcol = pg.col.device_ptr();
    DevBuf<int64_t> off_j(al, (size_t)pg.rows_max + 1);
    DevBuf<int32_t> col_j(al, (size_t)std::max<int64_t>(pg.entries_max, 1));
    DevBuf<int64_t> nb_dev(al, 2);
    {
        const int64_t nbh[2] = {0, pg.N};
        h2d(nb_dev.p, nbh, 2, s);
    }
    DevBuf<CountDesc> desc(al, 1);
    // batch boundaries: batch b covers records [batch[b], batch[b+1]) of one slice
    size_t b = 0;
    const size_t nbatch = pg.batch.size() ? pg.batch.size() - 1 : 0;
    for (int j = 0; j < pg.P; ++j) {
        const int64_t lo = pg.cut[j], hi = pg.cut[j + 1];
        const int64_t E = pg.ecut[j + 1] - pg.ecut[j];
        // skip to this slice's batches
        while (b < nbatch && pg.batch[b] < pg.rbase[j]) ++b;
        if (hi == lo || E == 0 || pg.rbase[j + 1] == pg.rbase[j]) continue;
        h2d(off_j.p, pg.off.p + lo, (size_t)(hi - lo + 1), s);
        k_rebase<<<grid_for(hi - lo + 1, 4), kThreads, 0, s>>>(off_j.p, hi - lo + 1, pg.ecut[j]);
        TC_LAUNCH_CHECK();
        h2d(col_j.p, pg.col.p + pg.ecut[j], (size_t)E, s);
        pg.streamed_bytes += (hi - lo + 1) * 8 + E * 4;
        for (; b < nbatch && pg.batch[b] < pg.rbase[j + 1]; ++b) {
            const int64_t r0 = pg.batch[b], r1 = pg.batch[b + 1];
            const int64_t nr = r1 - r0;
            DevBuf<int32_t> rv(al, (size_t)nr), rtc(al, (size_t)nr), rlen(al, (size_t)nr);
            DevBuf<int64_t> rpos(al, (size_t)nr), moff(al, (size_t)nr + 1);
            h2d(rv.p, pg.rv.p + r0, (size_t)nr, s);
            h2d(rtc.p, pg.rtc.p + r0, (size_t)nr, s);
            h2d(rlen.p, pg.rlen.p + r0, (size_t)nr, s);
            h2d(rpos.p, pg.rpos.p + r0, (size_t)nr, s);
            exclusive_scan(rlen.p, moff.p, nr, true, al, s);
            int64_t ids = 0;
            d2h(&ids, moff.p + nr, 1, s);
            TC_HIP(hipStreamSynchronize(s));
            DevBuf<int32_t> mcol(al, (size_t)std::max<int64_t>(ids, 1));
            k_gather_ranges<<<grid_for(nr * 64, 1), kThreads, 0, s>>>(hcol, rpos.p, moff.p, nr, mcol.p);
            TC_LAUNCH_CHECK();
            pg.streamed_bytes += nr * 20 + ids * 4;
            // task table of this batch
            DevBuf<int64_t> f(al, (size_t)nr);
            DevBuf<uint32_t> wmed(al, (size_t)nr), wlarge(al, (size_t)nr);
            k_slice_costs<<<grid_for(nr), kThreads, 0, s>>>(moff.p, mcol.p, rtc.p, nr, off_j.p, (int32_t)lo,
                                                             bp.small_max, max_medium_list(), f.p, wmed.p, wlarge.p);
            TC_LAUNCH_CHECK();
            Schedule sc;
            schedule_sources(f.p, wmed.p, wlarge.p, nr, 1, nb_dev.p, bp, al, al, s, sc);
            f.release();
            wmed.release();
            wlarge.release();
            CountDesc d{};
            d.off = off_j.p;
            d.col = col_j.p;
            d.bnd = sc.bnd.p;
            d.gid = nullptr;
            d.node_base = nb_dev.p;
            d.big = sc.big.p;
            d.totals = totals;
            d.tv = tv;
            d.m = E;
            d.nmed = sc.nmed;
            d.nbig = sc.nbig;
            d.k = 1;
            d.small_max = bp.small_max;
            d.search_ratio = search;
            d.soff = moff.p;
            d.scol = mcol.p;
            d.sid = rv.p;
            d.tcnt = rtc.p;
            d.row_lo = (int32_t)lo;
            h2d(desc.p, &d, 1, s);
            fill_zero(heads, 16, s);
            CountLaunch L{};
            L.descs = desc.p;
            L.ndesc = 1;
            L.total_tasks = sc.tasks;
            L.total_med = sc.nmed;
            L.total_large = sc.nbig - sc.nmed;
            L.max_m = E;
            L.heads = heads;
            L.workers = bp.workers;
            L.lds_max = lds_max;
            L.cuckoo_rounds = cuckoo_rounds;
            L.per_node = tv != nullptr;
            L.slice = true;
            count_launch(L, s);
            // buffers of this batch are released in stream order; the next
            // batch's descriptor copy is ordered after this launch
        }
    }
}

}  // namespace tc
