// Device build of the oriented adjacency (Fig. 1, first two loops) and of the
// task table (Section V-B), for k graphs packed into one node space.
//
// Packed labels: node v of graph g is x = node_base[g] + v.  Graphs occupy
// disjoint, consecutive label ranges both before and after the degree-order
// relabelling, so every sort below works on one key space.
//
//   1. canonical edge set  -- key (x_lo << GB) | x_hi, loops dropped, radix sort, unique
//   2. degrees             -- d_x = number of distinct neighbours (Section II)
//   3. degree order        -- sort (g, d_x, v): position r in the sorted list is the
//                             new label of x (Section III-A order, ties by id)
//   4. orientation         -- edge {a, b} stored at the lower label s as (s, t);
//                             stable radix passes order the keys by s >> 12,
//                             chunks of each 4096-row group place them into the rows
//   5. CSR                 -- col = t, off = exclusive scan of row lengths; each row
//                             then sorted ascending on its own
//   6. costs and tasks     -- f per node (Sections IV-B, IV-F, V-A), prefix sums,
//                             Eq. (1)/(2) targets, one binary search per task boundary
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>

#include "internal.h"

namespace tc {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int per_thread = 1) {
    int64_t b = ceil_div(n, (int64_t)kThreads * per_thread);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)1 << 30));
}

constexpr uint64_t kInvalid = ~0ull;

__global__ void k_fill_zero_u32(uint32_t *p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__device__ __forceinline__ int upper_bound_i64(const int64_t *a, int n, int64_t x) {
    // first index i in [0, n) with a[i] > x, or n
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] > x)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Step 1a: canonical keys.  err bit 0: id out of range; bit 1: a loop.
// Each thread takes kEdgeUnroll edges at a time: all endpoint loads are issued
// before the first key is stored.
constexpr int kEdgeUnroll = 4;

__global__ void k_edge_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m_in,
                            const int64_t *__restrict__ edge_base, const int64_t *__restrict__ node_base, int k,
                            int gb, uint64_t *__restrict__ keys, uint32_t *__restrict__ err) {
    const int64_t b1 = k == 1 ? node_base[0] : 0, n1 = k == 1 ? node_base[1] - b1 : 0;  // the one graph
    const int64_t step = (int64_t)blockDim.x * kEdgeUnroll;
    for (int64_t e0 = (int64_t)blockIdx.x * step + threadIdx.x; e0 < m_in; e0 += (int64_t)gridDim.x * step) {
        int32_t u[kEdgeUnroll], v[kEdgeUnroll];
#pragma unroll
        for (int j = 0; j < kEdgeUnroll; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            u[j] = e < m_in ? __builtin_nontemporal_load(&src[e]) : 0;
            v[j] = e < m_in ? __builtin_nontemporal_load(&dst[e]) : 0;
        }
        // each edge's graph (first node label and node count), all looked up
        // before any key is stored
        int64_t nb[kEdgeUnroll], ng[kEdgeUnroll];
        if (k == 1) {
#pragma unroll
            for (int j = 0; j < kEdgeUnroll; ++j) {
                nb[j] = b1;
                ng[j] = n1;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kEdgeUnroll; ++j) {
                const int64_t e = e0 + (int64_t)j * blockDim.x;
                const int g = e < m_in ? upper_bound_i64(edge_base, k + 1, e) - 1 : 0;
                nb[j] = node_base[g];
                ng[j] = node_base[g + 1] - nb[j];
            }
        }
        uint64_t key[kEdgeUnroll];
        uint32_t bad = 0;
#pragma unroll
        for (int j = 0; j < kEdgeUnroll; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            key[j] = kInvalid;
            if (e >= m_in) continue;
            if (u[j] < 0 || v[j] < 0 || u[j] >= ng[j] || v[j] >= ng[j]) {
                bad |= 1u;
            } else if (u[j] == v[j]) {
                bad |= 2u;  // a loop: dropped
            } else {
                const int32_t lo = u[j] < v[j] ? u[j] : v[j], hi = u[j] < v[j] ? v[j] : u[j];
                key[j] = ((uint64_t)(nb[j] + lo) << gb) | (uint64_t)(nb[j] + hi);
            }
        }
#pragma unroll
        for (int j = 0; j < kEdgeUnroll; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            if (e < m_in) keys[e] = key[j];
        }
        if (bad) atomicOr(err, bad);
    }
}

// Unique selection in two passes over tiles of sorted keys: count the first
// occurrences per tile, then (after a scan of the tile counts) write them.
constexpr int kSelItems = 16;
constexpr int kSelTile = kThreads * kSelItems;

// Same layout as k_unique_write below: each wave walks its contiguous quarter
// of the tile 64 keys at a time and compares each key with its predecessor
// (a shuffle; lane 0 takes the last key of the previous step).
__global__ __launch_bounds__(kThreads) void k_unique_count(const uint64_t *__restrict__ keys, int64_t n,
                                                           int64_t *__restrict__ partial) {
    constexpr int kWaves = kThreads / 64;
    __shared__ int32_t wsum[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t wbase = (int64_t)blockIdx.x * kSelTile + (int64_t)wave * 64 * kSelItems;
    uint64_t k[kSelItems];
#pragma unroll
    for (int r = 0; r < kSelItems; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = i < n ? keys[i] : kInvalid;
    }
    const int64_t i0 = wbase - 1;
    uint64_t carry = (i0 >= 0 && i0 < n) ? keys[i0] : kInvalid;  // key before this wave's range
    int32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < kSelItems; ++r) {
        uint64_t prev = __shfl_up(k[r], 1, 64);
        if (lane == 0) prev = carry;
        const int64_t i = wbase + r * 64 + lane;
        cnt += popc64(__ballot(k[r] != kInvalid && (i == 0 || prev != k[r])));
        carry = __shfl(k[r], 63, 64);
    }
    if (lane == 0) wsum[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w];
        partial[blockIdx.x] = t;
    }
}

// Each wave owns a contiguous quarter of the tile and walks it 64 keys at a
// time, so both the reads and the writes of selected keys are coalesced.
__global__ __launch_bounds__(kThreads) void k_unique_write(const uint64_t *__restrict__ keys, int64_t n,
                                                           const int64_t *__restrict__ offsets,
                                                           uint64_t *__restrict__ out) {
    constexpr int kWaves = kThreads / 64;
    __shared__ int32_t wcount[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t wbase = (int64_t)blockIdx.x * kSelTile + (int64_t)wave * 64 * kSelItems;
    uint64_t k[kSelItems];
    uint64_t sel[kSelItems];
    int32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < kSelItems; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = i < n ? keys[i] : kInvalid;
    }
    const int64_t i0 = wbase - 1;
    uint64_t carry = (i0 >= 0 && i0 < n) ? keys[i0] : kInvalid;  // key before this wave's range
#pragma unroll
    for (int r = 0; r < kSelItems; ++r) {
        uint64_t prev = __shfl_up(k[r], 1, 64);
        if (lane == 0) prev = carry;
        const int64_t i = wbase + r * 64 + lane;
        const bool f = k[r] != kInvalid && (i == 0 || prev != k[r]);
        sel[r] = __ballot(f);
        cnt += popc64(sel[r]);
        carry = __shfl(k[r], 63, 64);
    }
    if (lane == 0) wcount[wave] = cnt;
    __syncthreads();
    int64_t o = offsets[blockIdx.x];
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        if (w < wave) o += wcount[w];
#pragma unroll
    for (int r = 0; r < kSelItems; ++r) {
        if ((sel[r] >> lane) & 1ull) out[o + popc64(sel[r] & lanemask_lt())] = k[r];
        o += popc64(sel[r]);
    }
}

// Lanes of a wave holding equal, contiguous values of `key` form a run; the
// last lane of each run receives the run's sum of `val`.
template <class T>
__device__ __forceinline__ T run_sum_at_end(int64_t key, T val, bool *is_end) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(val, d, 64);
        const int64_t kd = __shfl_up(key, d, 64);
        if (lane >= d && kd == key) val += y;
    }
    const int64_t kn = __shfl_down(key, 1, 64);
    *is_end = (lane == 63) || (kn != key);
    return val;
}

// Runs of a sorted key array, one wave at a time.  The wave holds positions
// w0 .. w0+63 (i = w0 + lane) with label x (>= 0; -1 past the end m) and the
// labels xp, xn of positions i - 1 and i + 1 (-2 / -3 outside 0..m-1), all
// three loaded by the caller at once.  A run cut by the wave's edges is split
// into pieces.  Each lane that ends a piece gets the piece's length (the
// others 0) and *whole = whether the piece is the entire run: then the lane
// is the run's only writer and may store plainly; pieces of a longer run add
// atomically.  Starts and ends come from two ballots.
__device__ __forceinline__ int64_t run_piece_at_end(int64_t x, int64_t xp, int64_t xn, bool valid, int lane,
                                                    bool *whole) {
    const uint64_t starts = __ballot(valid && x != xp);
    const uint64_t ends = __ballot(valid && x != xn);
    *whole = false;
    if (!valid || !(((ends >> lane) & 1ull) || lane == 63)) return 0;
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t b = (starts | 1ull) & upto;  // lane 0 opens a piece
    const int first = 63 - __clzll((long long)b);
    *whole = ((starts >> first) & 1ull) && ((ends >> lane) & 1ull);
    return lane - first + 1;
}

// Labels key >> shift at positions i - 1, i, i + 1 of keys[0..m).
__device__ __forceinline__ void labels3(const uint64_t *__restrict__ keys, int64_t i, int64_t m, int shift,
                                        uint64_t *k, int64_t *xp, int64_t *x, int64_t *xn) {
    const bool valid = i < m;
    *k = valid ? keys[i] : 0;
    const uint64_t kp = (valid && i > 0) ? keys[i - 1] : 0;
    const uint64_t kn = (i + 1 < m) ? keys[i + 1] : 0;
    *x = valid ? (int64_t)(*k >> shift) : -1;
    *xp = (valid && i > 0) ? (int64_t)(kp >> shift) : -2;
    *xn = (i + 1 < m) ? (int64_t)(kn >> shift) : -3;
}

// Step 2: degrees.  Keys are sorted, so each lower endpoint forms one run,
// counted per piece; the upper endpoints are written out for the histogram
// below.
__global__ void k_degrees_lo(const uint64_t *__restrict__ keys, int64_t m, int gb, int32_t *__restrict__ deg,
                             uint32_t *__restrict__ hi_out) {
    const uint64_t mask = (1ull << gb) - 1;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const int64_t i = base + threadIdx.x;
        uint64_t k;
        int64_t lp, lo, ln;
        labels3(keys, i, m, gb, &k, &lp, &lo, &ln);
        bool whole;
        const int64_t cnt = run_piece_at_end(lo, lp, ln, i < m, lane, &whole);
        if (cnt) atomicAdd(&deg[lo], (int32_t)cnt);  // adds without a read: nothing to wait for
        // stores last: a wait for the loads of the next step would also wait
        // for every store issued before them
        if (i < m) hi_out[i] = (uint32_t)(k & mask);
    }
}

// Label histogram in LDS by buckets of kBins consecutive labels.  vals is
// grouped by bucket (x >> kBinBits ascending); bucket b is cut into
// S_b = ceil(len_b / kHistChunk) equal parts (cstart: exclusive prefix of
// S_b, so heavy buckets get more workgroups).  The workgroup of part j counts
// its values, then adds its counters to deg: plainly when it is its bucket's
// only workgroup, else atomically.
constexpr int kBinBits = 12;
constexpr int kBins = 1 << kBinBits;
constexpr int kHistThreads = 1024;
constexpr int64_t kHistChunk = (int64_t)1 << 17;

__global__ void k_val_bucket_bounds(const uint32_t *__restrict__ vals, int64_t m, int64_t nbuckets,
                                    int64_t *__restrict__ bstart) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nbuckets;
         b += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(vals[mid] >> kBinBits) < b)
                lo = mid + 1;
            else
                hi = mid;
        }
        bstart[b] = lo;
    }
}

__global__ void k_bucket_parts(const int64_t *__restrict__ bstart, int64_t nbuckets, int32_t *__restrict__ parts) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nbuckets;
         b += (int64_t)gridDim.x * blockDim.x)
        parts[b] = (int32_t)max((int64_t)1, (bstart[b + 1] - bstart[b] + kHistChunk - 1) / kHistChunk);
}

__global__ __launch_bounds__(kHistThreads) void k_bucket_hist(const uint32_t *__restrict__ vals,
                                                              const int64_t *__restrict__ bstart,
                                                              const int64_t *__restrict__ cstart, int64_t nbuckets,
                                                              int64_t N, int32_t *__restrict__ deg) {
    __shared__ uint32_t cnt[kBins];
    const int64_t c = blockIdx.x;
    if (c >= cstart[nbuckets]) return;  // the grid is an upper bound on the parts
    int64_t b = 0, h = nbuckets;       // last bucket whose first part is <= c
    while (h - b > 1) {
        const int64_t mid = (b + h) >> 1;
        if (cstart[mid] <= c)
            b = mid;
        else
            h = mid;
    }
    const int64_t j = c - cstart[b], S = cstart[b + 1] - cstart[b];
    for (int i = threadIdx.x; i < kBins; i += kHistThreads) cnt[i] = 0;
    __syncthreads();
    const int64_t r0 = bstart[b], len = bstart[b + 1] - r0;
    const int64_t p0 = r0 + len * j / S, p1 = r0 + len * (j + 1) / S;
    constexpr int kUnroll = 4;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += (int64_t)kHistThreads * kUnroll) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t q = p + (int64_t)u * kHistThreads;
            v[u] = q < p1 ? vals[q] : ~0u;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (v[u] != ~0u) atomicAdd(&cnt[v[u] & (kBins - 1)], 1u);
    }
    __syncthreads();
    const int64_t x0 = b << kBinBits;
    for (int i = threadIdx.x; i < kBins; i += kHistThreads) {
        const int64_t x = x0 + i;
        const uint32_t cc = cnt[i];
        if (cc == 0 || x >= N) continue;
        if (S == 1)
            deg[x] += (int32_t)cc;
        else
            atomicAdd(&deg[x], (int32_t)cc);
    }
}

// Step 4b: rows by group.  The oriented keys (s << gb) | t are sorted by
// s >> kGroupBits (stable radix passes over the label bits above
// kGroupBits: one pass for up to 2^20 labels).  Each group's keys are cut
// into chunks of at most kChunkKeys, one workgroup per chunk, so a group of
// millions of keys (rows of a power-law graph's middle degrees) is shared
// out like any other:
//   k_chunk_count  counts the chunk's keys per row of its group in LDS;
//   k_chunk_scan   (one workgroup per group) turns those counts into each
//                  chunk's offset inside each row, and writes row lengths
//                  and offsets;
//   k_chunk_place  puts every key at its row's next slot (LDS cursors).
// The order inside a row is whatever the slot atomics give: rows are sorted
// on their own afterwards.  Among 64 keys two rarely share one of 4096 rows,
// so the LDS atomics seldom conflict.
constexpr int kGroupBits = 12;
constexpr int kGroupRows = 1 << kGroupBits;
constexpr int kChunkThreads = 1024;
constexpr int kChunkUnroll = 8;  // keys per thread loaded together
constexpr int64_t kChunkKeys = (int64_t)kChunkThreads * kChunkUnroll * 2;
constexpr int kRowsPerThread = kGroupRows / kChunkThreads;

__global__ void k_group_bounds(const uint64_t *__restrict__ keys, int64_t m, int shift, int64_t ngroups,
                               int64_t *__restrict__ gstart) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= ngroups;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(keys[mid] >> (shift + kGroupBits)) < g)
                lo = mid + 1;
            else
                hi = mid;
        }
        gstart[g] = lo;
    }
}

// chunks of group g: cfirst[g] .. cfirst[g + 1] (cfirst = exclusive scan of this)
__global__ void k_group_chunks(const int64_t *__restrict__ gstart, int64_t ngroups, int64_t *__restrict__ nchunk) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += (int64_t)gridDim.x * blockDim.x)
        nchunk[g] = (gstart[g + 1] - gstart[g] + kChunkKeys - 1) / kChunkKeys;
}

// Chunk c's group and key range (cfirst: chunk starts per group, ngroups + 1
// entries; c < cfirst[ngroups]).
__device__ __forceinline__ int64_t chunk_group(const int64_t *__restrict__ cfirst, int64_t ngroups, int64_t c) {
    int64_t lo = 0, hi = ngroups;  // last g with cfirst[g] <= c
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (cfirst[mid] <= c)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kChunkThreads) void k_chunk_count(const uint64_t *__restrict__ keys, int shift,
                                                               const int64_t *__restrict__ gstart,
                                                               const int64_t *__restrict__ cfirst, int64_t ngroups,
                                                               uint32_t *__restrict__ cnt) {
    __shared__ uint32_t lc[kGroupRows];
    const int64_t nchunks = cfirst[ngroups];
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t g = chunk_group(cfirst, ngroups, c);
        const int64_t b = gstart[g] + (c - cfirst[g]) * kChunkKeys;
        const int64_t e = min(gstart[g + 1], b + kChunkKeys);
        for (int r = threadIdx.x; r < kGroupRows; r += kChunkThreads) lc[r] = 0u;
        __syncthreads();
        for (int64_t p0 = b + threadIdx.x; p0 < e; p0 += (int64_t)kChunkThreads * kChunkUnroll) {
            uint64_t k[kChunkUnroll];
#pragma unroll
            for (int u = 0; u < kChunkUnroll; ++u) {
                const int64_t p = p0 + (int64_t)u * kChunkThreads;
                k[u] = p < e ? keys[p] : 0;
            }
#pragma unroll
            for (int u = 0; u < kChunkUnroll; ++u)
                if (p0 + (int64_t)u * kChunkThreads < e) atomicAdd(&lc[(uint32_t)(k[u] >> shift) & (kGroupRows - 1)], 1u);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < kGroupRows; r += kChunkThreads) cnt[c * kGroupRows + r] = lc[r];
        __syncthreads();
    }
}

// One workgroup per group: cnt[c][r] becomes the number of keys of row r in
// the group's chunks before c; row lengths and offsets of the group's rows.
__global__ __launch_bounds__(kChunkThreads) void k_chunk_scan(const int64_t *__restrict__ gstart,
                                                              const int64_t *__restrict__ cfirst, int64_t ngroups,
                                                              int64_t N, uint32_t *__restrict__ cnt,
                                                              int32_t *__restrict__ rowlen,
                                                              int64_t *__restrict__ off) {
    __shared__ uint32_t wtot[kChunkThreads / 64];
    const int tid = threadIdx.x, lane = __lane_id(), wave = threadIdx.x >> 6;
    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t c0 = cfirst[g], c1 = cfirst[g + 1];
        // rows tid + j * kChunkThreads (coalesced over the chunk tables)
        uint32_t len[kRowsPerThread];
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) len[j] = 0u;
        // four chunks' counts are loaded before any is rewritten
        int64_t c = c0;
        for (; c + 4 <= c1; c += 4) {
            uint32_t v[4][kRowsPerThread];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < kRowsPerThread; ++j) v[i][j] = cnt[(c + i) * kGroupRows + tid + j * kChunkThreads];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < kRowsPerThread; ++j) {
                    cnt[(c + i) * kGroupRows + tid + j * kChunkThreads] = len[j];
                    len[j] += v[i][j];
                }
        }
        for (; c < c1; ++c) {
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j) {
                uint32_t *q = &cnt[c * kGroupRows + tid + j * kChunkThreads];
                const uint32_t v = *q;
                *q = len[j];
                len[j] += v;
            }
        }
        // row starts: exclusive scan over the group's rows in row order
        // (row r = tid + j * kChunkThreads: scan j-major, threads inside)
        const int64_t x0 = g << kGroupBits, gs = gstart[g];
        uint32_t carry = 0;
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) {
            const uint32_t inc = wave_inclusive_sum(len[j]);
            if (lane == 63) wtot[wave] = inc;
            __syncthreads();
            uint32_t before = 0, all = 0;
            for (int w = 0; w < kChunkThreads / 64; ++w) {
                const uint32_t t = wtot[w];
                before += w < wave ? t : 0u;
                all += t;
            }
            const uint32_t start = carry + before + inc - len[j];
            const int64_t x = x0 + tid + j * kChunkThreads;
            if (x < N) {
                rowlen[x] = (int32_t)len[j];
                off[x] = gs + start;
            }
            carry += all;
            __syncthreads();
        }
        if (g == ngroups - 1 && tid == 0) off[N] = gstart[ngroups];
    }
}

__global__ __launch_bounds__(kChunkThreads) void k_chunk_place(const uint64_t *__restrict__ keys, int shift,
                                                               const int64_t *__restrict__ gstart,
                                                               const int64_t *__restrict__ cfirst, int64_t ngroups,
                                                               int64_t N, const uint32_t *__restrict__ cnt,
                                                               const int64_t *__restrict__ off,
                                                               int32_t *__restrict__ col) {
    __shared__ uint32_t lc[kGroupRows];
    const uint64_t mask = (1ull << shift) - 1;
    const int64_t nchunks = cfirst[ngroups];
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t g = chunk_group(cfirst, ngroups, c);
        const int64_t gs = gstart[g];
        const int64_t b = gs + (c - cfirst[g]) * kChunkKeys;
        const int64_t e = min(gstart[g + 1], b + kChunkKeys);
        const int64_t x0 = g << kGroupBits;
        for (int r = threadIdx.x; r < kGroupRows; r += kChunkThreads)
            lc[r] = x0 + r < N ? (uint32_t)(off[x0 + r] - gs) + cnt[c * kGroupRows + r] : 0u;
        __syncthreads();
        for (int64_t p0 = b + threadIdx.x; p0 < e; p0 += (int64_t)kChunkThreads * kChunkUnroll) {
            uint64_t k[kChunkUnroll];
#pragma unroll
            for (int u = 0; u < kChunkUnroll; ++u) {
                const int64_t p = p0 + (int64_t)u * kChunkThreads;
                k[u] = p < e ? keys[p] : 0;
            }
#pragma unroll
            for (int u = 0; u < kChunkUnroll; ++u) {
                if (p0 + (int64_t)u * kChunkThreads < e) {
                    const uint32_t slot = atomicAdd(&lc[(uint32_t)(k[u] >> shift) & (kGroupRows - 1)], 1u);
                    col[gs + slot] = (int32_t)(k[u] & mask);
                }
            }
        }
        __syncthreads();
    }
}

// Step 3a: degree-order keys (g, d, v).
__global__ void k_rank_keys(const int32_t *__restrict__ deg, int64_t N, const int64_t *__restrict__ node_base, int k,
                            int db, int vb, uint64_t *__restrict__ keys) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
        int g = 0;
        if (k > 1) g = upper_bound_i64(node_base, k + 1, x) - 1;
        const uint64_t v = (uint64_t)(x - node_base[g]);
        keys[x] = ((uint64_t)g << (db + vb)) | ((uint64_t)deg[x] << vb) | v;
    }
}

// Step 3b: position r of the sorted list is the new label of x.
__global__ void k_rank_from_sorted(const uint64_t *__restrict__ keys, int64_t N, const int64_t *__restrict__ node_base,
                                   int db, int vb, int32_t *__restrict__ perm, int32_t *__restrict__ rank) {
    const uint64_t vmask = (1ull << vb) - 1;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[r];
        const int g = (int)(key >> (db + vb));
        const int64_t x = node_base[g] + (int64_t)(key & vmask);
        perm[r] = (int32_t)x;
        rank[x] = (int32_t)r;
    }
}

// Step 4: oriented keys (s << gb) | t with s the lower new label.
// Each thread takes kOrientUnroll keys at a time, so that all of their label
// lookups are in flight together; the key streams are marked non-temporal to
// leave the cache to the label array.
constexpr int kOrientUnroll = 4;

__global__ void k_orient_keys(const uint64_t *__restrict__ ukeys, int64_t m, int gb, const int32_t *__restrict__ rank,
                              uint64_t *__restrict__ okeys) {
    const uint64_t mask = (1ull << gb) - 1;
    const int64_t step = (int64_t)blockDim.x * kOrientUnroll;
    for (int64_t i0 = (int64_t)blockIdx.x * step + threadIdx.x; i0 < m; i0 += (int64_t)gridDim.x * step) {
        uint64_t k[kOrientUnroll];
        uint32_t ra[kOrientUnroll], rb[kOrientUnroll];
#pragma unroll
        for (int u = 0; u < kOrientUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            k[u] = i < m ? __builtin_nontemporal_load(&ukeys[i]) : 0;
        }
#pragma unroll
        for (int u = 0; u < kOrientUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            ra[u] = i < m ? (uint32_t)rank[k[u] >> gb] : 0u;
            rb[u] = i < m ? (uint32_t)rank[k[u] & mask] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kOrientUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            if (i < m) {
                const uint64_t s = ra[u] < rb[u] ? ra[u] : rb[u], t = ra[u] < rb[u] ? rb[u] : ra[u];
                __builtin_nontemporal_store((s << gb) | t, &okeys[i]);
            }
        }
    }
}

// One graph given as an edge list: bit 0 of chk[0] if an id is outside
// 0..n-1, bit 1 if an edge is a loop (the pairs are checked before anything
// else reads them as labels).  Each workgroup also stores how often src and
// dst change value from one edge to the next (chk[2 + 2b], chk[3 + 2b]):
// long runs of one id (an edge list made from adjacency lists) let the
// degrees be counted from the runs instead of a histogram.
constexpr int kCheckBlocks = 8192;  // partial counts: 16 B per workgroup

__global__ void k_check_pairs(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m,
                              int64_t n, unsigned long long *__restrict__ chk) {
    __shared__ unsigned long long part[2][kThreads / 64];
    const int64_t step = (int64_t)blockDim.x * kEdgeUnroll;
    uint32_t bad = 0;
    uint32_t bs = 0, bd = 0;  // value changes in src and dst
    for (int64_t e0 = (int64_t)blockIdx.x * step + threadIdx.x; e0 < m; e0 += (int64_t)gridDim.x * step) {
        int32_t u[kEdgeUnroll], v[kEdgeUnroll], up[kEdgeUnroll], vp[kEdgeUnroll];
#pragma unroll
        for (int j = 0; j < kEdgeUnroll; ++j) {
            const int64_t e = e0 + (int64_t)j * blockDim.x;
            u[j] = e < m ? src[e] : 0;
            v[j] = e < m ? dst[e] : 1;
            up[j] = (e < m && e > 0) ? src[e - 1] : u[j];
            vp[j] = (e < m && e > 0) ? dst[e - 1] : v[j];
        }
#pragma unroll
        for (int j = 0; j < kEdgeUnroll; ++j) {
            if (u[j] < 0 || v[j] < 0 || u[j] >= n || v[j] >= n) bad |= 1u;
            else if (u[j] == v[j]) bad |= 2u;
            bs += u[j] != up[j] ? 1u : 0u;
            bd += v[j] != vp[j] ? 1u : 0u;
        }
    }
    const uint32_t w = (__ballot(bad & 1u) ? 1u : 0u) | (__ballot(bad & 2u) ? 2u : 0u);
    if (w && __lane_id() == 0) atomicOr(&chk[0], (unsigned long long)w);
    const unsigned long long ts = wave_sum((unsigned long long)bs), td = wave_sum((unsigned long long)bd);
    if (__lane_id() == 0) {
        part[0][threadIdx.x >> 6] = ts;
        part[1][threadIdx.x >> 6] = td;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long t = 0;
        for (int q = 0; q < kThreads / 64; ++q) t += part[threadIdx.x][q];
        chk[2 + 2 * blockIdx.x + threadIdx.x] = t;
    }
}

// out[0] = chk[0] (the flags), out[1] / out[2] = the change counts of src /
// dst summed over the nblk workgroups of k_check_pairs (one workgroup).
__global__ void k_check_sums(const unsigned long long *__restrict__ chk, unsigned nblk,
                             unsigned long long *__restrict__ out) {
    __shared__ unsigned long long part[2][kThreads / 64];
    unsigned long long s0 = 0, s1 = 0;
    for (unsigned b = threadIdx.x; b < nblk; b += blockDim.x) {
        s0 += chk[2 + 2 * (size_t)b];
        s1 += chk[3 + 2 * (size_t)b];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (__lane_id() == 0) {
        part[0][threadIdx.x >> 6] = s0;
        part[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t0 = 0, t1 = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            t0 += part[0][w];
            t1 += part[1][w];
        }
        out[0] = chk[0];
        out[1] = t0;
        out[2] = t1;
    }
}

// Degrees from runs of equal ids: each run (cut at wave edges into pieces)
// adds its length with one atomic.  For edge lists whose runs are long.
__global__ void k_run_degrees(const int32_t *__restrict__ vals, int64_t m, int32_t *__restrict__ deg) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < m;
        // neighbours from the next lanes; the wave's two edge lanes load theirs
        const int32_t v0 = valid ? vals[i] : -1;
        const int32_t e0 = (lane == 0 && valid && i > 0) ? vals[i - 1] : -2;
        const int32_t e1 = (lane == 63 && i + 1 < m) ? vals[i + 1] : -3;
        const int64_t x = v0;
        int64_t xp = __shfl_up(v0, 1, 64), xn = __shfl_down(v0, 1, 64);
        if (lane == 0) xp = e0;
        if (lane == 63) xn = e1;
        if (!valid) xn = -3;
        bool whole;
        const int64_t cnt = run_piece_at_end(x, xp, xn, valid, lane, &whole);
        if (cnt) atomicAdd(&deg[x], (int32_t)cnt);
    }
}

// Oriented keys straight from a checked edge list of one graph (labels are
// the ids), as k_orient_keys does from pair keys.
__global__ void k_orient_pairs(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m, int gb,
                               const int32_t *__restrict__ rank, uint64_t *__restrict__ okeys) {
    const int64_t step = (int64_t)blockDim.x * kOrientUnroll;
    for (int64_t i0 = (int64_t)blockIdx.x * step + threadIdx.x; i0 < m; i0 += (int64_t)gridDim.x * step) {
        int32_t u[kOrientUnroll], v[kOrientUnroll];
        uint32_t ra[kOrientUnroll], rb[kOrientUnroll];
#pragma unroll
        for (int j = 0; j < kOrientUnroll; ++j) {
            const int64_t i = i0 + (int64_t)j * blockDim.x;
            u[j] = i < m ? __builtin_nontemporal_load(&src[i]) : 0;
            v[j] = i < m ? __builtin_nontemporal_load(&dst[i]) : 0;
        }
#pragma unroll
        for (int j = 0; j < kOrientUnroll; ++j) {
            const int64_t i = i0 + (int64_t)j * blockDim.x;
            ra[j] = i < m ? (uint32_t)rank[u[j]] : 0u;
            rb[j] = i < m ? (uint32_t)rank[v[j]] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kOrientUnroll; ++j) {
            const int64_t i = i0 + (int64_t)j * blockDim.x;
            if (i < m) {
                const uint64_t lo = ra[j] < rb[j] ? ra[j] : rb[j], hi = ra[j] < rb[j] ? rb[j] : ra[j];
                __builtin_nontemporal_store((lo << gb) | hi, &okeys[i]);
            }
        }
    }
}

// Oriented keys as k_orient_pairs, written in the tiles of the radix passes
// that order them (kRadixTile keys per workgroup, same XCD mapping), with the
// digit table of the first pass (key bits shift .. shift + bits) counted on
// the way.  Inside a tile any thread may make any key: kOrientTileThreads
// threads make kRadixTile / kOrientTileThreads keys each.
constexpr int kOrientTileThreads = 512;
constexpr int kOrientTileWaves = kOrientTileThreads / 64;
// Adds one round of a tile's digits to the wave's LDS table: lanes holding
// the same digit (all of them when the first lane's digit is everyone's,
// else found with one ballot per digit bit) are counted by the first of
// them, so no counter gets two writes in a round.  d = 256: no key.
__device__ __forceinline__ void tile_digit_round(uint32_t *hw, uint32_t d, int bits, bool full) {
    const int lane = __lane_id();
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
    uint64_t peers = ~0ull;
    if (__ballot(d == d0) != ~0ull) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            if (b < bits) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bal = __ballot(bit);
                peers &= bit ? bal : ~bal;
            }
        }
        if (!full) {
            const bool past = d >> 8;
            const uint64_t bal = __ballot(past);
            peers &= past ? bal : ~bal;
        }
    }
    if (d < 256u && lane == __ffsll((unsigned long long)peers) - 1) hw[d] += (uint32_t)popc64(peers);
    wave_lds_sync();
}

// The tile's digit counts, summed over the waves' tables, into the
// digit-major table of the first radix pass.
template <int WAVES>
__device__ __forceinline__ void tile_digit_flush(uint32_t (*hw)[256], int64_t t, int64_t tiles,
                                                 uint32_t *__restrict__ hist) {
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += WAVES * 64) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) c += hw[w][i];
        hist[(int64_t)i * tiles + t] = c;
    }
}

// Oriented keys (min label << gb) | max label under rank, of the pairs
// (src[i], dst[i]) (KEYS false) or of the pair keys (lo << gb) | hi (KEYS
// true), written in the first radix pass's tiles together with that pass's
// digit table (bits [shift, shift + bits) of the keys), so the pass does not
// read the keys to count them.
template <bool KEYS>
__global__ __launch_bounds__(kOrientTileThreads) void k_orient_hist(const int32_t *__restrict__ src,
                                                                    const int32_t *__restrict__ dst,
                                                                    const uint64_t *__restrict__ ukeys, int64_t m,
                                                                    int gb, const int32_t *__restrict__ rank,
                                                                    uint64_t *__restrict__ okeys, int shift, int bits,
                                                                    int64_t tiles, uint32_t *__restrict__ hist) {
    constexpr int kRounds = kRadixTile / kOrientTileThreads;
    __shared__ uint32_t hw[kOrientTileWaves][256];  // one table per wave
    for (int i = threadIdx.x; i < kOrientTileWaves * 256; i += kOrientTileThreads) (&hw[0][0])[i] = 0u;
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int64_t t = xcd_tile(blockIdx.x, tiles);
    const int64_t base = t * kRadixTile + (int64_t)wave * (64 * kRounds) + lane;
    const bool full = m - t * kRadixTile >= kRadixTile;  // every lane holds a key
    const uint32_t dmask = (1u << bits) - 1u;
    const uint64_t lmask = (1ull << gb) - 1;
    // all endpoints are loaded, then all ranks gathered, before any key is made
    int32_t u[kRounds], v[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * 64;
        if (KEYS) {
            const uint64_t k = i < m ? __builtin_nontemporal_load(&ukeys[i]) : 0;
            u[r] = (int32_t)(k >> gb);
            v[r] = (int32_t)(k & lmask);
        } else {
            u[r] = i < m ? __builtin_nontemporal_load(&src[i]) : 0;
            v[r] = i < m ? __builtin_nontemporal_load(&dst[i]) : 0;
        }
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * 64;
        u[r] = i < m ? rank[u[r]] : 0;
        v[r] = i < m ? rank[v[r]] : 0;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * 64;
        const uint32_t ra = (uint32_t)u[r], rb = (uint32_t)v[r];
        const uint64_t key = ((uint64_t)(ra < rb ? ra : rb) << gb) | (ra < rb ? rb : ra);
        if (i < m) __builtin_nontemporal_store(key, &okeys[i]);
        tile_digit_round(hw[wave], i < m ? (uint32_t)(key >> shift) & dmask : 256u, bits, full);
    }
    tile_digit_flush<kOrientTileWaves>(hw, t, tiles, hist);
}

// Step 1a as k_edge_keys, in the first radix pass's tiles with that pass's
// digit table (bits [0, bits) of the keys; a dropped pair's key kInvalid has
// every bit set): the canonical path sorts the keys next.
__global__ __launch_bounds__(kOrientTileThreads) void k_edge_keys_hist(
    const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m_in,
    const int64_t *__restrict__ edge_base, const int64_t *__restrict__ node_base, int k, int gb,
    uint64_t *__restrict__ keys, uint32_t *__restrict__ err, int bits, int64_t tiles,
    uint32_t *__restrict__ hist) {
    constexpr int kRounds = kRadixTile / kOrientTileThreads;
    __shared__ uint32_t hw[kOrientTileWaves][256];
    for (int i = threadIdx.x; i < kOrientTileWaves * 256; i += kOrientTileThreads) (&hw[0][0])[i] = 0u;
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int64_t t = xcd_tile(blockIdx.x, tiles);
    const int64_t base = t * kRadixTile + (int64_t)wave * (64 * kRounds) + lane;
    const bool full = m_in - t * kRadixTile >= kRadixTile;
    const int64_t b1 = k == 1 ? node_base[0] : 0, n1 = k == 1 ? node_base[1] - b1 : 0;  // the one graph
    int32_t u[kRounds], v[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t e = base + r * 64;
        u[r] = e < m_in ? __builtin_nontemporal_load(&src[e]) : 0;
        v[r] = e < m_in ? __builtin_nontemporal_load(&dst[e]) : 0;
    }
    uint32_t bad = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t e = base + r * 64;
        int64_t nb = b1, ng = n1;
        if (k != 1 && e < m_in) {
            const int g = upper_bound_i64(edge_base, k + 1, e) - 1;
            nb = node_base[g];
            ng = node_base[g + 1] - nb;
        }
        uint64_t key = kInvalid;
        if (e < m_in) {
            if (u[r] < 0 || v[r] < 0 || u[r] >= ng || v[r] >= ng) {
                bad |= 1u;
            } else if (u[r] == v[r]) {
                bad |= 2u;  // a loop: dropped
            } else {
                const int32_t lo = u[r] < v[r] ? u[r] : v[r], hi = u[r] < v[r] ? v[r] : u[r];
                key = ((uint64_t)(nb + lo) << gb) | (uint64_t)(nb + hi);
            }
            keys[e] = key;
        }
        tile_digit_round(hw[wave], e < m_in ? (uint32_t)key & ((1u << bits) - 1u) : 256u, bits, full);
    }
    if (bad) atomicOr(err, bad);
    tile_digit_flush<kOrientTileWaves>(hw, t, tiles, hist);
}

// Step 5b: rows sorted ascending.  The pair sort above orders by s only, so
// each row holds its entries in input order.  A wave takes 64 consecutive
// rows: rows of up to 8 entries are sorted by their own lane with a sorting
// network in registers; rows of up to 64 entries (one per lane) and up to 256
// entries (four per lane, element i = 4 lane + j) are sorted one after another
// by the whole wave with a bitonic network; longer rows are listed for one
// radix sort of (row, t) keys.
constexpr int kTinyRow = 8;
constexpr int kShortRow = 64;
constexpr int kMidRow = 256;
constexpr int kLdsRowMid = 2048;    // long rows up to this length: one wave each, in registers
constexpr int kLdsRowMax = 16384;   // up to this length: 1024-thread workgroups, 64 KB of LDS

__device__ __forceinline__ void cswap(int32_t &a, int32_t &b) {
    const int32_t lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

// Cost kind PRIOR of a row of length a: a * a + the row lengths of its
// targets (Section IV-B).  Rows sorted here add it up from the entries they
// already hold (f non-null), so no separate pass over the pairs is needed.
// Repeated entries in a sorted row mean a repeated edge in the input (only
// possible when the canonical sort was skipped): one flag for the build.
// Called by the whole wave.
__device__ __forceinline__ void note_repeat(bool repeat, unsigned int *__restrict__ dup) {
    if (__ballot(repeat) && __lane_id() == 0) atomicOr(dup, 1u);
}

__device__ __forceinline__ void wave_sort_row(int32_t *__restrict__ col, int64_t r0, int32_t a, int lane,
                                              const int32_t *__restrict__ dh, int64_t *__restrict__ f, int64_t row,
                                              unsigned int *__restrict__ dup) {
    if (a <= kShortRow) {
        int32_t x = lane < a ? col[r0 + lane] : INT32_MAX;
        if (f) {
            const int64_t c = wave_sum((int64_t)(lane < a ? dh[x] : 0));
            if (lane == 0) f[row] = (int64_t)a * a + c;
        }
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int d = k >> 1; d > 0; d >>= 1) {
                const int32_t y = __shfl_xor(x, d, 64);
                const bool up = (lane & k) == 0, lower = (lane & d) == 0;
                x = (lower == up) ? min(x, y) : max(x, y);
            }
        }
        if (lane < a) col[r0 + lane] = x;
        note_repeat(lane + 1 < a && x == __shfl_down(x, 1, 64), dup);
        return;
    }
    int32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = lane * 4 + j;
        v[j] = i < a ? col[r0 + i] : INT32_MAX;
    }
    if (f) {
        int64_t c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (lane * 4 + j < a) c += dh[v[j]];
        c = wave_sum(c);
        if (lane == 0) f[row] = (int64_t)a * a + c;
    }
#pragma unroll
    for (int k = 2; k <= kMidRow; k <<= 1) {
#pragma unroll
        for (int d = k >> 1; d > 0; d >>= 1) {
            if (d >= 4) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = lane * 4 + j;
                    const int32_t y = __shfl_xor(v[j], d >> 2, 64);
                    const bool up = (i & k) == 0, lower = (i & d) == 0;
                    v[j] = (lower == up) ? min(v[j], y) : max(v[j], y);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j & d) continue;
                    const int p = j | d;
                    const bool up = ((lane * 4 + j) & k) == 0;
                    const int32_t lo = min(v[j], v[p]), hi = max(v[j], v[p]);
                    v[j] = up ? lo : hi;
                    v[p] = up ? hi : lo;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = lane * 4 + j;
        if (i < a) col[r0 + i] = v[j];
    }
    bool rep = false;
#pragma unroll
    for (int j = 0; j < 3; ++j) rep |= lane * 4 + j + 1 < a && v[j] == v[j + 1];
    const int32_t nx = __shfl_down(v[0], 1, 64);
    rep |= lane < 63 && lane * 4 + 4 < a && v[3] == nx;
    note_repeat(rep, dup);
}

__global__ __launch_bounds__(kThreads) void k_sort_rows(const int64_t *__restrict__ off, int64_t N,
                                                        int32_t *__restrict__ col, int32_t *__restrict__ long_rows,
                                                        unsigned int *__restrict__ nlong,
                                                        const int32_t *__restrict__ dh, int64_t *__restrict__ f,
                                                        unsigned int *__restrict__ dup) {
    const int lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t g0 = wave * 64; g0 < N; g0 += nwaves * 64) {
        bool rep = false;
        const int64_t r = g0 + lane;
        int64_t r0 = 0;
        int32_t a = 0;
        if (r < N) {
            r0 = off[r];
            a = (int32_t)(off[r + 1] - r0);
        }
        if (f && r < N && a == 0) f[r] = 0;
        if (a >= 1 && a <= kTinyRow) {
            int32_t x[kTinyRow];
#pragma unroll
            for (int j = 0; j < kTinyRow; ++j) x[j] = j < a ? col[r0 + j] : INT32_MAX;
            if (f) {
                int64_t c = (int64_t)a * a;
#pragma unroll
                for (int j = 0; j < kTinyRow; ++j)
                    if (j < a) c += dh[x[j]];
                f[r] = c;
            }
            if (a >= 2) {
                // optimal 19-comparator network for 8 inputs; padding sorts last
                cswap(x[0], x[2]); cswap(x[1], x[3]); cswap(x[4], x[6]); cswap(x[5], x[7]);
                cswap(x[0], x[4]); cswap(x[1], x[5]); cswap(x[2], x[6]); cswap(x[3], x[7]);
                cswap(x[0], x[1]); cswap(x[2], x[3]); cswap(x[4], x[5]); cswap(x[6], x[7]);
                cswap(x[2], x[4]); cswap(x[3], x[5]);
                cswap(x[1], x[4]); cswap(x[3], x[6]);
                cswap(x[1], x[2]); cswap(x[3], x[4]); cswap(x[5], x[6]);
#pragma unroll
                for (int j = 0; j < kTinyRow; ++j)
                    if (j < a) col[r0 + j] = x[j];
#pragma unroll
                for (int j = 0; j + 1 < kTinyRow; ++j) rep |= j + 1 < a && x[j] == x[j + 1];
            }
        }
        note_repeat(rep, dup);
        // rows of 9 to 64 entries: the whole wave sorts 4 of them at a time,
        // their loads and degree gathers in flight together and their sorting
        // networks interleaved (one row at a time: 455 us on PA, 4: 411 us)
        uint64_t rest = __ballot(a > kTinyRow && a <= kShortRow);
        while (rest) {
            int lr[4];
            int64_t rc[4];
            int32_t ac[4], xc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                lr[u] = -1;
                rc[u] = 0;
                ac[u] = 0;
                if (rest) {
                    lr[u] = __ffsll((unsigned long long)rest) - 1;
                    rest &= rest - 1;
                    rc[u] = readlane64(r0, lr[u]);
                    ac[u] = readlane32(a, lr[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xc[u] = lane < ac[u] ? col[rc[u] + lane] : INT32_MAX;
            int64_t dv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) dv[u] = (f && lane < ac[u]) ? (int64_t)dh[xc[u]] : 0;
#pragma unroll
            for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
                for (int d = k >> 1; d > 0; d >>= 1) {
                    const bool up = (lane & k) == 0, lower = (lane & d) == 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int32_t y = __shfl_xor(xc[u], d, 64);
                        xc[u] = (lower == up) ? min(xc[u], y) : max(xc[u], y);
                    }
                }
            }
            bool rp = false;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (lane < ac[u]) col[rc[u] + lane] = xc[u];
                rp = rp || (lane + 1 < ac[u] && xc[u] == __shfl_down(xc[u], 1, 64));
            }
            note_repeat(rp, dup);
            if (f) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t c = wave_sum(dv[u]);
                    if (lane == 0 && lr[u] >= 0) f[g0 + lr[u]] = (int64_t)ac[u] * ac[u] + c;
                }
            }
        }
        rest = __ballot(a > kShortRow && a <= kMidRow);
        while (rest) {
            const int l = __ffsll((unsigned long long)rest) - 1;
            rest &= rest - 1;
            wave_sort_row(col, readlane64(r0, l), readlane32(a, l), lane, dh, f, g0 + l, dup);
        }
        // longer rows are listed for one radix sort; their PRIOR costs do not
        // depend on the order of their entries and are added up here, one
        // wave per row, so the task table can be built before they are sorted
        if (a > kMidRow) long_rows[atomicAdd(nlong, 1u)] = (int32_t)r;
        if (f) {
            uint64_t lng = __ballot(a > kMidRow);
            while (lng) {
                const int l = __ffsll((unsigned long long)lng) - 1;
                lng &= lng - 1;
                const int64_t w0 = readlane64(r0, l);
                const int32_t wa = readlane32(a, l);
                int64_t c = 0;
                for (int64_t p = lane; p < wa; p += 64) c += dh[col[w0 + p]];
                c = wave_sum(c);
                if (lane == 0) f[g0 + l] = (int64_t)wa * wa + c;
            }
        }
    }
}

// Total PRIOR cost of the rows scheduled for single waves (length <= small),
// before any cost is computed per row.  Over all rows the PRIOR costs add up
// to sum_v dhat_v * d_v (pair (v, t) contributes dhat_v to f(v) and dhat_t
// to f(v); dhat_t is counted once for each of t's d_t - dhat_t in-pairs);
// acc[0] gets that sum, acc[1] the entries of the longer rows, whose own
// costs k_prior_wide then subtracts.
__global__ void k_prior_total(const int64_t *__restrict__ off, const int32_t *__restrict__ deg, int64_t N, int small,
                              unsigned long long *__restrict__ acc) {
    int64_t part = 0, wide = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = off[r + 1] - off[r];
        part += a * (int64_t)deg[r];
        wide += a > small ? a : 0;
    }
    // one add per workgroup: adds to one address are serialised
    __shared__ int64_t wpart[2][kThreads / 64];
    part = wave_sum(part);
    wide = wave_sum(wide);
    if (__lane_id() == 0) {
        wpart[0][threadIdx.x >> 6] = part;
        wpart[1][threadIdx.x >> 6] = wide;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0, w = 0;
        for (int i = 0; i < kThreads / 64; ++i) {
            t += wpart[0][i];
            w += wpart[1][i];
        }
        atomicAdd(acc, (unsigned long long)t);
        atomicAdd(acc + 1, (unsigned long long)w);
    }
}

// Subtracts the PRIOR cost of each row longer than small from acc[0], one
// wave per row, unless those rows hold more than `limit` entries in all
// (acc[1]): then the early total is not made (the gathers would cost more
// than they save) and acc[0] is left as it is.
__global__ void k_prior_wide(const int64_t *__restrict__ off, const int32_t *__restrict__ col, int64_t N, int small,
                             int64_t limit, unsigned long long *__restrict__ acc) {
    if ((int64_t)acc[1] > limit) return;
    const int lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t part = 0;
    for (int64_t g0 = wave * 64; g0 < N; g0 += nwaves * 64) {
        const int64_t r = g0 + lane;
        int64_t r0 = 0, a = 0;
        if (r < N) {
            r0 = off[r];
            a = off[r + 1] - r0;
        }
        uint64_t wide = __ballot(a > small);
        while (wide) {
            const int l = __ffsll((unsigned long long)wide) - 1;
            wide &= wide - 1;
            const int64_t w0 = readlane64(r0, l), wa = readlane64(a, l);
            int64_t c = 0;
            for (int64_t p = lane; p < wa; p += 64) {
                const int32_t t = col[w0 + p];
                c += off[t + 1] - off[t];
            }
            c = wave_sum(c);
            if (lane == 0) part -= wa * wa + c;
        }
    }
    // one add per workgroup: adds to one address are serialised
    __shared__ int64_t wpart[kThreads / 64];
    part = wave_sum(part);
    if (lane == 0) wpart[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += wpart[w];
        atomicAdd(acc, (unsigned long long)t);
    }
}

// Entries of each long row left to the radix sort: rows of up to lds_max
// entries are sorted by k_long_sort_wave / k_long_sort and count 0 here.
__global__ void k_long_lengths(const int64_t *__restrict__ off, const int32_t *__restrict__ long_rows, int64_t L,
                               int64_t lds_max, int64_t *__restrict__ len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = long_rows[i];
        const int64_t a = off[r + 1] - off[r];
        len[i] = a <= lds_max ? 0 : a;
    }
}

// keys (i << gb) | t of the entries of long row i, from epos[i] on (one wave
// per row); rows with no entries left to the radix sort are skipped
__global__ void k_long_keys(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ long_rows, const int64_t *__restrict__ epos, int64_t L, int gb,
                            uint64_t *__restrict__ keys) {
    const int lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < L; i += nwaves) {
        const int64_t e = epos[i], a = epos[i + 1] - e;
        if (a == 0) continue;
        const int64_t r0 = off[long_rows[i]];
        for (int64_t p = lane; p < a; p += 64) keys[e + p] = ((uint64_t)i << gb) | (uint64_t)(uint32_t)col[r0 + p];
    }
}

// Long rows of up to 64 E entries, one wave per row: lane l holds entries
// l E .. l E + E - 1 in registers (padded with INT32_MAX) and the wave runs a
// bitonic network over all 64 E of them, exchanging across lanes by shuffles
// for distances of E or more; equal neighbours after the sort are repeats.
template <int E>
__device__ __forceinline__ void wave_sort_long(int32_t *__restrict__ col, int64_t r0, int32_t a, int lane,
                                               unsigned int *__restrict__ dup) {
    constexpr int N = 64 * E;
    int32_t v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int i = lane * E + j;
        v[j] = i < a ? col[r0 + i] : INT32_MAX;
    }
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int d = k >> 1; d > 0; d >>= 1) {
            if (d >= E) {
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int i = lane * E + j;
                    const int32_t y = __shfl_xor(v[j], d / E, 64);
                    const bool up = (i & k) == 0, lower = (i & d) == 0;
                    v[j] = (lower == up) ? min(v[j], y) : max(v[j], y);
                }
            } else {
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    if (j & d) continue;
                    const int p = j | d;
                    const bool up = ((lane * E + j) & k) == 0;
                    const int32_t lo = min(v[j], v[p]), hi = max(v[j], v[p]);
                    v[j] = up ? lo : hi;
                    v[p] = up ? hi : lo;
                }
            }
        }
    }
    bool rep = false;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int i = lane * E + j;
        if (i < a) col[r0 + i] = v[j];
        if (j + 1 < E) rep |= i + 1 < a && v[j] == v[j + 1];
    }
    const int32_t nx = __shfl_down(v[0], 1, 64);
    rep |= lane < 63 && lane * E + E < a && v[E - 1] == nx;
    note_repeat(rep, dup);
}

// Long rows of (32 E, min(hi, 64 E)] entries, one wave per row (one launch per
// E, so that each holds only the registers its rows need).
template <int E>
__global__ __launch_bounds__(kThreads) void k_long_sort_wave(const int64_t *__restrict__ off, int32_t *__restrict__ col,
                                                             const int32_t *__restrict__ long_rows, int64_t L,
                                                             int32_t hi, unsigned int *__restrict__ dup) {
    const int lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < L; i += nwaves) {
        const int32_t r = long_rows[i];
        const int64_t r0 = off[r];
        const int32_t a = (int32_t)(off[r + 1] - r0);
        if (a <= 32 * E || a > hi || a > 64 * E) continue;
        wave_sort_long<E>(col, r0, a, lane, dup);
    }
}

// Long rows of (lo, NMAX] entries, one workgroup per row: the row is loaded
// into LDS, padded to a power of two with INT32_MAX, sorted by a bitonic
// network (one barrier per stage) and written back; equal neighbours after
// the sort are repeated entries.
template <int THREADS, int NMAX>
__global__ __launch_bounds__(THREADS) void k_long_sort(const int64_t *__restrict__ off, int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ long_rows, int64_t L, int32_t lo,
                                                       int32_t hi, unsigned int *__restrict__ dup) {
    __shared__ int32_t v[NMAX];
    const int tid = threadIdx.x;
    for (int64_t i = blockIdx.x; i < L; i += gridDim.x) {
        const int32_t r = long_rows[i];
        const int64_t r0 = off[r];
        const int32_t a = (int32_t)(off[r + 1] - r0);
        if (a <= lo || a > hi) continue;  // the same in every thread of the block
        int n = 64;
        while (n < a) n <<= 1;
        for (int p = tid; p < n; p += THREADS) v[p] = p < a ? col[r0 + p] : INT32_MAX;
        __syncthreads();
        for (int k = 2; k <= n; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = tid; t < (n >> 1); t += THREADS) {
                    const int x = ((t & ~(j - 1)) << 1) | (t & (j - 1)), y = x + j;
                    const int32_t vx = v[x], vy = v[y];
                    if ((vx > vy) == ((x & k) == 0)) {
                        v[x] = vy;
                        v[y] = vx;
                    }
                }
                __syncthreads();
            }
        }
        bool rep = false;
        for (int p = tid; p < a; p += THREADS) {
            const int32_t x = v[p];
            col[r0 + p] = x;
            rep |= p > 0 && v[p - 1] == x;
        }
        note_repeat(rep, dup);
        __syncthreads();
    }
}

__global__ void k_long_write(const uint64_t *__restrict__ keys, int64_t E, int gb, const int64_t *__restrict__ off,
                             const int32_t *__restrict__ long_rows, const int64_t *__restrict__ epos,
                             int32_t *__restrict__ col, unsigned int *__restrict__ dup) {
    const uint64_t mask = (1ull << gb) - 1;
    bool rep = false;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < E; q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[q];
        const int64_t i = (int64_t)(k >> gb);
        col[off[long_rows[i]] + (q - epos[i])] = (int32_t)(k & mask);
        rep |= q > 0 && keys[q - 1] == k;  // (row, entry) keys: equal neighbours repeat an entry
    }
    note_repeat(rep, dup);
}

// Step 6a: per-node cost f (degree-order labels) over stored pairs (s, t).
//   kind PRIOR: f[s] += dhat_s + dhat_t;   kind NEW: f[t] += dhat_t + dhat_s.
__global__ void k_row_lengths(const int64_t *__restrict__ off, int64_t N, int32_t *__restrict__ dh) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x)
        dh[r] = (int32_t)(off[r + 1] - off[r]);
}

__global__ void k_edge_costs(const int32_t *__restrict__ dh, const uint64_t *__restrict__ okeys, int64_t m, int gb,
                             int kind, int64_t *__restrict__ f) {
    const uint64_t mask = (1ull << gb) - 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
        const int64_t i = base + threadIdx.x;
        int64_t s = -1 - (int64_t)threadIdx.x;
        int64_t c = 0;
        int64_t t = 0;
        if (i < m) {
            const uint64_t k = okeys[i];
            s = (int64_t)(k >> gb);
            t = (int64_t)(k & mask);
            c = (int64_t)dh[s] + (int64_t)dh[t];
        }
        if (kind == TC_COST_PRIOR) {
            bool end;
            const int64_t sum = run_sum_at_end<int64_t>(s, c, &end);
            if (i < m && end) atomicAdd((unsigned long long *)&f[s], (unsigned long long)sum);
        } else if (i < m) {
            atomicAdd((unsigned long long *)&f[t], (unsigned long long)c);
        }
    }
}

// Same costs computed row by row (used when the sorted pair keys are gone).
__global__ void k_row_costs(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ dh, int64_t N, int kind, int64_t *__restrict__ f) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = dh[r];
        if (kind == TC_COST_PRIOR) {
            int64_t sum = 0;
            for (int64_t p = off[r]; p < off[r + 1]; ++p) sum += a + (int64_t)dh[col[p]];
            atomicAdd((unsigned long long *)&f[r], (unsigned long long)sum);
        } else {
            for (int64_t p = off[r]; p < off[r + 1]; ++p) {
                const int32_t t = col[p];
                atomicAdd((unsigned long long *)&f[t], (unsigned long long)(a + (int64_t)dh[t]));
            }
        }
    }
}

__global__ void k_gather_deg(const int32_t *__restrict__ deg_old, const int32_t *__restrict__ perm, int64_t N,
                             int32_t *__restrict__ deg_rank) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x)
        deg_rank[r] = deg_old[perm[r]];
}

// Step 6b: finish f for the per-node kinds, mask lists handled by whole
// workgroups (their work is scheduled separately), flag them, and find the
// longest list.
__global__ void k_node_costs(const int64_t *__restrict__ off, const int32_t *__restrict__ deg_rank, int64_t N,
                             int kind, int small_max, int med_max, int64_t *__restrict__ f,
                             uint32_t *__restrict__ wide_med, uint32_t *__restrict__ wide_large,
                             int32_t *__restrict__ max_dhat) {
    int32_t local_max = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t dh = off[r + 1] - off[r];
        local_max = max(local_max, (int32_t)dh);
        int64_t c = f[r];
        if (kind == TC_COST_ONE) c = 1;
        if (kind == TC_COST_DEGREE) c = deg_rank[r];
        const bool w = dh > small_max;
        f[r] = w ? 0 : c;
        wide_med[r] = (w && dh <= med_max) ? 1u : 0u;
        wide_large[r] = (w && dh > med_max) ? 1u : 0u;
    }
    // one atomic per workgroup: atomics to one address are serialised
    __shared__ int32_t wmax[kThreads / 64];
    local_max = wave_reduce_max(local_max);
    if (__lane_id() == 0) wmax[threadIdx.x >> 6] = local_max;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = 0;
        for (int w = 0; w < kThreads / 64; ++w) m = max(m, wmax[w]);
        atomicMax(max_dhat, m);
    }
}

// out[0..3] = *a, *b, *c, *d; out[4], out[5] = *e0, *e1 (0 for NULL pointers)
__global__ void k_totals(const int64_t *a, const int64_t *b, const int64_t *c, const int32_t *d, const uint32_t *e0,
                         const uint32_t *e1, int64_t *out) {
    if (threadIdx.x == 0) {
        out[0] = *a;
        out[1] = *b;
        out[2] = *c;
        out[3] = d ? (int64_t)*d : 0;
        out[4] = e0 ? (int64_t)*e0 : 0;
        out[5] = e1 ? (int64_t)*e1 : 0;
    }
}

__global__ void k_compact_index(const uint32_t *__restrict__ flag, const int64_t *__restrict__ pos, int64_t n,
                                int32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) out[pos[i]] = (int32_t)i;
}

// Step 6c: task boundaries.  bnd[0] = 0; bnd[j+1] = first x with F[x] >= target[j]
// (target < 0 encodes "end": x = N).
__global__ void k_task_bounds(const int64_t *__restrict__ F, int64_t N, const int64_t *__restrict__ target,
                              int64_t ntargets, int32_t *__restrict__ bnd) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= ntargets;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (j == 0) {
            bnd[0] = 0;
            continue;
        }
        const int64_t tg = target[j - 1];
        int64_t x = N;
        if (tg >= 0) {
            int64_t lo = 0, hi = N;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (F[mid] >= tg)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            x = lo;
        }
        bnd[j] = (int32_t)x;
    }
}

// Step 6d (k > 1): merge interior graph starts into the boundaries, so no
// task spans two graphs, and record each task's graph.
__global__ void k_merge_bounds(const int32_t *__restrict__ bnd, int64_t nb1, const int64_t *__restrict__ node_base,
                               int k, int32_t *__restrict__ out) {
    const int64_t total = nb1 + (k - 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nb1) {
            const int64_t v = bnd[i];
            // interior starts strictly below v come first
            int lo = 1, hi = k;  // interior starts are node_base[1..k-1]
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (node_base[mid] < v)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (i + (lo - 1) < total) out[i + (lo - 1)] = (int32_t)v;
        } else {
            const int g = (int)(i - nb1) + 1;
            const int64_t v = node_base[g];
            // boundaries <= v come first
            int64_t lo = 0, hi = nb1;
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (bnd[mid] <= v)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo + (g - 1) < total) out[lo + (g - 1)] = (int32_t)v;
        }
    }
}

// Step 6e: where each task's scan begins.  A node of degree 0 or 1 has no
// pair of neighbours, hence no triangle to count; in the degree order such
// nodes lead every graph, and a task reaching into that block (for a graph
// with many isolated nodes, one task can hold millions of them, all of cost
// 0) would scan it node by node.  Degrees never decrease inside a task, so
// one wave per task finds its first node of degree >= 2 by a 64-way search.
__global__ void k_task_starts(const int32_t *__restrict__ bnd, int64_t tasks, const int32_t *__restrict__ deg,
                              int32_t *__restrict__ start) {
    const int lane = __lane_id();
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; c < tasks; c += nw) {
        // the answer lies in [lo, hi]; hi means "none below hi"
        int64_t lo = bnd[c], hi = bnd[c + 1];
        if (lo < hi && deg[lo] < 2) {
            while (hi - lo > 64) {
                const int64_t step = (hi - lo + 63) / 64;  // 64 probes cover [lo, hi)
                const int64_t p = min(lo + lane * step, hi - 1);
                const uint64_t b = __ballot(deg[p] >= 2);
                if (!b) {
                    lo = min(lo + 63 * step, hi - 1) + 1;
                } else {
                    const int j = __ffsll((unsigned long long)b) - 1;
                    const int64_t pj = min(lo + j * step, hi - 1);
                    lo = j > 0 ? min(lo + (j - 1) * step, hi - 1) + 1 : lo;
                    hi = pj;
                }
            }
            const int64_t p = lo + lane;
            const uint64_t b = __ballot(p < hi && deg[p] >= 2);
            lo = b ? lo + __ffsll((unsigned long long)b) - 1 : hi;
        }
        if (lane == 0) start[c] = (int32_t)lo;
    }
}

__global__ void k_task_graph(const int32_t *__restrict__ bnd, int64_t ntasks, const int64_t *__restrict__ node_base,
                             int k, int32_t *__restrict__ gid) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ntasks; c += (int64_t)gridDim.x * blockDim.x) {
        int g = upper_bound_i64(node_base, k + 1, (int64_t)bnd[c]) - 1;
        gid[c] = g < 0 ? 0 : (g > k - 1 ? k - 1 : g);
    }
}

template <class T>
void d2h(T *host, const T *dev, size_t count, hipStream_t s) {
    TC_HIP(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, s));
}

}  // namespace

void fill_zero(void *p, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)((bytes + 3) / 4);
    if (words <= 0) return;
    k_fill_zero_u32<<<grid_for(words, 4), kThreads, 0, s>>>((uint32_t *)p, words);
    TC_LAUNCH_CHECK();
}

// Eq. (1)/(2) cost targets: initial W targets ceil((i+1) H / W) with
// H = ceil(total/2); then C += max(ceil((total - C) / W), min_chunk) until C
// reaches total, which ends the last task at the end of the node range
// (encoded as -1).  The division by W uses a precomputed reciprocal.
std::vector<int64_t> task_targets(int64_t total, int32_t W, int64_t min_chunk, bool static_chunks) {
    std::vector<int64_t> t;
    if (static_chunks) {
        // comparison schedule: W tasks of equal cost, no shrinking tail
        for (int32_t i = 0; i + 1 < W; ++i)
            t.push_back((int64_t)(((unsigned __int128)(i + 1) * (uint64_t)total + W - 1) / W));
        t.push_back(-1);
        return t;
    }
    const int64_t H = (total + 1) / 2;
    const uint64_t w = (uint64_t)W;
    const uint64_t magic = ~0ull / w;  // floor((2^64 - 1) / W)
    auto ceil_div_w = [&](uint64_t r) -> uint64_t {
        uint64_t q = (uint64_t)(((unsigned __int128)r * magic) >> 64);
        uint64_t rem = r - q * w;
        while (rem >= w) {
            ++q;
            rem -= w;
        }
        return q + (rem != 0);
    };
    t.reserve((size_t)W * 8 + 16);
    for (int32_t i = 0; i < W; ++i) t.push_back((int64_t)ceil_div_w((uint64_t)(i + 1) * (uint64_t)H));
    int64_t C = H;
    while (C < total) {
        int64_t step = (int64_t)ceil_div_w((uint64_t)(total - C));
        if (step < min_chunk) step = min_chunk;
        C += step;
        t.push_back(C >= total ? -1 : C);
    }
    if (t.back() != -1) t.push_back(-1);
    return t;
}

namespace {
// Page-locked staging for small host-to-device uploads (grown on demand, kept
// for the life of the thread; each build synchronises before returning).
struct PinnedStage {
    void *p = nullptr;
    size_t cap = 0;
    void *get(size_t bytes) {
        if (bytes > cap) {
            if (p) (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
            const size_t want = std::max<size_t>(bytes, 1 << 20);
            if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                return nullptr;
            }
            cap = want;
        }
        return p;
    }
};
thread_local PinnedStage t_stage;
thread_local PinnedStage t_total;  // the early cost total and the entries of the wide rows
// Largest number of entries in rows longer than small_max for which the early
// cost total is made (about 0.1 ms of gathers on MI355X).
constexpr int64_t kEarlyWide = (int64_t)8 << 20;
thread_local PinnedStage t_words;  // small results read back at a synchronisation
thread_local PinnedStage t_bases;  // node and edge offsets of the packed graphs

// Copies count words from dev to host through pinned memory (one small copy)
// and waits for it.
template <class T>
void read_words(T *host, const T *dev, size_t count, hipStream_t s) {
    void *pin = t_words.get(count * sizeof(T));
    TC_HIP(hipMemcpyAsync(pin ? pin : (void *)host, dev, count * sizeof(T), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (pin) std::memcpy(host, pin, count * sizeof(T));
}

struct EventGuard {
    hipEvent_t e = nullptr;
    ~EventGuard() {
        if (e) (void)hipEventDestroy(e);
    }
};
}  // namespace

// Row sort in two parts.  sort_rows_begin enqueues the sort of every row of up
// to kMidRow entries and, with f non-null, the PRIOR cost of every row (dh:
// row lengths); longer rows are listed in long_rows / nlong.  sort_rows_finish
// sorts the L listed rows (L read from nlong by the caller).  Nothing in
// between waits for the device.
struct LongRows {
    DevBuf<int32_t> rows;
    DevBuf<unsigned int> n;
};

void sort_rows_begin(const int64_t *off, int64_t N, int32_t *col, const int32_t *dh, int64_t *f,
                     unsigned int *dup, LongRows &lr, Allocator &tmp, hipStream_t s) {
    lr.rows = DevBuf<int32_t>(tmp, (size_t)std::max<int64_t>(N, 1));
    lr.n = DevBuf<unsigned int>(tmp, 1);
    fill_zero(lr.n.p, 4, s);
    if (N <= 0) return;
    const int64_t waves = std::min<int64_t>(ceil_div(N, 64), (int64_t)device_cu_count() * 64);
    k_sort_rows<<<(unsigned)ceil_div(waves * 64, kThreads), kThreads, 0, s>>>(off, N, col, lr.rows.p, lr.n.p, dh,
                                                                               f, dup);
    TC_LAUNCH_CHECK();
}

// ka / kb: scratch of cap keys each.
// max_row: the longest row (launches for longer classes are skipped).
void sort_rows_finish(const int64_t *off, int32_t *col, int gb, uint64_t *ka, uint64_t *kb, int64_t cap,
                      unsigned int *dup, const LongRows &lr, unsigned int L, int32_t max_row, Allocator &tmp,
                      hipStream_t s) {
    if (L == 0) return;
    const int32_t *long_rows = lr.rows.p;
    // rows of up to kLdsRowMax entries are sorted in LDS, longer ones (at most
    // sqrt(2m) entries in an oriented adjacency: only above ~1.3e8 edges) by
    // the radix sort of their (row, entry) keys; TC_LONG_ROW_LDS=<k> lowers
    // the LDS limit (testing)
    static const int32_t lds_rows = [] {
        const char *e = std::getenv("TC_LONG_ROW_LDS");
        return e && e[0] ? std::max(0, std::min(std::atoi(e), kLdsRowMax)) : kLdsRowMax;
    }();
    const int64_t sort_blocks = std::min<int64_t>(L, (int64_t)device_cu_count() * 16);
    if (lds_rows > kMidRow) {
        // kMidRow = 256 = 32 * 8: the three launches cover (256, 2048]
        static_assert(kMidRow == 32 * 8 && kLdsRowMid == 64 * 32, "long-row classes");
        const int32_t hi = std::min(lds_rows, kLdsRowMid);
        const int64_t waves = std::min<int64_t>(L, (int64_t)device_cu_count() * 32);
        const unsigned blocks = (unsigned)ceil_div(waves * 64, kThreads);
        k_long_sort_wave<8><<<blocks, kThreads, 0, s>>>(off, col, long_rows, L, hi, dup);
        TC_LAUNCH_CHECK();
        if (hi > 512 && max_row > 512) {
            k_long_sort_wave<16><<<blocks, kThreads, 0, s>>>(off, col, long_rows, L, hi, dup);
            TC_LAUNCH_CHECK();
        }
        if (hi > 1024 && max_row > 1024) {
            k_long_sort_wave<32><<<blocks, kThreads, 0, s>>>(off, col, long_rows, L, hi, dup);
            TC_LAUNCH_CHECK();
        }
    }
    if (lds_rows > kLdsRowMid && max_row > kLdsRowMid) {
        k_long_sort<1024, kLdsRowMax><<<(unsigned)sort_blocks, 1024, 0, s>>>(off, col, long_rows, L, kLdsRowMid,
                                                                             lds_rows, dup);
        TC_LAUNCH_CHECK();
    }
    DevBuf<int64_t> len(tmp, L), epos(tmp, (size_t)L + 1);
    k_long_lengths<<<grid_for(L), kThreads, 0, s>>>(off, long_rows, L, std::max(lds_rows, kMidRow), len.p);
    TC_LAUNCH_CHECK();
    exclusive_scan(len.p, epos.p, L, true, tmp, s);
    int64_t E = 0;
    d2h(&E, epos.p + L, 1, s);
    TC_HIP(hipStreamSynchronize(s));
    if (E == 0) return;
    if (E > cap) throw Error(TC_ERR_DEVICE, "long-row scratch smaller than the long rows");
    const int64_t lw = std::min<int64_t>(L, (int64_t)device_cu_count() * 64);
    k_long_keys<<<(unsigned)ceil_div(lw * 64, kThreads), kThreads, 0, s>>>(off, col, long_rows, epos.p, L, gb, ka);
    TC_LAUNCH_CHECK();
    const int lb = std::max(1, bits_for((uint64_t)(L - 1)));
    uint64_t *sorted = radix_sort_u64(ka, kb, E, 0, gb + lb, tmp, s);
    k_long_write<<<grid_for(E, 4), kThreads, 0, s>>>(sorted, E, gb, off, long_rows, epos.p, col, dup);
    TC_LAUNCH_CHECK();
}

// Both parts with the long-row count read in between.
void sort_rows(const int64_t *off, int64_t N, int32_t *col, int gb, uint64_t *ka, uint64_t *kb, int64_t cap,
               unsigned int *dup, int32_t max_row, Allocator &tmp, hipStream_t s) {
    LongRows lr;
    sort_rows_begin(off, N, col, nullptr, nullptr, dup, lr, tmp, s);
    unsigned int L = 0;
    d2h(&L, lr.n.p, 1, s);
    TC_HIP(hipStreamSynchronize(s));
    sort_rows_finish(off, col, gb, ka, kb, cap, dup, lr, L, max_row, tmp, s);
}

void build_into(const int32_t *src, const int32_t *dst, const Packing &pk, const BuildParams &bp, Allocator &al,
                Allocator &tmp, hipStream_t s, Oriented &out);
void schedule_into(const Packing &pk, const BuildParams &bp, Allocator &al, Allocator &tmp, hipStream_t s,
                   Oriented &out, const uint64_t *okeys, int gb, int64_t *f_prior = nullptr,
                   PresetTargets *pre = nullptr, Piggyback *pb = nullptr);

// samp[j] = col[j * kSampleStride]: the first level of the one-wave kernel's
// binary searches in long rows (a few MB that stay cached, so a search reads
// one line of col instead of several)
__global__ void k_sample_col(const int32_t *__restrict__ col, int64_t ns, int32_t *__restrict__ samp) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += (int64_t)gridDim.x * blockDim.x)
        samp[j] = col[j << kSampleShift];
}

// Dense core.  The rows at the end of the degree order belong to the nodes of
// highest degree; every member of such a row u lies in (u, N), a range so
// short that the row fills a good share of it.  From the first row among the
// last kCoreScan that holds kCoreMinRow entries or more and fills at least
// 1/kCoreDensity of (u, N), the adjacency among those last labels is kept as
// bitmaps too (the layout of core_origin), at most min(2 M, 1 GiB) bytes in
// all: a test of one id then reads one word, and two rows meet by AND-ing
// words.
constexpr int64_t kCoreScan = (int64_t)1 << 17;
constexpr int kCoreMinRow = 32;
constexpr int64_t kCoreMaxWords = (int64_t)1 << 28;

// far[0] = max of N - u over the qualifying rows u >= u0 (0: none); far[1] =
// 1 + the last row u >= u0 of 2 kCoreMinProbe entries or more (0: none)
__global__ void k_core_start(const int64_t *__restrict__ off, int64_t N, int64_t u0, int32_t *__restrict__ far) {
    const int64_t u = u0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool q = false, lng = false;
    if (u < N) {
        const int64_t L = off[u + 1] - off[u];
        q = L >= kCoreMinRow && kCoreDensity * L >= N - 1 - u;
        lng = L >= 2 * kCoreMinProbe;
    }
    const uint64_t b = __ballot(q), bl = __ballot(lng);
    // the first qualifying lane of the wave holds its smallest row, the last
    // long one its largest
    if (q && (int)__lane_id() == __builtin_ctzll(b)) atomicMax(&far[0], (int32_t)(N - u));
    if (lng && (int)__lane_id() == 63 - __builtin_clzll(bl)) atomicMax(&far[1], (int32_t)(u + 1));
}

// One wave per core row u: each entry x sets bit x in row u (the upper
// triangle; k_core_mirror fills the lower one).  A row is sorted, so the
// entries of one word sit in adjacent lanes; their bits are OR-ed across the
// lanes first and each word takes one atomic OR per wave.
__global__ __launch_bounds__(kThreads) void k_core_bits(const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ col, int64_t lo, int64_t N,
                                                        int64_t kw, uint32_t *__restrict__ bm) {
    const int lane = (int)__lane_id();
    const int64_t u = lo + ((int64_t)blockIdx.x * kThreads + threadIdx.x) / 64;
    if (u >= N) return;  // the whole wave
    const int64_t org = core_origin(u, lo, kw);
    const int64_t r1 = off[u + 1];
    for (int64_t e0 = off[u]; e0 < r1; e0 += 64) {
        const int64_t e = e0 + lane;
        const bool ok = e < r1;
        const int32_t x = ok ? col[e] : 0;
        const int32_t w = ok ? (int32_t)(org + (x >> 5)) : -1 - lane;  // distinct keys past the row
        uint32_t bits = ok ? 1u << (x & 31) : 0u;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t ob = __shfl_up(bits, d, 64);
            const int32_t ow = __shfl_up(w, d, 64);
            if (lane >= d && ow == w) bits |= ob;
        }
        const int32_t nw = __shfl_down(w, 1, 64);
        if (ok && (lane == 63 || nw != w)) atomicOr(&bm[w], bits);
    }
}

// 32 x 32 bit transpose across the 32 lanes of a half-wave: lane r holds row
// r; afterwards lane r holds bit r of every row k at bit k.
__device__ __forceinline__ uint32_t transpose32(uint32_t w, int r) {
    constexpr uint32_t kHi[5] = {0xFFFF0000u, 0xFF00FF00u, 0xF0F0F0F0u, 0xCCCCCCCCu, 0xAAAAAAAAu};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int j = 16 >> q;
        const uint32_t o = __shfl_xor(w, j, 32);
        w = (r & j) ? (w & kHi[q]) | ((o & kHi[q]) >> j) : (w & ~kHi[q]) | ((o & ~kHi[q]) << j);
    }
    return w;
}

// Index t of the upper triangle (b <= c) of an n x n grid, row-major, as (b, c):
// counted from the end, q = pairs - 1 - t lies in the row of k = n - b pairs
// with k (k - 1) / 2 <= q < k (k + 1) / 2.
__device__ __forceinline__ void upper_pair(int64_t t, int64_t n, int64_t *b, int64_t *c) {
    const int64_t q = n * (n + 1) / 2 - 1 - t;
    int64_t k = (int64_t)((sqrt(8.0 * (double)q + 1.0) + 1.0) * 0.5);
    while (k > 1 && k * (k - 1) / 2 > q) --k;
    while (k * (k + 1) / 2 <= q) ++k;
    *b = n - k;
    *c = n - 1 - (q - k * (k - 1) / 2);
}

// The lower triangle as the mirror of the upper one.  Block (b, c) holds the
// rows of labels 32 (b0 + b) .. + 31 and their word of labels 32 (b0 + c) ..
// + 31 (b0 = lo >> 5).  A workgroup takes a tile of kMirG x kMirG blocks, row
// blocks B kMirG .. and word columns C kMirG .. with B <= C: it stages the tile
// in LDS (each row's kMirG words read together), transposes every block in
// place, half-wave by half-wave (blocks (i, j) and (j, i) swap their
// transposes), and writes the result as the tile of row blocks C kMirG .. and
// word columns B kMirG .. (a tile on the diagonal: OR-ed into itself, its
// upper blocks then holding both halves).  Rows below lo do not exist.
constexpr int kMirG = 16;
constexpr int kMirRows = 32 * kMirG;
constexpr int kMirPad = kMirG + 1;  // LDS row stride: the block reads hit distinct banks

__global__ __launch_bounds__(kThreads) void k_core_mirror(int64_t lo, int64_t N, int64_t kw, int64_t nb,
                                                          int64_t ng, uint32_t *__restrict__ bm) {
    __shared__ uint32_t A[kMirRows * kMirPad];
    int64_t B, C;
    upper_pair(blockIdx.x, ng, &B, &C);
    const bool diag = B == C;
    const int64_t b0 = lo >> 5;
    for (int idx = threadIdx.x; idx < kMirRows * kMirG; idx += kThreads) {
        const int row = idx / kMirG, col = idx % kMirG;
        const int64_t bi = B * kMirG + row / 32, cj = C * kMirG + col;
        const int64_t ru = (b0 + bi) * 32 + (row & 31);
        uint32_t w = 0u;
        if (bi < nb && cj < nb && ru >= lo && ru < N) w = bm[core_origin(ru, lo, kw) + b0 + cj];
        A[row * kMirPad + col] = w;
    }
    __syncthreads();
    const int r = (int)(threadIdx.x & 31);
    for (int p = (int)(threadIdx.x >> 5); p < kMirG * (kMirG + 1) / 2; p += kThreads / 32) {
        int i = 0, rem = p;  // p -> (i, j), i <= j
        while (rem >= kMirG - i) {
            rem -= kMirG - i;
            ++i;
        }
        const int j = i + rem;
        const uint32_t x = A[(i * 32 + r) * kMirPad + j], y = A[(j * 32 + r) * kMirPad + i];
        const uint32_t tx = transpose32(x, r), ty = transpose32(y, r);
        if (i == j) {
            A[(i * 32 + r) * kMirPad + j] = diag ? x | tx : tx;
        } else {
            A[(i * 32 + r) * kMirPad + j] = diag ? x | ty : ty;
            A[(j * 32 + r) * kMirPad + i] = diag ? y | tx : tx;
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kMirRows * kMirG; idx += kThreads) {
        const int row = idx / kMirG, col = idx % kMirG;
        const int64_t bi = C * kMirG + row / 32, cj = B * kMirG + col;
        const int64_t rv = (b0 + bi) * 32 + (row & 31);
        if (bi < nb && cj < nb && rv >= lo && rv < N) bm[core_origin(rv, lo, kw) + b0 + cj] = A[row * kMirPad + col];
    }
}

// Words of the core from label lo on.
inline int64_t core_words(int64_t N, int64_t lo) {
    return lo >= N ? 0 : (N - lo) * (((N - 1) >> 5) - (lo >> 5) + 1);
}

// Builds the core of a one-graph handle without a device budget (else none).
// A core none of whose rows holds 2 kCoreMinProbe entries is left out: its
// rows are too short for the bit tests, and no list in it is long enough for
// the workgroup kernels' AND.
void build_core(const Packing &pk, const BuildParams &bp, Allocator &al, hipStream_t s, Oriented &out) {
    const int64_t N = pk.N;
    out.core = Oriented::CoreLayout{};
    out.core.lo = (int32_t)N;
    if (!bp.core || pk.k != 1 || al.budget || out.M == 0 || N < 2) return;
    const int64_t u0 = std::max<int64_t>(0, N - kCoreScan);
    DevBuf<int32_t> far(al, 2);
    fill_zero(far.p, 8, s);
    k_core_start<<<grid_for(N - u0), kThreads, 0, s>>>(out.off.p, N, u0, far.p);
    TC_LAUNCH_CHECK();
    int32_t hfar[2] = {0, 0};
    read_words(hfar, far.p, 2, s);
    if (hfar[0] <= 0) return;
    int64_t lo = N - hfar[0];
    const int64_t cap = std::min<int64_t>(kCoreMaxWords, out.M / 2);
    if (core_words(N, lo) > cap) {
        int64_t a = lo, b = N;  // smallest first label whose core fits the cap
        while (a < b) {
            const int64_t mid = a + (b - a) / 2;
            if (core_words(N, mid) <= cap)
                b = mid;
            else
                a = mid + 1;
        }
        lo = a;
    }
    const int64_t words = core_words(N, lo);
    if (lo >= N || words <= 0 || (int64_t)hfar[1] - 1 < lo) return;
    out.bm = DevBuf<uint32_t>(al, (size_t)words);
    fill_zero(out.bm.p, (size_t)words * 4, s);
    out.core.lo = (int32_t)lo;
    out.core.wl = (int32_t)((N - 1) >> 5);
    out.core.kw = (int32_t)(out.core.wl - (lo >> 5) + 1);
    out.core.words = words;
    k_core_bits<<<(unsigned)ceil_div((N - lo) * 64, (int64_t)kThreads), kThreads, 0, s>>>(
        out.off.p, out.col.p, lo, N, out.core.kw, out.bm.p);
    TC_LAUNCH_CHECK();
    const int64_t nb = out.core.kw, ng = ceil_div(nb, (int64_t)kMirG);
    k_core_mirror<<<(unsigned)(ng * (ng + 1) / 2), kThreads, 0, s>>>(lo, N, out.core.kw, nb, ng, out.bm.p);
    TC_LAUNCH_CHECK();
}

void build_oriented_device(const int32_t *src, const int32_t *dst, const Packing &pk, const BuildParams &bp,
                           Allocator &al, hipStream_t s, Oriented &out) {
    const int64_t N = pk.N, M_in = pk.M_in;
    // One scratch region for every temporary of the build (bump allocation),
    // sized from the input: keys 16 B/edge, sort tables < 4 B/edge,
    // node arrays < 80 B/node, task targets.
    const size_t arena_bytes = (size_t)M_in * 20 + (size_t)N * 80 + (size_t)bp.workers * 128 + (8u << 20);
    void *arena = al.get(arena_bytes);
    Allocator tmp = al;
    tmp.arena = (uint8_t *)arena;
    tmp.arena_size = arena_bytes;
    tmp.arena_used = 0;
    try {
        build_into(src, dst, pk, bp, al, tmp, s, out);
    } catch (...) {
        al.put(arena, arena_bytes);
        throw;
    }
    al.put(arena, arena_bytes);
    const int64_t ns = ceil_div(out.M, kSampleStride);
    out.samp = DevBuf<int32_t>(al, (size_t)std::max<int64_t>(ns, 1));
    if (ns > 0) {
        k_sample_col<<<grid_for(ns, 4), kThreads, 0, s>>>(out.col.p, ns, out.samp.p);
        TC_LAUNCH_CHECK();
    }
    build_core(pk, bp, al, s, out);
}

namespace {
void add_endpoint_counts(const uint64_t *keys, int64_t M, int gb, int32_t *deg, int64_t N, uint32_t *spare,
                         Allocator &tmp, hipStream_t s);
void add_pair_counts(const int32_t *src, const int32_t *dst, int64_t M, int gb, int32_t *deg, int64_t N,
                     uint32_t *spare, Allocator &tmp, hipStream_t s, bool runs_src, bool runs_dst);
}  // namespace

// One build.  simple: the input is taken to be a simple graph (no edge
// twice, no loop): degrees are counted from the endpoints as given and the
// canonical sort is skipped.  Returns false when that assumption fails (a
// loop in the input, or a repeated entry in a sorted row); out is then
// incomplete and the caller builds again without it.
static bool build_pass(const int32_t *src, const int32_t *dst, const Packing &pk, const BuildParams &bp,
                       Allocator &al, Allocator &tmp, hipStream_t s, Oriented &out, bool simple) {
    const int64_t N = pk.N, M_in = pk.M_in;
    const int k = pk.k;
    const int gb = std::max(1, bits_for((uint64_t)std::max<int64_t>(N - 1, 1)));  // bits of a packed label

    out.node_base = DevBuf<int64_t>(al, (size_t)k + 1);
    DevBuf<int64_t> edge_base(tmp, (size_t)k + 1);
    {
        // both tables in one copy from pinned memory (a copy from pageable
        // memory is staged and waited for); the staging is free again at the
        // check pass's read-back, before any later build writes it
        const size_t bytes = (size_t)(k + 1) * sizeof(int64_t);
        auto *pin = static_cast<int64_t *>(t_bases.get(2 * bytes));
        if (pin) {
            std::memcpy(pin, pk.node_base.data(), bytes);
            std::memcpy(pin + (k + 1), pk.edge_base.data(), bytes);
            TC_HIP(hipMemcpyAsync(out.node_base.p, pin, bytes, hipMemcpyHostToDevice, s));
            TC_HIP(hipMemcpyAsync(edge_base.p, pin + (k + 1), bytes, hipMemcpyHostToDevice, s));
        } else {
            TC_HIP(hipMemcpyAsync(out.node_base.p, pk.node_base.data(), bytes, hipMemcpyHostToDevice, s));
            TC_HIP(hipMemcpyAsync(edge_base.p, pk.edge_base.data(), bytes, hipMemcpyHostToDevice, s));
        }
    }
    DevBuf<uint32_t> err(tmp, 4);  // [0]: input errors, [1]: repeated entry
    fill_zero(err.p, 16, s);

    // ---- 1. canonical edge set
    int64_t M = 0;
    DevBuf<uint64_t> ka(tmp, (size_t)std::max<int64_t>(M_in, 1));
    DevBuf<uint64_t> kb(tmp, (size_t)std::max<int64_t>(M_in, 1));
    uint64_t *ukeys = kb.p;
    // one graph given as an edge list: the ids are the labels, so a simple
    // input needs no pair keys at all (degrees and orientation read it)
    const bool pairs = simple && k == 1;
    bool runs_src = false, runs_dst = false;
    if (M_in > 0 && pairs) {
        const unsigned nblk = std::min<unsigned>(grid_for(M_in, 4 * kEdgeUnroll), kCheckBlocks);
        DevBuf<unsigned long long> chk(tmp, 2 + 2 * (size_t)nblk);
        fill_zero(chk.p, 16, s);
        k_check_pairs<<<nblk, kThreads, 0, s>>>(src, dst, M_in, N, chk.p);
        TC_LAUNCH_CHECK();
        DevBuf<unsigned long long> sums(tmp, 3);
        k_check_sums<<<1, kThreads, 0, s>>>(chk.p, nblk, sums.p);
        TC_LAUNCH_CHECK();
        unsigned long long hc[3] = {0, 0, 0};
        read_words(hc, sums.p, 3, s);
        if (hc[0] & 1u) throw Error(TC_ERR_ID_RANGE, "an edge endpoint is outside 0..n-1 of its graph");
        if (hc[0] & 2u) return false;  // a loop: take the canonical path
        const unsigned long long bs = hc[1], bd = hc[2];
        // count runs when they average 4 or more edges
        runs_src = (int64_t)bs * 4 <= M_in;
        runs_dst = (int64_t)bd * 4 <= M_in;
        M = M_in;
    } else if (M_in > 0) {
        // the canonical path sorts the keys next: they come with the first
        // radix pass's digit table
        const int64_t tiles = ceil_div(M_in, (int64_t)kRadixTile);
        const int bits0 = std::min(8, 2 * gb);
        DevBuf<uint32_t> h0(tmp, simple ? 1 : (size_t)tiles * 256);
        if (simple) {
            k_edge_keys<<<grid_for(M_in, 4 * kEdgeUnroll), kThreads, 0, s>>>(src, dst, M_in, edge_base.p,
                                                                              out.node_base.p, k, gb, ka.p, err.p);
        } else {
            k_edge_keys_hist<<<(unsigned)tiles, kOrientTileThreads, 0, s>>>(
                src, dst, M_in, edge_base.p, out.node_base.p, k, gb, ka.p, err.p, bits0, tiles, h0.p);
        }
        TC_LAUNCH_CHECK();
        uint32_t herr = 0;
        if (simple) {
            d2h(&herr, err.p, 1, s);
            TC_HIP(hipStreamSynchronize(s));
            if (herr & 1u) throw Error(TC_ERR_ID_RANGE, "an edge endpoint is outside 0..n-1 of its graph");
            if (herr & 2u) return false;  // a loop: take the canonical path
            M = M_in;
            ukeys = ka.p;
        } else {
            uint64_t *sorted = radix_sort_u64_hist(ka.p, kb.p, M_in, 0, 2 * gb, h0.p, tmp, s);
            uint64_t *other = sorted == ka.p ? kb.p : ka.p;
            M = unique_sorted_keys(sorted, M_in, other, &ukeys, tmp, s);  // synchronises
            d2h(&herr, err.p, 1, s);
            TC_HIP(hipStreamSynchronize(s));
            if (herr & 1u) throw Error(TC_ERR_ID_RANGE, "an edge endpoint is outside 0..n-1 of its graph");
        }
    }
    out.M = M;
    uint64_t *spare = ukeys == ka.p ? kb.p : ka.p;

    // ---- 2. degrees
    DevBuf<int32_t> deg(tmp, (size_t)std::max<int64_t>(N, 1));
    fill_zero(deg.p, deg.bytes(), s);
    if (pairs)
        add_pair_counts(src, dst, M, gb, deg.p, N, reinterpret_cast<uint32_t *>(spare), tmp, s, runs_src, runs_dst);
    else if (simple)
        add_endpoint_counts(ukeys, M, gb, deg.p, N, reinterpret_cast<uint32_t *>(spare), tmp, s);
    else
        add_degrees(ukeys, M, gb, deg.p, N, reinterpret_cast<uint32_t *>(spare), tmp, s);  // spare: >= 2 M words

    // ---- 3. degree order
    out.perm = DevBuf<int32_t>(al, (size_t)std::max<int64_t>(N, 1));
    DevBuf<int32_t> rank(tmp, (size_t)std::max<int64_t>(N, 1));
    degree_rank(deg.p, N, out.node_base.p, k, pk.max_n, out.perm.p, rank.p, tmp, s);

    // ---- 4. orientation, 5. CSR
    out.col = DevBuf<int32_t>(al, (size_t)std::max<int64_t>(M, 1));
    out.off = DevBuf<int64_t>(al, (size_t)N + 1);
    DevBuf<int32_t> rowlen(tmp, (size_t)std::max<int64_t>(N, 1));
    fill_zero(rowlen.p, rowlen.bytes(), s);
    uint64_t *okeys = nullptr;
    if (M > 0) {
        // order by s >> kGroupBits, then place each group of rows (in key
        // order inside a row: rows are sorted below)
        if (gb > kGroupBits) {
            // the keys come out in the radix passes' tiles with the first
            // pass's digit table, so that pass does not read them to count
            const int64_t tiles = ceil_div(M, (int64_t)kRadixTile);
            const int shift = gb + kGroupBits, bits = std::min(8, 2 * gb - shift);
            DevBuf<uint32_t> h1(tmp, (size_t)tiles * 256);
            if (pairs)
                k_orient_hist<false><<<(unsigned)tiles, kOrientTileThreads, 0, s>>>(
                    src, dst, nullptr, M, gb, rank.p, spare, shift, bits, tiles, h1.p);
            else
                k_orient_hist<true><<<(unsigned)tiles, kOrientTileThreads, 0, s>>>(
                    nullptr, nullptr, ukeys, M, gb, rank.p, spare, shift, bits, tiles, h1.p);
            TC_LAUNCH_CHECK();
            okeys = radix_sort_u64_hist(spare, ukeys, M, shift, 2 * gb, h1.p, tmp, s);
        } else {
            if (pairs)
                k_orient_pairs<<<grid_for(M, 4 * kOrientUnroll), kThreads, 0, s>>>(src, dst, M, gb, rank.p, spare);
            else
                k_orient_keys<<<grid_for(M, 4 * kOrientUnroll), kThreads, 0, s>>>(ukeys, M, gb, rank.p, spare);
            TC_LAUNCH_CHECK();
            okeys = spare;  // one group: no sort
        }
        const int64_t ngroups = ceil_div(N, (int64_t)kGroupRows);
        DevBuf<int64_t> gstart(tmp, (size_t)ngroups + 1);
        k_group_bounds<<<grid_for(ngroups + 1), kThreads, 0, s>>>(okeys, M, gb, ngroups, gstart.p);
        TC_LAUNCH_CHECK();
        // chunks of at most kChunkKeys keys per group; their number is only
        // known on the device, so the kernels loop over an upper bound
        DevBuf<int64_t> cfirst(tmp, (size_t)ngroups + 1);
        k_group_chunks<<<grid_for(ngroups), kThreads, 0, s>>>(gstart.p, ngroups, cfirst.p);
        TC_LAUNCH_CHECK();
        exclusive_scan(cfirst.p, cfirst.p, ngroups, true, tmp, s);  // in place: tile-local staging
        const int64_t max_chunks = ceil_div(M, kChunkKeys) + ngroups;
        DevBuf<uint32_t> cnt(tmp, (size_t)max_chunks * kGroupRows);
        const int64_t wg = (int64_t)device_cu_count() * 2;  // resident 1024-thread workgroups
        k_chunk_count<<<(unsigned)std::min<int64_t>(max_chunks, wg), kChunkThreads, 0, s>>>(okeys, gb, gstart.p,
                                                                                           cfirst.p, ngroups, cnt.p);
        TC_LAUNCH_CHECK();
        k_chunk_scan<<<(unsigned)std::min<int64_t>(ngroups, wg), kChunkThreads, 0, s>>>(
            gstart.p, cfirst.p, ngroups, N, cnt.p, rowlen.p, out.off.p);
        TC_LAUNCH_CHECK();
        k_chunk_place<<<(unsigned)std::min<int64_t>(max_chunks, wg), kChunkThreads, 0, s>>>(
            okeys, gb, gstart.p, cfirst.p, ngroups, N, cnt.p, out.off.p, out.col.p);
        TC_LAUNCH_CHECK();
    } else {
        exclusive_scan(rowlen.p, out.off.p, N, true, tmp, s);
    }

    // ---- 6. costs, wide lists, task table
    out.deg = DevBuf<int32_t>(al, (size_t)std::max<int64_t>(N, 1));
    if (N > 0) {
        k_gather_deg<<<grid_for(N, 4), kThreads, 0, s>>>(deg.p, out.perm.p, N, out.deg.p);
        TC_LAUNCH_CHECK();
    }
    uint32_t *dup = err.p + 1;
    if (bp.cost_fn == TC_COST_PRIOR && M > 0) {
        // The row sort adds up the PRIOR costs on the way.  Their total is
        // known before it (k_prior_total), so the host computes the task
        // targets while the device sorts.
        DevBuf<int64_t> f(tmp, (size_t)N);
        DevBuf<unsigned long long> acc(tmp, 2);
        fill_zero(acc.p, 16, s);
        const int64_t tw = std::min<int64_t>(ceil_div(N, 64), (int64_t)device_cu_count() * 8);  // waves
        // the early total is made when the rows longer than small_max hold at
        // most kEarlyWide entries (their costs need a gather per entry)
        // a few workgroups per CU: each adds its partial sums to the same two words
        k_prior_total<<<std::min<unsigned>(grid_for(N, 4), (unsigned)device_cu_count() * 4), kThreads, 0, s>>>(
            out.off.p, out.deg.p, N, bp.small_max, acc.p);
        TC_LAUNCH_CHECK();
        k_prior_wide<<<(unsigned)ceil_div(tw * 64, kThreads), kThreads, 0, s>>>(out.off.p, out.col.p, N,
                                                                                 bp.small_max, kEarlyWide, acc.p);
        TC_LAUNCH_CHECK();
        auto *htot = static_cast<unsigned long long *>(t_total.get(2 * sizeof(unsigned long long)));
        PresetTargets pre;
        EventGuard ev;
        if (htot) {
            TC_HIP(hipMemcpyAsync(htot, acc.p, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
            TC_HIP(hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
            TC_HIP(hipEventRecord(ev.e, s));
        }
        BuildParams bpr = bp;
        bpr.rounds = bp.rounds > 0 ? bp.rounds : auto_rounds(pk.k, M);
        LongRows lr;
        sort_rows_begin(out.off.p, N, out.col.p, rowlen.p, f.p, dup, lr, tmp, s);
        if (htot) {  // host work that overlaps the row sort
            TC_HIP(hipEventSynchronize(ev.e));
            if ((int64_t)htot[1] <= kEarlyWide) {
                pre.total = (int64_t)htot[0];
                pre.targets = schedule_targets(pre.total, bpr);
            }
        }
        // the task table is enqueued behind the row sort; the long-row count
        // and the repeat flag come back with the schedule's totals
        Piggyback pb;
        pb.dev[0] = lr.n.p;
        pb.dev[1] = dup;
        schedule_into(pk, bp, al, tmp, s, out, nullptr, gb, f.p, &pre, &pb);
        const unsigned int L = pb.host[0];
        if (L == 0) {
            TC_HIP(hipStreamSynchronize(s));
            return !(simple && pb.host[1]);  // an edge given twice: take the canonical path
        }
        sort_rows_finish(out.off.p, out.col.p, gb, ka.p, kb.p, M_in, dup, lr, L, out.max_dhat, tmp, s);
    } else {
        schedule_into(pk, bp, al, tmp, s, out, okeys, gb);
        if (M > 0) sort_rows(out.off.p, N, out.col.p, gb, ka.p, kb.p, M_in, dup, out.max_dhat, tmp, s);
    }
    if (simple && M > 0) {
        uint32_t hdup = 0;
        d2h(&hdup, dup, 1, s);
        TC_HIP(hipStreamSynchronize(s));
        if (hdup) return false;  // an edge given twice: take the canonical path
    }
    return true;
}

// Most inputs are simple graphs; for them the first pass is the build.  A
// loop or a repeated edge sends the build down the canonical path (sort and
// unique selection of the pairs) from the start.
void build_into(const int32_t *src, const int32_t *dst, const Packing &pk, const BuildParams &bp, Allocator &al,
                Allocator &tmp, hipStream_t s, Oriented &out) {
    const size_t mark = tmp.arena_used;
    if (build_pass(src, dst, pk, bp, al, tmp, s, out, true)) return;
    tmp.arena_used = mark;  // every scratch buffer of the first pass is released
    build_pass(src, dst, pk, bp, al, tmp, s, out, false);
}

// Step 6 proper.  okeys (sorted pair keys) speed up the edge costs when the
// build still holds them; otherwise costs are computed row by row.
void schedule_into(const Packing &pk, const BuildParams &bp, Allocator &al, Allocator &tmp, hipStream_t s,
                   Oriented &out, const uint64_t *okeys, int gb, int64_t *f_prior, PresetTargets *pre,
                   Piggyback *pb) {
    const int64_t N = pk.N, M = out.M;
    DevBuf<int64_t> f_own;
    int64_t *f = f_prior;  // PRIOR costs computed by the caller, else computed here
    if (!f_prior) {
        f_own = DevBuf<int64_t>(tmp, (size_t)std::max<int64_t>(N, 1));
        f = f_own.p;
        fill_zero(f, f_own.bytes(), s);
    }
    if (!f_prior && M > 0 && (bp.cost_fn == TC_COST_PRIOR || bp.cost_fn == TC_COST_NEW)) {
        DevBuf<int32_t> dh(tmp, (size_t)N);
        k_row_lengths<<<grid_for(N, 4), kThreads, 0, s>>>(out.off.p, N, dh.p);
        TC_LAUNCH_CHECK();
        if (okeys) {
            k_edge_costs<<<grid_for(M, 4), kThreads, 0, s>>>(dh.p, okeys, M, gb, bp.cost_fn, f);
        } else {
            k_row_costs<<<grid_for(N, 1), kThreads, 0, s>>>(out.off.p, out.col.p, dh.p, N, bp.cost_fn, f);
        }
        TC_LAUNCH_CHECK();
    }
    DevBuf<uint32_t> wmed(tmp, (size_t)std::max<int64_t>(N, 1)), wlarge(tmp, (size_t)std::max<int64_t>(N, 1));
    DevBuf<int32_t> maxd(tmp, 1);
    fill_zero(maxd.p, 4, s);
    if (N > 0) {
        k_node_costs<<<grid_for(N, 16), kThreads, 0, s>>>(out.off.p, out.deg.p, N, bp.cost_fn, bp.small_max,
                                                          max_medium_list(), f, wmed.p, wlarge.p, maxd.p);
        TC_LAUNCH_CHECK();
    }
    Schedule sc;
    BuildParams bpr = bp;
    bpr.rounds = bp.rounds > 0 ? bp.rounds : auto_rounds(pk.k, M);
    out.rounds = bpr.rounds;
    // labels follow the degree order inside each graph, so degrees never
    // decrease inside a task
    schedule_sources(f, wmed.p, wlarge.p, N, pk.k, out.node_base.p, bpr, al, tmp, s, sc, maxd.p, &out.max_dhat, pre,
                     out.deg.p, pb);
    out.bnd = std::move(sc.bnd);
    out.gid = std::move(sc.gid);
    out.start = std::move(sc.start);
    out.big = std::move(sc.big);
    out.tasks = sc.tasks;
    out.total_cost = sc.total_cost;
    out.nmed = sc.nmed;
    out.nbig = sc.nbig;
}

std::vector<int64_t> schedule_targets(int64_t total, const BuildParams &bp) {
    int64_t min_chunk = bp.min_chunk;
    if (min_chunk <= 0) {
        // automatic floor: about 1/64 of an initial task's cost, at least 256
        min_chunk = std::max<int64_t>(256, total / ((int64_t)bp.workers * 128 + 1));
    }
    const int64_t W = (int64_t)bp.workers * std::max(1, bp.rounds);
    if (W > INT32_MAX) throw Error(TC_ERR_INVALID_ARG, "workers * rounds too large");
    return task_targets(total, (int32_t)W, min_chunk, bp.static_chunks != 0);
}

void schedule_sources(const int64_t *f, const uint32_t *wmed, const uint32_t *wlarge, int64_t N, int k,
                      const int64_t *node_base, const BuildParams &bp, Allocator &al, Allocator &tmp, hipStream_t s,
                      Schedule &out, const int32_t *maxd_dev, int32_t *maxd_host, PresetTargets *pre,
                      const int32_t *deg_sorted, Piggyback *pb) {
    DevBuf<int64_t> F(tmp, (size_t)N + 1);
    DevBuf<int64_t> pmed(tmp, (size_t)N + 1), plarge(tmp, (size_t)N + 1);
    exclusive_scan(f, F.p, N, true, tmp, s);
    exclusive_scan(wmed, pmed.p, N, true, tmp, s);
    exclusive_scan(wlarge, plarge.p, N, true, tmp, s);
    // the three totals, the longest list and the caller's extra words in one copy
    int64_t hv[6] = {0, 0, 0, 0, 0, 0};
    DevBuf<int64_t> tot6(tmp, 6);
    k_totals<<<1, 64, 0, s>>>(F.p + N, pmed.p + N, plarge.p + N, maxd_dev, pb ? pb->dev[0] : nullptr,
                              pb ? pb->dev[1] : nullptr, tot6.p);
    TC_LAUNCH_CHECK();

    // task table from targets (bnd, and for k > 1 the merged bounds and graph
    // ids), then where each task's scan begins
    auto make_table = [&](const std::vector<int64_t> &tg) {
        const int64_t ntg = (int64_t)tg.size();
        DevBuf<int32_t> bnd(al, (size_t)ntg + 1);
        task_bounds(F.p, N, tg, bnd.p, tmp, s);
        if (k > 1) {
            const int64_t tot = ntg + 1 + (k - 1);
            out.bnd = DevBuf<int32_t>(al, (size_t)tot);
            k_merge_bounds<<<grid_for(tot), kThreads, 0, s>>>(bnd.p, ntg + 1, node_base, k, out.bnd.p);
            TC_LAUNCH_CHECK();
            out.tasks = tot - 1;
            out.gid = DevBuf<int32_t>(al, (size_t)out.tasks);
            k_task_graph<<<grid_for(out.tasks), kThreads, 0, s>>>(out.bnd.p, out.tasks, node_base, k, out.gid.p);
            TC_LAUNCH_CHECK();
        } else {
            out.bnd = std::move(bnd);
            out.gid = DevBuf<int32_t>();
            out.tasks = ntg;
        }
        out.start = DevBuf<int32_t>();
        if (deg_sorted && out.tasks > 0) {
            out.start = DevBuf<int32_t>(al, (size_t)out.tasks);
            k_task_starts<<<grid_for(out.tasks * 64), kThreads, 0, s>>>(out.bnd.p, out.tasks, deg_sorted,
                                                                         out.start.p);
            TC_LAUNCH_CHECK();
        }
    };
    // Targets computed ahead (from the early total) give the task table
    // before the totals come back; it stands if the totals agree.
    const int64_t ahead_total = pre ? pre->total : -1;
    if (ahead_total >= 0) make_table(pre->targets);

    // (also the point after which the pinned staging of the targets is free)
    read_words(hv, tot6.p, 6, s);
    if (pb) {
        pb->host[0] = (uint32_t)hv[4];
        pb->host[1] = (uint32_t)hv[5];
    }
    out.total_cost = hv[0];
    out.nmed = hv[1];
    out.nbig = hv[1] + hv[2];
    if (maxd_host) *maxd_host = (int32_t)hv[3];

    out.big = DevBuf<int32_t>(al, (size_t)std::max<int64_t>(out.nbig, 1));
    if (out.nmed > 0) {
        k_compact_index<<<grid_for(N, 4), kThreads, 0, s>>>(wmed, pmed.p, N, out.big.p);
        TC_LAUNCH_CHECK();
    }
    if (out.nbig > out.nmed) {
        k_compact_index<<<grid_for(N, 4), kThreads, 0, s>>>(wlarge, plarge.p, N, out.big.p + out.nmed);
        TC_LAUNCH_CHECK();
    }
    if (ahead_total != out.total_cost) {
        make_table(schedule_targets(out.total_cost, bp));
        // the pinned staging of the targets is reused by the next call
        TC_HIP(hipStreamSynchronize(s));
    }
    // Scratch buffers are released in stream order when this scope ends.
}

int32_t auto_rounds(int32_t k, int64_t M) {
    if (k <= 1) return 1;
    const int64_t r = ceil_div(M * 4, (int64_t)64 << 20);
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(r, 64));
}

void task_bounds(const int64_t *F, int64_t N, const std::vector<int64_t> &targets, int32_t *bnd, Allocator &tmp,
                 hipStream_t s) {
    const int64_t ntg = (int64_t)targets.size();
    DevBuf<int64_t> dtg(tmp, (size_t)std::max<int64_t>(ntg, 1));
    void *pin = t_stage.get((size_t)ntg * sizeof(int64_t));
    if (pin) {
        // the staging buffer is reused by the next call; every caller
        // synchronises the stream before that
        std::memcpy(pin, targets.data(), ntg * sizeof(int64_t));
        TC_HIP(hipMemcpyAsync(dtg.p, pin, ntg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    } else {
        TC_HIP(hipMemcpyAsync(dtg.p, targets.data(), ntg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    }
    k_task_bounds<<<grid_for(ntg + 1), kThreads, 0, s>>>(F, N, dtg.p, ntg, bnd);
    TC_LAUNCH_CHECK();
}

int64_t unique_sorted_keys(uint64_t *sorted, int64_t n, uint64_t *out, uint64_t **res, Allocator &tmp,
                           hipStream_t s) {
    *res = out;
    if (n <= 0) return 0;
    const int64_t nt = ceil_div(n, kSelTile);
    DevBuf<int64_t> part(tmp, (size_t)nt + 1);
    k_unique_count<<<(unsigned)nt, kThreads, 0, s>>>(sorted, n, part.p);
    TC_LAUNCH_CHECK();
    exclusive_scan(part.p, part.p, nt, true, tmp, s);
    int64_t M = 0;
    d2h(&M, part.p + nt, 1, s);
    TC_HIP(hipStreamSynchronize(s));
    if (M == n) {
        *res = sorted;  // no duplicates and no self-loops: already the set
        return M;
    }
    k_unique_write<<<(unsigned)nt, kThreads, 0, s>>>(sorted, n, part.p, out);
    TC_LAUNCH_CHECK();
    return M;
}

namespace {
// deg[x] += occurrences of x in vals[0..M) (labels below N < 2^gb): the
// values are grouped by bucket (label bits above kBinBits; vals_tmp holds M
// more), then each bucket is counted in LDS.
void histogram_add(uint32_t *vals, uint32_t *vals_tmp, int64_t M, int gb, int32_t *deg, int64_t N, Allocator &tmp,
                   hipStream_t s, const uint32_t *first = nullptr) {
    // with first given, the values are read from it (vals: scratch)
    const uint32_t *hs;
    if (first)
        hs = gb > kBinBits ? radix_sort_u32_from(first, vals, vals_tmp, M, kBinBits, gb, tmp, s) : first;
    else
        hs = gb > kBinBits ? radix_sort_u32(vals, vals_tmp, M, kBinBits, gb, tmp, s) : vals;
    const int64_t nbuckets = gb > kBinBits ? (int64_t)1 << (gb - kBinBits) : 1;
    DevBuf<int64_t> bstart(tmp, (size_t)nbuckets + 1), cstart(tmp, (size_t)nbuckets + 1);
    DevBuf<int32_t> parts(tmp, (size_t)nbuckets);
    k_val_bucket_bounds<<<grid_for(nbuckets + 1), kThreads, 0, s>>>(hs, M, nbuckets, bstart.p);
    TC_LAUNCH_CHECK();
    k_bucket_parts<<<grid_for(nbuckets), kThreads, 0, s>>>(bstart.p, nbuckets, parts.p);
    TC_LAUNCH_CHECK();
    exclusive_scan(parts.p, cstart.p, nbuckets, true, tmp, s);
    const int64_t pmax = nbuckets + ceil_div(M, kHistChunk);  // parts, at most
    k_bucket_hist<<<(unsigned)pmax, kHistThreads, 0, s>>>(hs, bstart.p, cstart.p, nbuckets, N, deg);
    TC_LAUNCH_CHECK();
}

// One endpoint of every pair key: the lower (hi == 0) or the upper label.
__global__ void k_endpoint(const uint64_t *__restrict__ keys, int64_t m, int gb, int hi,
                           uint32_t *__restrict__ out) {
    const uint64_t mask = (1ull << gb) - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = __builtin_nontemporal_load(&keys[i]);
        out[i] = (uint32_t)(hi ? (k & mask) : (k >> gb));
    }
}

// Degrees of a simple graph given as one edge list (labels are the ids):
// the number of times each id occurs in src and in dst, read in place.
void add_pair_counts(const int32_t *src, const int32_t *dst, int64_t M, int gb, int32_t *deg, int64_t N,
                     uint32_t *spare, Allocator &tmp, hipStream_t s, bool runs_src, bool runs_dst) {
    if (M <= 0) return;
    const int32_t *arr[2] = {src, dst};
    const bool runs[2] = {runs_src, runs_dst};
    for (int q = 0; q < 2; ++q) {
        if (runs[q]) {
            k_run_degrees<<<grid_for(M, 4), kThreads, 0, s>>>(arr[q], M, deg);
            TC_LAUNCH_CHECK();
        } else {
            histogram_add(spare, spare + M, M, gb, deg, N, tmp, s, reinterpret_cast<const uint32_t *>(arr[q]));
        }
    }
}

// Degrees of a simple graph given as pair keys in any order: the number of
// keys each label is an endpoint of.
void add_endpoint_counts(const uint64_t *keys, int64_t M, int gb, int32_t *deg, int64_t N, uint32_t *spare,
                         Allocator &tmp, hipStream_t s) {
    if (M <= 0) return;
    for (int hi = 0; hi < 2; ++hi) {
        k_endpoint<<<grid_for(M, 4), kThreads, 0, s>>>(keys, M, gb, hi, spare);  // spare: 2 M words
        TC_LAUNCH_CHECK();
        histogram_add(spare, spare + M, M, gb, deg, N, tmp, s);
    }
}
}  // namespace

void add_degrees(const uint64_t *ukeys, int64_t M, int gb, int32_t *deg, int64_t N, uint32_t *spare, Allocator &tmp,
                 hipStream_t s) {
    if (M <= 0) return;
    uint32_t *hi = spare;  // 2 M words
    uint32_t *hi_tmp = hi + M;
    k_degrees_lo<<<grid_for(M, 4), kThreads, 0, s>>>(ukeys, M, gb, deg, hi);
    TC_LAUNCH_CHECK();
    histogram_add(hi, hi_tmp, M, gb, deg, N, tmp, s);
}

void degree_rank(const int32_t *deg, int64_t N, const int64_t *node_base, int k, int32_t max_n, int32_t *perm,
                 int32_t *rank, Allocator &tmp, hipStream_t s) {
    const int vb = std::max(1, bits_for((uint64_t)std::max<int64_t>(max_n - 1, 1)));
    const int db = vb;  // a degree is below n
    const int kb_bits = bits_for((uint64_t)(k - 1));
    if (kb_bits + db + vb > 64) throw Error(TC_ERR_TOO_LARGE, "too many graphs of this size in one handle");
    if (N <= 0) return;
    DevBuf<uint64_t> ra(tmp, (size_t)N), rb(tmp, (size_t)N);
    k_rank_keys<<<grid_for(N, 4), kThreads, 0, s>>>(deg, N, node_base, k, db, vb, ra.p);
    TC_LAUNCH_CHECK();
    // keys are made in label order, so v already ascends within every
    // (g, d): a stable sort by (g, d) alone gives the (g, d, v) order
    uint64_t *sorted = radix_sort_u64(ra.p, rb.p, N, vb, kb_bits + db + vb, tmp, s);
    k_rank_from_sorted<<<grid_for(N, 4), kThreads, 0, s>>>(sorted, N, node_base, db, vb, perm, rank);
    TC_LAUNCH_CHECK();
}

void reschedule_device(const Packing &pk, const BuildParams &bp, Allocator &al, hipStream_t s, Oriented &out) {
    const size_t arena_bytes = (size_t)pk.N * 48 + (size_t)bp.workers * 128 + (8u << 20);
    void *arena = al.get(arena_bytes);
    Allocator tmp = al;
    tmp.arena = (uint8_t *)arena;
    tmp.arena_size = arena_bytes;
    tmp.arena_used = 0;
    try {
        schedule_into(pk, bp, al, tmp, s, out, nullptr, 0);
    } catch (...) {
        al.put(arena, arena_bytes);
        throw;
    }
    al.put(arena, arena_bytes);
}

}  // namespace tc
