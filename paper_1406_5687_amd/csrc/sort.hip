// LSD radix sort of 64-bit keys over a bit range, 8 bits per pass.
//
// Each pass: (1) per-tile digit histograms, (2) one exclusive scan over the
// digit-major histogram table giving every (digit, tile) its output base,
// (3) a stable scatter: each wave ranks its keys among equal digits with
// ballots, the tile is reordered by digit in LDS, and runs of equal digits
// are written out contiguously.
#include "internal.h"

namespace tc {

namespace {

constexpr int kSortWaves = 4;
constexpr int kSortThreads = kSortWaves * 64;
constexpr int kSortRounds = 16;                        // keys per lane
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 keys per block
constexpr int kRadix = 256;

// Key r of lane l in wave w sits at tile offset w * 64 * kSortRounds + r * 64 + l:
// each wave owns a contiguous quarter of the tile, read 64 keys at a time.
__device__ __forceinline__ int64_t key_index(int64_t tile_base, int wave, int r, int lane) {
    return tile_base + (int64_t)wave * 64 * kSortRounds + r * 64 + lane;
}

template <class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                             int64_t nblocks, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kRadix];
    for (int i = threadIdx.x; i < kRadix; i += kSortThreads) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    // all of the lane's keys are loaded before any is ranked
    K kk[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        kk[r] = i < n ? keys[i] : (K)0;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        uint32_t d = 256u;  // inactive
        if (i < n) d = (uint32_t)(kk[r] >> shift) & 0xffu;
        const uint64_t peers = match_peers9(d);
        const int leader = __ffsll((unsigned long long)peers) - 1;
        if (d < 256u && leader == lane) atomicAdd(&h[d], (uint32_t)popc64(peers));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRadix; i += kSortThreads) hist[(int64_t)i * nblocks + blockIdx.x] = h[i];
}

template <class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K *__restrict__ keys, K *__restrict__ out,
                                                                int64_t n, int shift, int64_t nblocks,
                                                                const int64_t *__restrict__ base) {
    __shared__ uint32_t wcnt[kSortWaves][kRadix];
    __shared__ uint32_t bstart[kRadix];
    __shared__ int64_t gbase[kRadix];
    __shared__ K stage[kSortTile];
    __shared__ uint32_t scan_tmp[kSortWaves];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    K k[kSortRounds];
    uint32_t rank[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        k[r] = i < n ? keys[i] : (K)0;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        const uint32_t d = i < n ? (uint32_t)(k[r] >> shift) & 0xffu : 256u;
        const uint64_t peers = match_peers9(d);
        const int leader = __ffsll((unsigned long long)peers) - 1;
        uint32_t before = 0;
        if (d < 256u) before = wcnt[wave][d];
        wave_lds_sync();
        if (d < 256u && leader == lane) wcnt[wave][d] = before + (uint32_t)popc64(peers);
        wave_lds_sync();
        rank[r] = before + (uint32_t)popc64(peers & lanemask_lt());
    }
    __syncthreads();
    // per digit: offsets of each wave, tile total, start of the digit in the tile
    {
        const int d = threadIdx.x;  // kSortThreads == kRadix
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = wcnt[w][d];
            wcnt[w][d] = tot;
            tot += c;
        }
        // block exclusive scan of tot over digits
        uint32_t inc = wave_inclusive_sum(tot);
        if (lane == 63) scan_tmp[wave] = inc;
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w)
            if (w < wave) add += scan_tmp[w];
        bstart[d] = add + inc - tot;
        gbase[d] = base[(int64_t)d * nblocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        if (i < n) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & 0xffu;
            stage[bstart[d] + wcnt[wave][d] + rank[r]] = k[r];
        }
    }
    __syncthreads();
    const int64_t valid = n - tile < kSortTile ? n - tile : kSortTile;
    for (int i = threadIdx.x; i < valid; i += kSortThreads) {
        const K key = stage[i];
        const uint32_t d = (uint32_t)(key >> shift) & 0xffu;
        const int64_t at = gbase[d] + (i - (int64_t)bstart[d]);
        if ((uint64_t)at < (uint64_t)n) out[at] = key;
    }
}

template <class K>
K *radix_sort_impl(K *keys, K *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al, hipStream_t s) {
    if (n <= 1 || end_bit <= begin_bit) return keys;
    const int64_t nb = ceil_div(n, kSortTile);
    DevBuf<uint32_t> hist(al, (size_t)(nb * kRadix));
    DevBuf<int64_t> base(al, (size_t)(nb * kRadix) + 1);
    K *a = keys, *b = tmp;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        k_radix_hist<K><<<(unsigned)nb, kSortThreads, 0, s>>>(a, n, shift, nb, hist.p);
        TC_LAUNCH_CHECK();
        exclusive_scan(hist.p, base.p, nb * kRadix, false, al, s);
        k_radix_scatter<K><<<(unsigned)nb, kSortThreads, 0, s>>>(a, b, n, shift, nb, base.p);
        TC_LAUNCH_CHECK();
        K *t = a;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

// Sorts keys[0..n) by bits [begin_bit, end_bit).  tmp must hold n keys.
// Returns whichever of keys / tmp holds the result.
uint64_t *radix_sort_u64(uint64_t *keys, uint64_t *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al,
                         hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, tmp, n, begin_bit, end_bit, al, s);
}

uint32_t *radix_sort_u32(uint32_t *keys, uint32_t *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al,
                         hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, tmp, n, begin_bit, end_bit, al, s);
}

}  // namespace tc
