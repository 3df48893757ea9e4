// LSD radix sort of 32- or 64-bit keys over a bit range, 8 bits per pass (the
// last pass takes what is left of the range).
//
// Each pass: (1) per-tile digit histograms (per-wave counters, one writer per
// digit and round), (2) one exclusive scan over the digit-major histogram
// table giving every (digit, tile) its output base, (3) a stable scatter:
// each wave ranks its keys among equal digits with ballots over the digit
// bits, the tile is reordered by digit in LDS, and runs of equal digits are
// written out contiguously.
#include "internal.h"

namespace tc {

namespace {

constexpr int kSortWaves = 4;
constexpr int kSortThreads = kSortWaves * 64;
constexpr int kSortRounds = 16;                        // keys per lane
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 keys per block
static_assert(kSortTile == kRadixTile && kSortWaves == 4 && kSortRounds == 16, "tile layout shared with callers");
constexpr int kRadix = 256;

// Key r of lane l in wave w sits at tile offset w * 64 * kSortRounds + r * 64 + l:
// each wave owns a contiguous quarter of the tile, read 64 keys at a time.
__device__ __forceinline__ int64_t key_index(int64_t tile_base, int wave, int r, int lane) {
    return tile_base + (int64_t)wave * 64 * kSortRounds + r * 64 + lane;
}

// Digit of a key in the pass at `shift`: `bits` (<= 8) bits, so that a
// range whose width is not a multiple of 8 ignores the bits above it.
template <class K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t dmask) {
    return (uint32_t)(key >> shift) & dmask;
}

template <class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                             int bits, int64_t nblocks, uint32_t *__restrict__ hist) {
    const uint32_t dmask = (1u << bits) - 1u;
    __shared__ uint32_t hw[kSortWaves][kRadix];  // one histogram per wave
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&hw[0][0])[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = xcd_tile(blockIdx.x, nblocks);  // digit-table entries and output runs of
    const int64_t tile = t * kSortTile;               // neighbouring tiles share one L2
    // all of the lane's keys are loaded before any is ranked
    K kk[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        kk[r] = i < n ? keys[i] : (K)0;
    }
    const bool full = n - tile >= kSortTile;  // block-uniform: every lane holds a key
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        const uint32_t d = i < n ? digit_of(kk[r], shift, dmask) : 256u;  // 256: past the end
        // lanes holding the same digit (all of them when the first lane's
        // digit is everyone's, else one ballot per digit bit); the first of
        // them adds their number to the wave's counter, so no counter gets
        // two writes in one round and no LDS atomics are needed
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
        if (sizeof(K) == 4) {
            // 32-bit keys: one LDS add per key measured faster here (the
            // tile's loads are shorter, the ballots not hidden behind them)
            if (__ballot(d == d0) == ~0ull) {
                if (lane == 0 && d0 < 256u) atomicAdd(&hw[wave][d0], 64u);
            } else if (d < 256u) {
                atomicAdd(&hw[wave][d], 1u);
            }
            continue;
        }
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
        if (d < 256u && lane == __ffsll((unsigned long long)peers) - 1) hw[wave][d] += (uint32_t)popc64(peers);
        wave_lds_sync();
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRadix; i += kSortThreads) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) c += hw[w][i];
        hist[(int64_t)i * nblocks + t] = c;
    }
}

template <class K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K *__restrict__ keys, K *__restrict__ out,
                                                                int64_t n, int shift, int bits, int64_t nblocks,
                                                                const int64_t *__restrict__ base) {
    static_assert(kSortThreads >= kRadix, "one thread per digit in the tile scan");
    const uint32_t dmask = (1u << bits) - 1u;
    __shared__ uint32_t wcnt[kSortWaves][kRadix];
    __shared__ uint32_t bstart[kRadix];
    __shared__ int64_t gbase[kRadix];
    __shared__ K stage[kSortTile];
    __shared__ uint32_t scan_tmp[kSortWaves];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kSortWaves * kRadix; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const int64_t t = xcd_tile(blockIdx.x, nblocks);
    const int64_t tile = t * kSortTile;
    const bool full = n - tile >= kSortTile;  // block-uniform: every lane holds a key
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
        const uint32_t d = i < n ? digit_of(k[r], shift, dmask) : 256u;  // 256: past the end
        // lanes of this wave holding the same digit: all of them when the
        // first lane's digit is everyone's, else one ballot per digit bit
        // (plus one for the past-the-end flag in the last tile)
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
        const int d = threadIdx.x;  // threads past the last digit add nothing
        uint32_t tot = 0;
        if (d < kRadix) {
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t c = wcnt[w][d];
                wcnt[w][d] = tot;
                tot += c;
            }
        }
        // block exclusive scan of tot over digits
        uint32_t inc = wave_inclusive_sum(tot);
        if (lane == 63) scan_tmp[wave] = inc;
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w)
            if (w < wave) add += scan_tmp[w];
        if (d < kRadix) {
            bstart[d] = add + inc - tot;
            gbase[d] = base[(int64_t)d * nblocks + t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = key_index(tile, wave, r, lane);
        if (i < n) {
            const uint32_t d = digit_of(k[r], shift, dmask);
            stage[bstart[d] + wcnt[wave][d] + rank[r]] = k[r];
        }
    }
    __syncthreads();
    const int64_t valid = n - tile < kSortTile ? n - tile : kSortTile;
    for (int i = threadIdx.x; i < valid; i += kSortThreads) {
        const K key = stage[i];
        const uint32_t d = digit_of(key, shift, dmask);
        const int64_t at = gbase[d] + (i - (int64_t)bstart[d]);
        if ((uint64_t)at < (uint64_t)n) out[at] = key;
    }
}

// With `first` given, the first pass reads it instead of keys (first is
// never written; the result is in keys or tmp).
// With first_hist given, the first pass takes that digit table instead of
// counting one.
template <class K>
K *radix_sort_impl(K *keys, K *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al, hipStream_t s,
                   const K *first = nullptr, const uint32_t *first_hist = nullptr) {
    if (n <= 1 || end_bit <= begin_bit) {
        if (first && n > 0) TC_HIP(hipMemcpyAsync(keys, first, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s));
        return keys;
    }
    const int64_t nb = ceil_div(n, kSortTile);
    DevBuf<uint32_t> hist(al, (size_t)(nb * kRadix));
    DevBuf<int64_t> base(al, (size_t)(nb * kRadix) + 1);
    const K *in = first ? first : keys;
    K *a = keys, *b = tmp;
    if (first) {
        a = tmp;  // written by the first pass
        b = keys;
    }
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        const int bits = std::min(8, end_bit - shift);
        K *outp = first && shift == begin_bit ? a : b;
        if (first_hist && shift == begin_bit) {
            exclusive_scan(first_hist, base.p, nb * kRadix, false, al, s);
        } else {
            k_radix_hist<K><<<(unsigned)nb, kSortThreads, 0, s>>>(in, n, shift, bits, nb, hist.p);
            TC_LAUNCH_CHECK();
            exclusive_scan(hist.p, base.p, nb * kRadix, false, al, s);
        }
        k_radix_scatter<K><<<(unsigned)nb, kSortThreads, 0, s>>>(in, outp, n, shift, bits, nb, base.p);
        TC_LAUNCH_CHECK();
        if (!(first && shift == begin_bit)) {
            K *t = a;
            a = b;
            b = t;
        }
        in = a;
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

uint64_t *radix_sort_u64_hist(uint64_t *keys, uint64_t *tmp, int64_t n, int begin_bit, int end_bit,
                              const uint32_t *first_hist, Allocator &al, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, tmp, n, begin_bit, end_bit, al, s, nullptr, first_hist);
}

uint32_t *radix_sort_u32(uint32_t *keys, uint32_t *tmp, int64_t n, int begin_bit, int end_bit, Allocator &al,
                         hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, tmp, n, begin_bit, end_bit, al, s);
}

// The same, reading the keys from first (left unchanged): keys and tmp are
// both scratch of n keys.
uint32_t *radix_sort_u32_from(const uint32_t *first, uint32_t *keys, uint32_t *tmp, int64_t n, int begin_bit,
                              int end_bit, Allocator &al, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, tmp, n, begin_bit, end_bit, al, s, first);
}

}  // namespace tc
