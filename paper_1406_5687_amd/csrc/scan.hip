// Device-wide exclusive prefix sums (reduce, scan of block sums, apply).
#include "internal.h"

namespace tc {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ __forceinline__ T block_exclusive_sum(T x, T *wave_tot, T *block_total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = wave_inclusive_sum(x);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const T v = wave_tot[w];
        if (w < wave) base += v;
        tot += v;
    }
    __syncthreads();
    *block_total = tot;
    return base + inc - x;
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Tin *__restrict__ in, int64_t n,
                                                             Tout *__restrict__ partial) {
    __shared__ Tout wave_tot[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // every load is issued before the first is used (positions past the end
    // read the last element, then count 0: no branch around the loads)
    Tin v[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        v[j] = in[i < n ? i : n - 1];
    }
    Tout s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        s += i < n ? (Tout)v[j] : (Tout)0;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) wave_tot[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        Tout t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t += wave_tot[w];
        partial[blockIdx.x] = t;
    }
}

// Exclusive scan of one tile per block, shifted by offsets[blockIdx.x]
// (offsets may be NULL).  Writes out[n] = total when write_total.
template <class Tin, class Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const Tin *__restrict__ in, int64_t n,
                                                            const Tout *__restrict__ offsets, Tout *__restrict__ out,
                                                            int write_total) {
    __shared__ Tout wave_tot[kScanThreads / 64];
    __shared__ Tout stage[kScanTile];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // coalesced loads (all issued before the first is used; positions past
    // the end read the last element and stage 0) into LDS, then each thread
    // scans a contiguous run
    {
        Tin ld[kScanItems];
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t i = base + j * kScanThreads + threadIdx.x;
            ld[j] = in[i < n ? i : n - 1];
        }
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t i = base + j * kScanThreads + threadIdx.x;
            stage[j * kScanThreads + threadIdx.x] = i < n ? (Tout)ld[j] : (Tout)0;
        }
    }
    __syncthreads();
    Tout v[kScanItems];
    Tout run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = stage[threadIdx.x * kScanItems + j];
        run += v[j];
    }
    Tout block_total;
    Tout excl = block_exclusive_sum(run, wave_tot, &block_total);
    const Tout off = offsets ? offsets[blockIdx.x] : (Tout)0;
    excl += off;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        stage[threadIdx.x * kScanItems + j] = excl;
        excl += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int idx = j * kScanThreads + threadIdx.x;
        const int64_t i = base + idx;
        if (i < n) out[i] = stage[idx];
    }
    if (write_total && threadIdx.x == 0 && base + kScanTile >= n) out[n] = off + block_total;
}

template <class Tin, class Tout>
void scan_impl(const Tin *in, Tout *out, int64_t n, bool write_total, Allocator &al, hipStream_t s) {
    if (n <= 0) {
        if (write_total) fill_zero(out, sizeof(Tout), s);
        return;
    }
    const int64_t nb = ceil_div(n, kScanTile);
    if (nb == 1) {
        k_scan_apply<Tin, Tout><<<1, kScanThreads, 0, s>>>(in, n, nullptr, out, write_total ? 1 : 0);
        TC_LAUNCH_CHECK();
        return;
    }
    DevBuf<Tout> partial(al, (size_t)nb + 1);
    k_scan_reduce<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, partial.p);
    TC_LAUNCH_CHECK();
    scan_impl<Tout, Tout>(partial.p, partial.p, nb, false, al, s);  // in place is safe: tile-local staging
    k_scan_apply<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, partial.p, out, write_total ? 1 : 0);
    TC_LAUNCH_CHECK();
}

}  // namespace

void exclusive_scan(const uint32_t *in, int64_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s) {
    scan_impl<uint32_t, int64_t>(in, out, n, write_total, al, s);
}
void exclusive_scan(const int32_t *in, int64_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s) {
    scan_impl<int32_t, int64_t>(in, out, n, write_total, al, s);
}
void exclusive_scan(const int64_t *in, int64_t *out, int64_t n, bool write_total, Allocator &al, hipStream_t s) {
    scan_impl<int64_t, int64_t>(in, out, n, write_total, al, s);
}
void exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, bool write_total, Allocator &al,
                    hipStream_t s) {
    scan_impl<uint32_t, uint32_t>(in, out, n, write_total, al, s);
}

}  // namespace tc
