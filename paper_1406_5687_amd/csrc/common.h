// Shared host/device helpers for the gfx950 triangle-counting library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

#include "tc.h"

namespace tc {

// ----------------------------------------------------------------- errors

struct Error : std::runtime_error {
    tc_status code;
    Error(tc_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e != hipSuccess)
        throw Error(TC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" +
                                       std::to_string(line) + ")");
}
#define TC_HIP(x) ::tc::hip_check((x), #x, __FILE__, __LINE__)
#define TC_LAUNCH_CHECK() ::tc::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int bits_for(uint64_t max_value) {  // bits needed to hold values 0..max_value
    int b = 0;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

// ------------------------------------------------------- device allocator

// Device memory comes from the caller's allocator callbacks when given,
// otherwise from the stream-ordered pool (hipMallocAsync).  An optional
// budget caps the bytes outstanding through one Allocator.
struct Allocator {
    void *(*fn_alloc)(size_t, void *, void *) = nullptr;
    void (*fn_free)(void *, size_t, void *, void *) = nullptr;
    void *ctx = nullptr;
    hipStream_t stream = nullptr;
    uint64_t budget = 0;  // 0 = none
    uint64_t live = 0;
    uint64_t peak = 0;
    // Optional bump region: requests are carved from it while it has room and
    // released all at once by its owner (put() ignores them).
    uint8_t *arena = nullptr;
    size_t arena_size = 0;
    size_t arena_used = 0;

    void *get(size_t bytes) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (arena && arena_used + bytes <= arena_size) {
            void *p = arena + arena_used;
            arena_used += bytes;
            return p;
        }
        if (budget && live + bytes > budget)
            throw Error(TC_ERR_OUT_OF_MEMORY, "device budget exceeded: need " + std::to_string(live + bytes) +
                                                  " bytes, budget " + std::to_string(budget));
        void *p = nullptr;
        if (fn_alloc) {
            p = fn_alloc(bytes, (void *)stream, ctx);
        } else {
            if (hipMallocAsync(&p, bytes, stream) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
            }
        }
        if (!p) throw Error(TC_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) + " bytes failed");
        live += bytes;
        if (live > peak) peak = live;
        return p;
    }
    void put(void *p, size_t bytes) {
        if (!p) return;
        if (arena && (uint8_t *)p >= arena && (uint8_t *)p < arena + arena_size) return;
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (fn_free)
            fn_free(p, bytes, (void *)stream, ctx);
        else
            (void)hipFreeAsync(p, stream);
        live -= bytes;
    }
};

// Owning device buffer.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    Allocator *a = nullptr;
    DevBuf() = default;
    DevBuf(Allocator &al, size_t count) : n(count), a(&al) { p = (T *)al.get(count * sizeof(T)); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), a(o.a) {
        o.p = nullptr;
        o.n = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            a = o.a;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p && a) a->put(p, n * sizeof(T));
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Page-locked host buffer (hipHostMalloc), readable by kernels through its
// device address.
template <class T>
struct HostBuf {
    T *p = nullptr;
    size_t n = 0;
    HostBuf() = default;
    explicit HostBuf(size_t count) { reset(count); }
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    HostBuf(HostBuf &&o) noexcept : p(o.p), n(o.n) {
        o.p = nullptr;
        o.n = 0;
    }
    HostBuf &operator=(HostBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~HostBuf() { release(); }
    void reset(size_t count) {
        release();
        const size_t bytes = (count ? count : 1) * sizeof(T);
        if (hipHostMalloc((void **)&p, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw Error(TC_ERR_OUT_OF_MEMORY, "page-locked host allocation of " + std::to_string(bytes) +
                                                  " bytes failed");
        }
        n = count;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    T *device_ptr() const {
        void *d = nullptr;
        if (hipHostGetDevicePointer(&d, (void *)p, 0) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(TC_ERR_DEVICE, "host buffer has no device address");
        }
        return (T *)d;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// -------------------------------------------------------- device helpers

#ifdef __HIPCC__
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Global-address-space views of device pointers: loads through them compile
// to global_load (not flat_load, which also waits on the LDS counter).
template <class T>
using gptr_t = __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ gptr_t<const T> gview(const T *p) {
    return (gptr_t<const T>)p;
}

template <class T>
__device__ __forceinline__ gptr_t<T> gview_mut(T *p) {
    return (gptr_t<T>)p;
}

// Orders this wave's LDS traffic: writes issued before are visible to reads
// issued after, for every lane of the wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ __forceinline__ T wave_inclusive_sum(T x) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (__lane_id() >= d) x += y;
    }
    return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

template <class T>
__device__ __forceinline__ T wave_reduce_max(T x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const T y = __shfl_xor(x, d, 64);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

__device__ __forceinline__ int32_t readlane32(int32_t x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

__device__ __forceinline__ int64_t readlane64(int64_t x, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int32_t uniform32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ int64_t uniform64(int64_t x) { return readlane64(x, __builtin_amdgcn_readfirstlane(__lane_id())); }

// Lanes of the wave holding the same 9-bit value v (bit 8 flags an inactive
// lane), found with one ballot per bit.
// Workgroups go to the 8 XCDs round-robin by index.  Item of workgroup b
// (b < nb): each XCD takes one contiguous range of the nb items, so data that
// neighbouring items share stays in one XCD's L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ __forceinline__ uint64_t match_peers9(uint32_t v) {
    uint64_t peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        const bool bit = (v >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}
#endif

}  // namespace tc
