// Persistent counting kernels: the node iterator of Fig. 1 run task by task
// (Fig. 10) by workers that pull tasks from an atomic queue head in place of
// the coordinator of Fig. 11.
//
// For a source s with sorted list L = N_s (|L| = a) and each entry t_i = L[i],
// the triangles found at the stored edge (s, t_i) are the members of
// N_{t_i} that are also in L (Fig. 1: S = N_s intersect N_u).  Every member
// of N_{t_i} lies after t_i in the order, so only lists of t_0..t_{a-2} can
// contribute.
//
// Work layout on gfx950: L is inserted into an LDS hash table; the rows
// N_{t_i} of all targets are laid end to end into one virtual sequence of
// sum_i |N_{t_i}| ids, and a wave walks that sequence 64 ids per step: each
// lane loads one id (consecutive lanes read consecutive addresses of a row)
// and probes the hash table.  The row a lane falls in is found from the
// segment starts inside the 64-wide window (one ballot), so short rows never
// leave lanes idle and long rows need no per-row loop.
//
//   - lists with 2 <= a <= small_max (at most 128): one wave per list, tasks
//     of consecutive sources pulled by waves (k_count_small);
//   - longer lists: one 1024-thread workgroup per list, its 16 waves splitting
//     the virtual sequence (k_count_big); lists longer than lds_max are probed
//     by binary search in device memory instead of the LDS table.
//
// Per-node counts (Section II): a triangle {s, t_i, w} found at probe w adds
// one to each of s, t_i and w.  Counts for entries of L are gathered in LDS
// counters indexed by list position and flushed with one device atomic per
// non-zero position.
#include "internal.h"

namespace tc {

namespace {

constexpr int kSmallMax = 128;
constexpr int kSmallHashBits = 9;
constexpr int kSmallHash = 1 << kSmallHashBits;  // load factor <= 1/4
constexpr int kSmallWaves = 4;

constexpr int kLdsMax = 4096;
constexpr int kBigHashBits = 13;
constexpr int kBigHash = 1 << kBigHashBits;  // load factor <= 1/2
constexpr int kBigWaves = 16;
constexpr int kBigThreads = kBigWaves * 64;

constexpr int kWin = 4;           // 64-id windows walked per step
constexpr int kStep = 64 * kWin;  // ids per step

__device__ __forceinline__ uint32_t hash_slot(int32_t x, int bits) {
    return ((uint32_t)x * 2654435769u) >> (32 - bits);
}

__device__ __forceinline__ int find_desc(const CountDesc *__restrict__ d, int nd, int64_t c, bool big) {
    int lo = 0, hi = nd - 1;  // largest h whose first index is <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = big ? d[mid].big_base : d[mid].task_base;
        if (b <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int graph_of(const int64_t *__restrict__ node_base, int k, int64_t x) {
    if (k <= 1) return 0;
    int lo = 0, hi = k + 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (node_base[mid] > x)
            hi = mid;
        else
            lo = mid + 1;
    }
    const int g = lo - 1;
    return g < 0 ? 0 : (g > k - 1 ? k - 1 : g);
}

__device__ __forceinline__ void add_u64(int64_t *p, uint64_t v) {
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// --------------------------------------------------------------- one wave

// Walks the virtual sequence of target-row ids from e_begin to e_end (a
// multiple of kStep apart, e_end may pass total), kStep ids per step: marks
// the row starts that fall inside the step, finds every lane's row with one
// ballot per 64-id window, loads the 4 ids of each lane together, then probes
// them together.  `cur` is the row holding e_begin.
//   IN_LDS: membership in the source list by the LDS hash (key/pos);
//   otherwise by binary search in the sorted list col[rs .. rs+a) (huge lists).
// Per-node counts go to LDS counters by list position, or (huge lists) to tv.
template <int HBITS, bool PER_NODE, bool IN_LDS, class PosT>
__device__ __forceinline__ uint32_t walk_steps(const int32_t *key, const PosT *pos, const int32_t *P,
                                               const int64_t *base, const PosT *tpos, int32_t *cnt, uint8_t *flag,
                                               gptr_t<const int32_t> col, int64_t m, int32_t nt, int32_t total,
                                               int cur, int32_t e_begin, int32_t e_end, int64_t rs, int32_t a,
                                               int32_t i0, int64_t *__restrict__ tv) {
    constexpr uint32_t kMask = (1u << HBITS) - 1;
    const int lane = __lane_id();
    const uint64_t upto = lanemask_lt() | (1ull << lane);
    uint32_t hits = 0;
    for (int32_t e0 = e_begin; e0 < e_end; e0 += kStep) {
#pragma unroll
        for (int q = 0; q < kWin; ++q) {
            const int jj = cur + 1 + lane + 64 * q;
            if (jj < nt) {
                const int32_t p = P[jj] - e0;
                if (p < kStep) flag[p] = 1;
            }
        }
        wave_lds_sync();
        uint64_t M[kWin];
        int pre[kWin];
        int acc = 0;
#pragma unroll
        for (int q = 0; q < kWin; ++q) {
            M[q] = __ballot(flag[64 * q + lane] != 0);
            pre[q] = acc;
            acc += popc64(M[q]);
        }
#pragma unroll
        for (int q = 0; q < kWin; ++q) flag[64 * q + lane] = 0;
        int seg[kWin];
        int64_t at[kWin];
        int32_t w[kWin];
#pragma unroll
        for (int q = 0; q < kWin; ++q) {
            seg[q] = cur + pre[q] + popc64(M[q] & upto);
            const int32_t e = e0 + 64 * q + lane;
            const int64_t x = e < total ? base[seg[q]] + e : -1;
            at[q] = (uint64_t)x < (uint64_t)m ? x : -1;
        }
#pragma unroll
        for (int q = 0; q < kWin; ++q) w[q] = col[at[q] < 0 ? 0 : at[q]];
#pragma unroll
        for (int q = 0; q < kWin; ++q) w[q] = at[q] < 0 ? -1 : w[q];
        if (IN_LDS) {
            uint32_t sl[kWin];
            int32_t k[kWin];
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                sl[q] = hash_slot(w[q], HBITS);
                k[q] = key[sl[q]];
            }
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                while (k[q] != w[q] && k[q] != -1) {  // collision chain (rare)
                    sl[q] = (sl[q] + 1) & kMask;
                    k[q] = key[sl[q]];
                }
            }
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                const bool hit = w[q] >= 0 && k[q] == w[q];
                hits += hit ? 1u : 0u;
                if (PER_NODE && hit) {
                    atomicAdd(&cnt[pos[sl[q]]], 1);
                    atomicAdd(&cnt[tpos[seg[q]]], 1);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                if (w[q] < 0) continue;
                int32_t lo = 0, hi = a;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (col[rs + mid] < w[q])
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < a && col[rs + lo] == w[q]) {
                    ++hits;
                    if (PER_NODE) {
                        add_u64(&tv[w[q]], 1);
                        add_u64(&tv[col[rs + i0 + tpos[seg[q]]]], 1);
                    }
                }
            }
        }
        int nc = cur + acc;
        if (nc + 1 < nt && P[nc + 1] == e0 + kStep) ++nc;
        cur = nc;
        wave_lds_sync();
    }
    return hits;
}

struct alignas(16) SmallLds {
    int64_t base[kSmallMax];  // per target row: row start minus its prefix
    int32_t key[kSmallHash];  // hashed source list, -1 = empty
    int32_t P[kSmallMax + 1]; // exclusive prefix of row lengths, then the total
    int32_t cnt[kSmallMax];   // per-position counts (per-node mode)
    uint8_t pos[kSmallHash];  // list position of each hashed id
    uint8_t tpos[kSmallMax];  // list position of each target row
    uint8_t flag[kStep];      // row starts inside the current step
};

// One source s whose list (a entries, 2 <= a <= 128) is already in registers:
// x0 = L[lane], x1 = L[64 + lane].
template <bool PER_NODE>
__device__ __forceinline__ uint64_t source_small(SmallLds &S, gptr_t<const int32_t> col, gptr_t<const int64_t> off,
                                                 int64_t *__restrict__ tv, int64_t m, int32_t s, int32_t a,
                                                 int32_t x0, int32_t x1, int lane) {
    const bool h0 = lane < a, h1 = lane + 64 < a;
    if (h0) {
        uint32_t sl = hash_slot(x0, kSmallHashBits);
        while (atomicCAS(&S.key[sl], -1, x0) != -1) sl = (sl + 1) & (kSmallHash - 1);
        if (PER_NODE) S.pos[sl] = (uint8_t)lane;
    }
    if (h1) {
        uint32_t sl = hash_slot(x1, kSmallHashBits);
        while (atomicCAS(&S.key[sl], -1, x1) != -1) sl = (sl + 1) & (kSmallHash - 1);
        if (PER_NODE) S.pos[sl] = (uint8_t)(64 + lane);
    }
    // rows of t_0 .. t_{a-2}; empty rows are dropped so row starts are distinct.
    // Loads are unconditional (x0 / x1 hold valid labels in every lane) so all
    // four are in flight together.
    const int64_t r0 = off[x0], e0r = off[x0 + 1];
    const int64_t r1 = off[x1], e1r = off[x1 + 1];
    const int32_t b0 = lane < a - 1 ? (int32_t)(e0r - r0) : 0;
    const int32_t b1 = lane + 64 < a - 1 ? (int32_t)(e1r - r1) : 0;
    const uint64_t m0 = __ballot(b0 > 0), m1 = __ballot(b1 > 0);
    const int n0 = popc64(m0);
    const int32_t inc0 = wave_inclusive_sum(b0);
    const int32_t tot0 = readlane32(inc0, 63);
    const int32_t inc1 = tot0 + wave_inclusive_sum(b1);
    const int32_t total = readlane32(inc1, 63);
    if (b0 > 0) {
        const int j = popc64(m0 & lanemask_lt());
        S.P[j] = inc0 - b0;
        S.base[j] = r0 - (int64_t)(inc0 - b0);
        S.tpos[j] = (uint8_t)lane;
    }
    if (b1 > 0) {
        const int j = n0 + popc64(m1 & lanemask_lt());
        S.P[j] = inc1 - b1;
        S.base[j] = r1 - (int64_t)(inc1 - b1);
        S.tpos[j] = (uint8_t)(64 + lane);
    }
    const int nt = n0 + popc64(m1);
    if (lane == 0) S.P[nt] = total;
    wave_lds_sync();

    const int32_t e_end = ((total + kStep - 1) / kStep) * kStep;
    const uint32_t hits = walk_steps<kSmallHashBits, PER_NODE, true, uint8_t>(
        S.key, S.pos, S.P, S.base, S.tpos, S.cnt, S.flag, col, m, nt, total, 0, 0, e_end, 0, a, 0, tv);
    if (PER_NODE) {
        const uint64_t hs = wave_sum((uint64_t)hits);
        wave_lds_sync();
        if (h0) {
            const int32_t c = S.cnt[lane];
            if (c) {
                add_u64(&tv[x0], (uint64_t)c);
                S.cnt[lane] = 0;
            }
        }
        if (h1) {
            const int32_t c = S.cnt[64 + lane];
            if (c) {
                add_u64(&tv[x1], (uint64_t)c);
                S.cnt[64 + lane] = 0;
            }
        }
        if (lane == 0 && hs) add_u64(&tv[s], hs);
    }
    // empty the whole table (two 16-byte stores per lane)
    static_assert(kSmallHash == 64 * 8, "table clear assumes 8 slots per lane");
    int4 *kv = reinterpret_cast<int4 *>(S.key);
    kv[lane] = make_int4(-1, -1, -1, -1);
    kv[64 + lane] = make_int4(-1, -1, -1, -1);
    wave_lds_sync();
    return (uint64_t)hits;
}

template <bool PER_NODE>
__global__ __launch_bounds__(kSmallWaves * 64) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_count_small(const CountDesc *__restrict__ descs, int ndesc,
                                                                  int64_t total_tasks, uint32_t *__restrict__ head,
                                                                  int nworkers) {
    __shared__ SmallLds lds[kSmallWaves];
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    SmallLds &S = lds[wave];
    for (int i = lane; i < kSmallHash; i += 64) S.key[i] = -1;
    for (int i = lane; i < kSmallMax; i += 64) S.cnt[i] = 0;
    for (int i = lane; i < kStep; i += 64) S.flag[i] = 0;
    wave_lds_sync();

    int64_t c = (int64_t)blockIdx.x * kSmallWaves + wave;
    while (c < total_tasks) {
        const int h = ndesc > 1 ? find_desc(descs, ndesc, c, false) : 0;
        const gptr_t<const int32_t> col = gview(descs[h].col);
        const gptr_t<const int64_t> off = gview(descs[h].off);
        int64_t *__restrict__ tv = descs[h].tv;
        const int64_t m = descs[h].m;
        const int64_t lt = c - descs[h].task_base;
        const int32_t v0 = descs[h].bnd[lt], v1 = descs[h].bnd[lt + 1];
        const int g = descs[h].gid ? descs[h].gid[lt] : 0;
        const int small_max = descs[h].small_max;
        uint64_t tri = 0;
        for (int32_t s0 = v0; s0 < v1; s0 += 64) {
            const int32_t sv = min(s0 + lane, v1 - 1);
            const int64_t o0 = off[sv], o1 = off[sv + 1];
            const int32_t al = s0 + lane < v1 ? (int32_t)(o1 - o0) : 0;
            uint64_t work = __ballot(al >= 2 && al <= small_max);
            if (!work) continue;
            // the list of the next source is loaded while the current one is counted;
            // indices are clamped into the list so every lane loads a valid label
            int j = __ffsll((unsigned long long)work) - 1;
            int32_t a = readlane32(al, j);
            int64_t rs = readlane64(o0, j);
            int32_t x0 = col[rs + min(lane, a - 1)];
            int32_t x1 = col[rs + min(lane + 64, a - 1)];
            while (work) {
                work &= work - 1;
                int jn = j, an = a;
                int64_t rn = rs;
                if (work) {
                    jn = __ffsll((unsigned long long)work) - 1;
                    an = readlane32(al, jn);
                    rn = readlane64(o0, jn);
                }
                const int32_t nx0 = col[rn + min(lane, an - 1)];
                const int32_t nx1 = col[rn + min(lane + 64, an - 1)];
                tri += source_small<PER_NODE>(S, col, off, tv, m, s0 + j, a, x0, x1, lane);
                j = jn;
                a = an;
                rs = rn;
                x0 = nx0;
                x1 = nx1;
            }
        }
        tri = wave_sum(tri);
        if (lane == 0 && tri) add_u64(&descs[h].totals[g], tri);
        uint32_t nxt = 0;
        if (lane == 0) nxt = atomicAdd(head, 1u);
        c = (int64_t)nworkers + (int64_t)(uint32_t)readlane32((int32_t)nxt, 0);
    }
}

// ---------------------------------------------------------- one workgroup

struct BigLds {
    int64_t base[kLdsMax];
    int32_t key[kBigHash];
    int32_t P[kLdsMax + 1];
    int32_t cnt[kLdsMax];
    int16_t pos[kBigHash];
    int16_t tpos[kLdsMax];
    uint8_t flag[kBigWaves][kStep];
    int32_t wsum[kBigWaves];
    int32_t wcnt[kBigWaves];
    uint64_t whits[kBigWaves];
    int64_t item;
};

// Lays out the rows of targets i in [i0, i1) (positions in the source list)
// into P / base / tpos (tpos relative to i0).  Returns (rows, total ids).
__device__ __forceinline__ void big_rows(BigLds &S, gptr_t<const int32_t> col, gptr_t<const int64_t> off,
                                         int64_t rs, int32_t i0, int32_t i1, int32_t *nt_out, int32_t *total_out) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    int32_t carry_n = 0, carry_sum = 0;
    for (int32_t rb = i0; rb < i1; rb += kBigThreads) {
        const int32_t i = rb + (int32_t)threadIdx.x;
        int32_t b = 0;
        int64_t r = 0;
        if (i < i1) {
            const int32_t t = col[rs + i];
            r = off[t];
            b = (int32_t)(off[t + 1] - r);
        }
        const int32_t inc = wave_inclusive_sum(b);
        const uint64_t m = __ballot(b > 0);
        if (lane == 63) {
            S.wsum[wave] = inc;
            S.wcnt[wave] = popc64(m);
        }
        __syncthreads();
        int32_t sb = 0, cb = 0, st = 0, ct = 0;
#pragma unroll
        for (int w = 0; w < kBigWaves; ++w) {
            const int32_t ws = S.wsum[w], wc = S.wcnt[w];
            if (w < wave) {
                sb += ws;
                cb += wc;
            }
            st += ws;
            ct += wc;
        }
        if (b > 0) {
            const int j = carry_n + cb + popc64(m & lanemask_lt());
            const int32_t p = carry_sum + sb + inc - b;
            S.P[j] = p;
            S.base[j] = r - (int64_t)p;
            S.tpos[j] = (int16_t)(i - i0);
        }
        carry_n += ct;
        carry_sum += st;
        __syncthreads();
    }
    if (threadIdx.x == 0) S.P[carry_n] = carry_sum;
    __syncthreads();
    *nt_out = carry_n;
    *total_out = carry_sum;
}

// This wave's contiguous share of the virtual sequence, in whole steps.
template <bool PER_NODE>
__device__ __forceinline__ uint64_t big_windows(BigLds &S, gptr_t<const int32_t> col, int64_t *__restrict__ tv,
                                                int64_t m, int64_t rs, int32_t a, int32_t i0, int32_t nt,
                                                int32_t total, bool in_lds) {
    const int wave = threadIdx.x >> 6;
    const int32_t nsteps = (total + kStep - 1) / kStep;
    const int32_t per = (nsteps + kBigWaves - 1) / kBigWaves;
    const int32_t s0 = wave * per;
    const int32_t s1 = min(nsteps, s0 + per);
    if (s0 >= s1) return 0;
    const int32_t e_begin = s0 * kStep;
    int lo = 0, hi = nt - 1;  // row holding e_begin: last row whose start is <= it
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.P[mid] <= e_begin)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (in_lds)
        return walk_steps<kBigHashBits, PER_NODE, true, int16_t>(S.key, S.pos, S.P, S.base, S.tpos, S.cnt,
                                                                 S.flag[wave], col, m, nt, total, lo, e_begin,
                                                                 s1 * kStep, rs, a, i0, tv);
    return walk_steps<kBigHashBits, PER_NODE, false, int16_t>(S.key, S.pos, S.P, S.base, S.tpos, S.cnt,
                                                              S.flag[wave], col, m, nt, total, lo, e_begin,
                                                              s1 * kStep, rs, a, i0, tv);
}

template <bool PER_NODE>
__global__ __launch_bounds__(kBigThreads) void k_count_big(const CountDesc *__restrict__ descs, int ndesc,
                                                           int64_t total_big, uint32_t *__restrict__ head,
                                                           int lds_max) {
    __shared__ BigLds S;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kBigHash; i += kBigThreads) S.key[i] = -1;
    for (int i = threadIdx.x; i < kLdsMax; i += kBigThreads) S.cnt[i] = 0;
    for (int i = threadIdx.x; i < kBigWaves * kStep; i += kBigThreads) (&S.flag[0][0])[i] = 0;
    if (threadIdx.x == 0) S.item = blockIdx.x;
    __syncthreads();

    for (;;) {
        const int64_t item = S.item;
        if (item >= total_big) break;
        const int h = ndesc > 1 ? find_desc(descs, ndesc, item, true) : 0;
        const gptr_t<const int32_t> col = gview(descs[h].col);
        const gptr_t<const int64_t> off = gview(descs[h].off);
        int64_t *__restrict__ tv = descs[h].tv;
        const int64_t m = descs[h].m;
        const int32_t s = descs[h].big[item - descs[h].big_base];
        const int64_t rs = off[s];
        const int32_t a = (int32_t)(off[s + 1] - rs);
        uint64_t hits = 0;
        if (a <= lds_max) {
            for (int32_t k = threadIdx.x; k < a; k += kBigThreads) {
                const int32_t x = col[rs + k];
                uint32_t sl = hash_slot(x, kBigHashBits);
                while (atomicCAS(&S.key[sl], -1, x) != -1) sl = (sl + 1) & (kBigHash - 1);
                S.pos[sl] = (int16_t)k;
            }
            __syncthreads();
            int32_t nt, total;
            big_rows(S, col, off, rs, 0, a - 1, &nt, &total);
            hits = big_windows<PER_NODE>(S, col, tv, m, rs, a, 0, nt, total, true);
            __syncthreads();
            if (PER_NODE) {
                for (int32_t k = threadIdx.x; k < a; k += kBigThreads) {
                    const int32_t c = S.cnt[k];
                    if (c) {
                        add_u64(&tv[col[rs + k]], (uint64_t)c);
                        S.cnt[k] = 0;
                    }
                }
            }
            for (int i = threadIdx.x; i < kBigHash; i += kBigThreads) S.key[i] = -1;
        } else {
            for (int32_t i0 = 0; i0 < a - 1; i0 += lds_max) {
                const int32_t i1 = min(a - 1, i0 + lds_max);
                int32_t nt, total;
                big_rows(S, col, off, rs, i0, i1, &nt, &total);
                hits += big_windows<PER_NODE>(S, col, tv, m, rs, a, i0, nt, total, false);
                __syncthreads();
            }
        }
        // block total of hits
        const uint64_t wh = wave_sum(hits);
        if (lane == 0) S.whits[wave] = wh;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t H = 0;
            for (int w = 0; w < kBigWaves; ++w) H += S.whits[w];
            if (H) {
                const int g = graph_of(descs[h].node_base, descs[h].k, s);
                add_u64(&descs[h].totals[g], H);
                if (PER_NODE) add_u64(&tv[s], H);
            }
            S.item = (int64_t)gridDim.x + (int64_t)atomicAdd(head, 1u);
        }
        __syncthreads();
    }
}

__global__ void k_scatter(const int64_t *__restrict__ tv, const int32_t *__restrict__ perm, int64_t n,
                          int64_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[perm[i]] = tv[i];
}

}  // namespace

int max_small_list() { return kSmallMax; }

int small_kernel_waves_per_cu(bool per_node) {
    static int cached[2] = {0, 0};
    int &c = cached[per_node ? 1 : 0];
    if (!c) {
        int blocks = 0;
        if (per_node)
            TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_count_small<true>, kSmallWaves * 64, 0));
        else
            TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_count_small<false>, kSmallWaves * 64, 0));
        c = std::max(1, blocks) * kSmallWaves;
    }
    return c;
}
int max_lds_list() { return kLdsMax; }

int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    TC_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int cus = 0;
    TC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    cus = cus > 0 ? cus : 1;
    if (dev >= 0 && dev < 64) cached[dev] = cus;
    return cus;
}

void count_launch(const CountLaunch &L, hipStream_t s) {
    const int lds_max = L.lds_max < 2 ? kLdsMax : (L.lds_max > kLdsMax ? kLdsMax : L.lds_max);
    if (L.total_tasks > 0) {
        // never launch more workers than can be resident at once: a worker that
        // starts late would hold its first task until the end
        const int resident = small_kernel_waves_per_cu(L.per_node) / kSmallWaves * device_cu_count();
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(L.workers, kSmallWaves), resident));
        if (L.per_node)
            k_count_small<true><<<blocks, kSmallWaves * 64, 0, s>>>(L.descs, L.ndesc, L.total_tasks, L.heads,
                                                                    blocks * kSmallWaves);
        else
            k_count_small<false><<<blocks, kSmallWaves * 64, 0, s>>>(L.descs, L.ndesc, L.total_tasks, L.heads,
                                                                     blocks * kSmallWaves);
        TC_LAUNCH_CHECK();
    }
    if (L.total_big > 0) {
        const int blocks = (int)std::min<int64_t>(L.big_blocks, L.total_big);
        if (L.per_node)
            k_count_big<true><<<blocks, kBigThreads, 0, s>>>(L.descs, L.ndesc, L.total_big, L.heads + 1, lds_max);
        else
            k_count_big<false><<<blocks, kBigThreads, 0, s>>>(L.descs, L.ndesc, L.total_big, L.heads + 1, lds_max);
        TC_LAUNCH_CHECK();
    }
}

void scatter_per_node(const int64_t *tv, const int32_t *perm, int64_t n, int64_t *out, hipStream_t s) {
    if (n <= 0) return;
    const int64_t b = std::min<int64_t>(ceil_div(n, 256 * 4), 1 << 20);
    k_scatter<<<(unsigned)b, 256, 0, s>>>(tv, perm, n, out);
    TC_LAUNCH_CHECK();
}

}  // namespace tc
