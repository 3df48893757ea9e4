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
// sum_i |N_{t_i}| ids, and a wave walks that sequence 256 ids per step: each
// lane loads four ids (consecutive lanes read consecutive addresses of a row)
// and probes the hash table.  The row a lane falls in is found from the row
// starts inside the step (one ballot per 64-id window), so short rows never
// leave lanes idle and long rows need no per-row loop.
//
// The table is two-choice (cuckoo): an id sits in one of two slots taken from
// one multiplicative hash, so every probe is two independent LDS reads and no
// loop.  With linear probing a wave would walk each 64-id window's collision
// chains until its slowest lane ends, which on power-law lists costs more
// than the probe itself.  A list whose insertion gives up (rare below half
// load) is hashed by linear probing instead.
//
//   - lists with 2 <= a <= small_max (at most 128): one wave per list, tasks
//     of consecutive sources pulled by waves (k_count_small);
//   - longer lists: one workgroup per list (k_count_wide): 4 waves for lists
//     up to 768 entries, 8 waves up to 1920; lists longer than the LDS table
//     (lds_max) are probed by binary search in device memory instead.
//
// Search variant (one-wave lists): a target row N_{t_i} much longer than the
// part of L after t_i (the only entries that can be in it: every member of
// N_{t_i} lies after t_i) is not walked.  Instead each candidate L[j], j > i,
// is looked up in N_{t_i} by binary search in device memory, 64 (i, j) pairs
// per wave step.  A row takes this path when it holds at least a whole walk
// step (256 ids) and its length exceeds R times the a - 1 - i candidates
// (R = the descriptor's search_ratio; -1 = every row, 0 = none); results do
// not depend on the choice.
//
// Per-node counts (Section II): a triangle {s, t_i, w} found at probe w adds
// one to each of s, t_i and w.  Counts for entries of L are gathered in LDS
// counters indexed by list position and flushed with one device atomic per
// non-zero position.
//
// Row addressing: when the adjacency has fewer than 2^29 entries, row starts
// are 32-bit and rows are read with buffer loads (hardware range check);
// otherwise 64-bit offsets and global loads are used (IDX32 = false).
#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace tc {

namespace {

constexpr int kSmallMax = 128;
constexpr int kSmallHashBits = 9;
constexpr int kSmallHash = 1 << kSmallHashBits;  // load factor <= 1/4
constexpr int kSmallWaves = 4;

constexpr int kMedWaves = 4;
constexpr int kMedMax = 768;  // 24 KB of LDS per workgroup: six resident per CU
constexpr int kMedHashBits = 11;  // load factor <= 1/2

constexpr int kLdsMax = 1920;    // 52 KB of LDS per workgroup: three resident per CU
constexpr int kBigHashBits = 12;  // load factor <= 1/2
constexpr int kBigWaves = 8;
constexpr int kBigThreads = kBigWaves * 64;

// empty LDS table slot (ids are at most 2^31 - 2; padding lanes carry -1)
constexpr int32_t kEmpty = 0x7FFFFFFF;

constexpr int kWin = 4;           // 64-id windows walked per step
constexpr int kStep = 64 * kWin;  // ids per step
// flag bytes: position p of a step is byte (p % 64) * 4 + p / 64, so lane l
// finds its four window flags in one 32-bit word; byte kStep is a sink.
constexpr int kFlagBytes = kStep + 4;

// multiplicative hash on the low 24 bits (full-rate 24-bit multiply): the top
// `bits` bits of the 32-bit product are the slot; the next `bits` bits are
// the other slot of the two-choice table
__device__ __forceinline__ uint32_t hash_slot(int32_t x, int bits) {
    return (uint32_t)__umul24((uint32_t)x, 0x9E3779u) >> (32 - bits);
}
__device__ __forceinline__ uint32_t hash_slot2(int32_t x, int bits) {
    return ((uint32_t)__umul24((uint32_t)x, 0x9E3779u) >> (32 - 2 * bits)) & ((1u << bits) - 1);
}

// Two-choice (cuckoo) insertion of x into an LDS table of 2^bits slots (-1 =
// empty): x takes its first slot; a key it displaces moves to its other slot,
// and so on, at most `rounds` moves.  Safe with other lanes inserting at the
// same time (each move is one atomic exchange).  Returns false when a key is
// still homeless after the last move: that key is then missing from the
// table and the caller rebuilds the table with linear probing.
template <int HBITS>
__device__ __forceinline__ bool cuckoo_place(int32_t *key, int32_t x, int rounds) {
    uint32_t sl = hash_slot(x, HBITS);
    for (int r = 0; r < rounds; ++r) {
        const int32_t old = atomicExch(&key[sl], x);
        if (old == kEmpty) return true;
        x = old;
        const uint32_t s1 = hash_slot(x, HBITS);
        sl = s1 == sl ? hash_slot2(x, HBITS) : s1;
    }
    return false;
}

// The slot that holds x in a two-choice table (x must be in it).
template <int HBITS>
__device__ __forceinline__ uint32_t cuckoo_slot(const int32_t *key, int32_t x) {
    const uint32_t s1 = hash_slot(x, HBITS);
    return key[s1] == x ? s1 : hash_slot2(x, HBITS);
}

// The slot that holds x in a linear-probing table (x must be in it).
template <int HBITS>
__device__ __forceinline__ uint32_t linear_slot(const int32_t *key, int32_t x) {
    uint32_t sl = hash_slot(x, HBITS);
    while (key[sl] != x) sl = (sl + 1) & ((1u << HBITS) - 1);
    return sl;
}

// which = 0: tasks, 1: medium lists, 2: long lists
__device__ __forceinline__ int find_desc(const CountDesc *__restrict__ d, int nd, int64_t c, int which) {
    int lo = 0, hi = nd - 1;  // largest h whose first index is <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = which == 0 ? d[mid].task_base : (which == 1 ? d[mid].med_base : d[mid].large_base);
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

// Per-node counter add: PN 3 packs two 16-bit counters per word (slot i in
// half i & 1 of word i / 2; a slot's count stays below 2^16).
template <int PN>
__device__ __forceinline__ void cnt_add(int32_t *cnt, int i, int v) {
    if (PN == 3)
        atomicAdd(&cnt[i >> 1], v << ((i & 1) << 4));
    else
        atomicAdd(&cnt[i], v);
}

__device__ __forceinline__ int mbcnt64(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Reads col entries: buffer loads with a 32-bit byte offset when IDX32,
// global loads otherwise.
template <bool IDX32>
struct ColReader;

template <>
struct ColReader<true> {
    __amdgpu_buffer_rsrc_t rsrc;
    // col and m are the same in every lane; building the descriptor from
    // first-lane copies keeps it in scalar registers (no per-load waterfall)
    __device__ __forceinline__ ColReader(const int32_t *col, int64_t m) {
        const uint64_t base = (uint64_t)uniform64((int64_t)(uintptr_t)col);
        const int32_t bytes = uniform32((int32_t)(m * 4));
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)base, (short)0, bytes, 0x00020000);
    }
    // offsets at or past the end read 0 (hardware range check); callers mask those lanes
    __device__ __forceinline__ int32_t load(int32_t idx, bool ok) const {
        const uint32_t byte_off = ok ? (uint32_t)idx << 2 : 0xffffffffu;
        return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rsrc, byte_off, 0, 0);
    }
};

template <>
struct ColReader<false> {
    gptr_t<const int32_t> col;
    int64_t m;
    __device__ __forceinline__ ColReader(const int32_t *c, int64_t mm) : col(gview(c)), m(mm) {}
    __device__ __forceinline__ int32_t load(int64_t idx, bool ok) const {
        ok = ok && (uint64_t)idx < (uint64_t)m;
        return col[ok ? idx : 0];
    }
};

template <bool IDX32>
using idx_t = typename std::conditional<IDX32, int32_t, int64_t>::type;

// Walks the virtual sequence of target-row ids from e_begin to e_end (a
// multiple of kStep apart, e_end may pass total), kStep ids per step: marks
// the row starts that fall inside the step, finds every lane's row with one
// ballot per 64-id window, loads the 4 ids of each lane together, then probes
// them together.  `cur` is the row holding e_begin.  Row indices are clamped
// so every LDS read is valid and lanes past the end are masked.
//   IN_LDS: membership in the source list by the LDS hash (key/pos): with
//   CUCKOO a two-choice table (two independent reads per id, no loop),
//   otherwise linear probing (collision chains entered only when some lane
//   needs one);
//   otherwise by binary search in the sorted list col[rs .. rs+a) (huge lists).
// The return value is the wave's hits spread over its lanes (sum over lanes).
// Per-node counts go to LDS counters by list position, or (huge lists) to tv.
// PN, how per-node counts are kept: 0 by list position (pos[slot]; the
// one-wave kernel); 1 the same, and a step inside one row adds its target's
// share at once; 2 by table slot (tpos holds the slot of each row's target),
// with the one-row share (the 4-wave tier); 3 as 2 in 16-bit halves
// (cnt_add; the 8-wave tier).
template <int HBITS, bool PER_NODE, bool IN_LDS, bool CUCKOO, bool IDX32, int PN, class PosT>
__device__ __forceinline__ uint32_t walk_steps(const int32_t *key, const PosT *pos, const int32_t *P,
                                               const idx_t<IDX32> *base, const PosT *tpos, int32_t *cnt,
                                               uint8_t *flag, const ColReader<IDX32> &rd,
                                               gptr_t<const int32_t> gcol, int32_t nt, int32_t total, int cur,
                                               int32_t e_begin, int32_t e_end, int64_t rs, int32_t a, int32_t i0,
                                               int64_t *__restrict__ tv) {
    constexpr uint32_t kMask = (1u << HBITS) - 1;
    const int lane = __lane_id();
    uint32_t *flag_word = reinterpret_cast<uint32_t *>(flag);
    uint32_t hits = 0;   // per lane
    uint32_t whits = 0;  // per wave
    // wave-uniform by construction; first-lane copies keep them in scalar registers
    cur = uniform32(cur);
    nt = uniform32(nt);
    total = uniform32(total);
    e_begin = uniform32(e_begin);
    e_end = uniform32(e_end);
    // A step wholly inside the sequence (every step of a source but its last)
    // needs no masking of lanes past the end: the body is instantiated twice.
    auto step = [&](int32_t e0, auto full_c) {
        constexpr bool FULL = decltype(full_c)::value;
        int seg[kWin];
        int32_t w[kWin];
        bool ok[kWin];
        int acc = 0;
        const bool one_row = uniform32(P[cur + 1]) >= e0 + kStep;
        if (one_row) {
            // no row starts inside the step: every id lies in row cur
            const idx_t<IDX32> b = base[cur];
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                seg[q] = cur;
                const int32_t e = e0 + 64 * q + lane;
                ok[q] = FULL || e < total;
                w[q] = rd.load(b + e, ok[q]);
            }
        } else {
            // row starts inside (e0, e0 + kStep); rows past the last read the total
            for (int jb = cur + 1;; jb += 64) {
                const int jj = min(jb + lane, nt);
                const int32_t p = P[jj] - e0;  // >= 1
                if (p < kStep) flag[((p & 63) << 2) + (p >> 6)] = 1;
                if (readlane32(p, 63) >= kStep || jb + 63 >= nt) break;
            }
            wave_lds_sync();
            const uint32_t fw = flag_word[lane];
            flag_word[lane] = 0u;
            uint64_t M[kWin];
            int pre[kWin];
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                M[q] = __ballot(((fw >> (8 * q)) & 0xffu) != 0u);
                pre[q] = acc;
                acc += popc64(M[q]);
            }
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                seg[q] = min(cur + pre[q] + mbcnt64(M[q]) + (int)((fw >> (8 * q)) & 1u), nt - 1);
                const int32_t e = e0 + 64 * q + lane;
                ok[q] = FULL || e < total;
                w[q] = rd.load(base[seg[q]] + e, ok[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < kWin; ++q) w[q] = ok[q] ? w[q] : -1;
        if (IN_LDS) {
            uint32_t sl[kWin];
            bool hit[kWin];
            uint32_t sh = 0;  // hits of the step (scalar)
            if (CUCKOO) {
                // two-choice table: an id is in one of its two slots or absent
                uint32_t s2[kWin];
                int32_t k1[kWin], k2[kWin];
                // An id whose first slot is empty is absent: every key that
                // ever took a slot keeps it occupied, and a key sits in its
                // second slot only after its first was taken.  Lanes that need
                // no second read all read slot 0 (one broadcast), so the second
                // read touches few banks.
                bool first[kWin], need[kWin];
#pragma unroll
                for (int q = 0; q < kWin; ++q) {
                    const uint32_t p = __umul24((uint32_t)w[q], 0x9E3779u);
                    sl[q] = p >> (32 - HBITS);
                    s2[q] = (p >> (32 - 2 * HBITS)) & kMask;
                    k1[q] = key[sl[q]];
                }
#pragma unroll
                for (int q = 0; q < kWin; ++q) {
                    first[q] = k1[q] == w[q];
                    need[q] = !first[q] & (k1[q] != kEmpty);
                    k2[q] = key[need[q] ? s2[q] : 0u];
                }
#pragma unroll
                for (int q = 0; q < kWin; ++q) {
                    const bool c2 = k2[q] == w[q];
                    hit[q] = ok[q] & (first[q] | (need[q] & c2));
                    sl[q] = first[q] ? sl[q] : s2[q];
                    // the step's hits from ballots of the compares themselves
                    // (scalar masks; a ballot of a combined condition is not)
                    const uint64_t b1 = __ballot(first[q]);
                    uint64_t bh = b1 | (__ballot(k1[q] != kEmpty) & ~b1 & __ballot(c2));
                    if (!FULL) bh &= __ballot(ok[q]);
                    sh += (uint32_t)popc64(bh);
                }
            } else {
                int32_t k[kWin];
#pragma unroll
                for (int q = 0; q < kWin; ++q) {
                    sl[q] = hash_slot(w[q], HBITS);
                    k[q] = key[sl[q]];
                }
                bool need = false;
#pragma unroll
                for (int q = 0; q < kWin; ++q) need = need || (k[q] != w[q] && k[q] != kEmpty);
                if (__ballot(need)) {
#pragma unroll
                    for (int q = 0; q < kWin; ++q) {
                        while (k[q] != w[q] && k[q] != kEmpty) {  // collision chain
                            sl[q] = (sl[q] + 1) & kMask;
                            k[q] = key[sl[q]];
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kWin; ++q) {
                    hit[q] = ok[q] && k[q] == w[q];
                    sh += (uint32_t)popc64(__ballot(hit[q]));
                }
            }
            whits += sh;
            // Per-node counts: each hit adds one to the count of its id and one
            // to that of its row's target.  By table slot (PN 2) a hit's
            // counter is at hand; by list position its position is read by
            // the hit lanes only.  In the workgroup kernels (PN >= 1; long
            // rows) a step that lies in one row adds the target's share once;
            // in the one-wave kernel such steps are rarer and the extra branch
            // did not pay.
            if (PER_NODE && PN >= 1 && one_row) {
#pragma unroll
                for (int q = 0; q < kWin; ++q)
                    if (hit[q]) cnt_add<PN>(cnt, PN >= 2 ? (int)sl[q] : (int)pos[sl[q]], 1);
                if (lane == 0 && sh) cnt_add<PN>(cnt, tpos[cur], (int)sh);
            } else if (PER_NODE) {
#pragma unroll
                for (int q = 0; q < kWin; ++q) {
                    if (hit[q]) {
                        cnt_add<PN>(cnt, PN >= 2 ? (int)sl[q] : (int)pos[sl[q]], 1);
                        cnt_add<PN>(cnt, tpos[seg[q]], 1);
                    }
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < kWin; ++q) {
                if (!ok[q]) continue;
                int32_t lo = 0, hi = a;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (gcol[rs + mid] < w[q])
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < a && gcol[rs + lo] == w[q]) {
                    ++hits;
                    if (PER_NODE) {
                        add_u64(&tv[w[q]], 1);
                        add_u64(&tv[gcol[rs + i0 + tpos[seg[q]]]], 1);
                    }
                }
            }
        }
        int nc = cur + acc;
        if (nc + 1 < nt && uniform32(P[nc + 1]) == e0 + kStep) ++nc;
        cur = nc;
        wave_lds_sync();
    };
    for (int32_t e0 = e_begin; e0 < e_end; e0 += kStep) {
        if (e0 + kStep <= total)
            step(e0, std::true_type{});
        else
            step(e0, std::false_type{});
    }
    return hits + (lane == 0 ? whits : 0u);
}

// --------------------------------------------------------------- one wave

template <bool IDX32>
struct alignas(16) SmallLds {
    idx_t<IDX32> base[kSmallMax];  // per target row: row start minus its prefix
    int32_t key[kSmallHash];       // hashed source list, -1 = empty
    int32_t P[kSmallMax + 1];      // exclusive prefix of row lengths, then the total
    int32_t cnt[kSmallMax];        // per-position counts (per-node mode)
    uint8_t pos[kSmallHash];       // list position of each hashed id
    uint8_t tpos[kSmallMax];       // list position of each target row
    int32_t slen[kSmallMax];       // length of each searched row
    alignas(4) uint8_t flag[kFlagBytes];
};

// The searched rows of one source (flags q0 / q1 of lanes i and 64 + i, row
// lengths l0 / l1 and starts r0 / r1 relative to the row reader): the pairs
// (i, j), j = i+1 .. a-1, of all of them are numbered in order.  Searched row
// k sits at slot kSmallMax - 1 - k of base / tpos / slen and its first pair
// number at P[kSmallMax - k]; the walk uses slots below its own row count,
// which is at most te minus the searched rows, so the two never meet.
// Returns the number of pairs; *nrows receives the number of searched rows.
template <bool IDX32>
__device__ __forceinline__ int32_t search_setup(SmallLds<IDX32> &S, bool q0, bool q1, int32_t l0, int32_t l1,
                                                idx_t<IDX32> r0, idx_t<IDX32> r1, uint64_t Q0, uint64_t Q1,
                                                int32_t a, int *nrows) {
    const int lane = __lane_id();
    const int32_t c0 = q0 ? a - 1 - lane : 0, c1 = q1 ? a - 65 - lane : 0;
    const int32_t ic0 = wave_inclusive_sum(c0);
    const int32_t ic1 = readlane32(ic0, 63) + wave_inclusive_sum(c1);
    const int ns0 = popc64(Q0);
    if (q0) {
        const int k = mbcnt64(Q0), sl = kSmallMax - 1 - k;
        S.base[sl] = r0;
        S.slen[sl] = l0;
        S.tpos[sl] = (uint8_t)lane;
        S.P[kSmallMax - k] = ic0 - c0;
    }
    if (q1) {
        const int k = ns0 + mbcnt64(Q1), sl = kSmallMax - 1 - k;
        S.base[sl] = r1;
        S.slen[sl] = l1;
        S.tpos[sl] = (uint8_t)(64 + lane);
        S.P[kSmallMax - k] = ic1 - c1;
    }
    *nrows = uniform32(ns0 + popc64(Q1));
    return uniform32(readlane32(ic1, 63));
}

// Looks the pairs of the searched rows up, 64 per step: lane p finds its row
// by binary search over the rows' first pair numbers, takes L[j] from the
// lanes holding the list (x0 / x1), and looks it up in N_{t_i} by a
// branch-free binary search in device memory.  A hit is the triangle
// {s, t_i, L[j]}.
template <bool PER_NODE, bool IDX32>
__device__ __forceinline__ uint32_t search_pairs(SmallLds<IDX32> &S, const ColReader<IDX32> &rd, int32_t npairs,
                                                 int ns, int32_t a, int32_t x0, int32_t x1,
                                                 gptr_t<const int32_t> samp, int64_t ebase) {
    const int lane = __lane_id();
    uint32_t hits = 0;
    for (int32_t p0 = 0; p0 < npairs; p0 += 64) {
        const int32_t p = p0 + lane;
        const bool okp = p < npairs;
        int lo = 0, hi = ns - 1;  // last searched row whose first pair is <= p
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.P[kSmallMax - mid] <= p)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int sl = kSmallMax - 1 - lo;
        const int i = S.tpos[sl];
        const int j = min(i + 1 + (p - S.P[kSmallMax - lo]), a - 1);
        const int32_t xa = __shfl(x0, j & 63, 64), xb = __shfl(x1, j & 63, 64);
        const int32_t x = j < 64 ? xa : xb;
        idx_t<IDX32> rb = S.base[sl];
        int32_t n = okp ? S.slen[sl] : 1;
        if (samp && n > 1) {
            // first level: the samples inside the row (entries j * stride of
            // col, j in [js, je)) narrow the search to one stride of the row
            const int64_t g0 = ebase + (int64_t)rb, g1 = g0 + n;
            const int64_t js = (g0 + kSampleStride - 1) >> kSampleShift, je = (g1 + kSampleStride - 1) >> kSampleShift;
            int64_t b0 = g0, b1 = min(g1, js << kSampleShift);
            if (je > js && samp[js] <= x) {
                int64_t at = js, m = je - js;  // at: the last sample <= x so far
                while (m > 1) {
                    const int64_t half = m >> 1;
                    if (samp[at + half] <= x) at += half;
                    m -= half;
                }
                b0 = at << kSampleShift;
                b1 = min(g1, b0 + kSampleStride);
            }
            rb = (idx_t<IDX32>)(b0 - ebase);
            n = (int32_t)(b1 - b0);
        }
        int32_t at = 0;
        while (n > 1) {  // at: the last entry <= x so far (or 0), N_t[at .. at + n) still open
            const int32_t half = n >> 1;
            if (rd.load(rb + at + half, true) <= x) at += half;
            n -= half;
        }
        const bool hit = okp && rd.load(rb + at, true) == x;
        if (hit) {
            ++hits;
            if (PER_NODE) {
                atomicAdd(&S.cnt[i], 1);
                atomicAdd(&S.cnt[j], 1);
            }
        }
    }
    return hits;
}

// The one-wave kernel's core rows (flags z0 / z1 of targets lane and 64 +
// lane, bitmap origins o0 / o1): for each such target t_i the entries L[j],
// j > i, of the list are tested against the bitmap of N_{t_i}, lane j reading
// the word of L[j].  Per-node counts are summed in registers: c0 / c1 for the
// entries lane and 64 + lane (both the hits of L[j] and, for the entry t_i,
// those of its row).  Returns this lane's hits.
template <bool PER_NODE>
__device__ __forceinline__ uint32_t core_rows_small(gptr_t<const uint32_t> bm, uint64_t Z0, uint64_t Z1, int32_t o0,
                                                    int32_t o1, int32_t a, int32_t x0, int32_t x1, int32_t &c0,
                                                    int32_t &c1) {
    const int lane = __lane_id();
    uint32_t hits = 0;
    const int32_t s0 = x0 >> 5, s1 = x1 >> 5;
    const uint32_t m0 = 1u << (x0 & 31), m1 = 1u << (x1 & 31);
    // kRows rows per round, their words loaded together
    constexpr int kRows = 4;
    while (Z0 | Z1) {
        int i[kRows];
        int32_t og[kRows];
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
            if (Z0) {
                const int l = __builtin_ctzll(Z0);
                Z0 &= Z0 - 1;
                i[q] = l;
                og[q] = readlane32(o0, l);
            } else if (Z1) {
                const int l = __builtin_ctzll(Z1);
                Z1 &= Z1 - 1;
                i[q] = 64 + l;
                og[q] = readlane32(o1, l);
            } else {
                i[q] = 1 << 30;  // no row: every lane is masked
                og[q] = 0;
            }
        }
        uint32_t w0[kRows], w1[kRows];
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
            const bool v0 = lane > i[q] && lane < a;
            const bool v1 = 64 + lane > i[q] && 64 + lane < a;
            w0[q] = v0 ? bm[og[q] + s0] : 0u;
            w1[q] = v1 ? bm[og[q] + s1] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
            const bool h0 = (w0[q] & m0) != 0u, h1 = (w1[q] & m1) != 0u;
            hits += (uint32_t)h0 + (uint32_t)h1;
            if (PER_NODE) {
                c0 += (int32_t)h0;
                c1 += (int32_t)h1;
                const int32_t rh = popc64(__ballot(h0)) + popc64(__ballot(h1));
                if (lane == (i[q] & 63)) {
                    if (i[q] < 64)
                        c0 += rh;
                    else if (i[q] < 128)
                        c1 += rh;
                }
            }
        }
    }
    return hits;
}

// One source s whose list (a entries, 2 <= a <= 128) is already in registers:
// x0 = L[lane], x1 = L[64 + lane] (clamped copies beyond a).  The first te
// entries are the targets (te = a - 1 for a resident adjacency); their rows
// are off[t - row_lo] .. off[t - row_lo + 1].
template <bool PER_NODE, bool IDX32, bool SLICE, bool CORE>
__device__ __forceinline__ uint64_t source_small(SmallLds<IDX32> &S, const ColReader<IDX32> &rd,
                                                 gptr_t<const int32_t> gcol, gptr_t<const int64_t> off,
                                                 int64_t *__restrict__ tv, int32_t s, int32_t a, int32_t te,
                                                 int32_t row_lo, int64_t ebase, int32_t x0, int32_t x1, int lane,
                                                 int32_t sr, int rounds, gptr_t<const int32_t> samp,
                                                 gptr_t<const uint32_t> bm, int32_t br, int32_t clo, int32_t cwl,
                                                 int32_t ckw) {
    const bool h0 = lane < a, h1 = lane + 64 < a;
    bool cuckoo = rounds > 0;
    if (cuckoo) {
        bool bad = h0 && !cuckoo_place<kSmallHashBits>(S.key, x0, rounds);
        if (h1 && !bad) bad = !cuckoo_place<kSmallHashBits>(S.key, x1, rounds);
        cuckoo = __ballot(bad) == 0;
        wave_lds_sync();
        if (cuckoo) {
            if (PER_NODE && h0) S.pos[cuckoo_slot<kSmallHashBits>(S.key, x0)] = (uint8_t)lane;
            if (PER_NODE && h1) S.pos[cuckoo_slot<kSmallHashBits>(S.key, x1)] = (uint8_t)(64 + lane);
        } else {
            // a key found no place: empty the table and probe linearly instead
            int4 *kv = reinterpret_cast<int4 *>(S.key);
            kv[lane] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
            kv[64 + lane] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
            wave_lds_sync();
        }
    }
    if (!cuckoo) {
        if (h0) {
            uint32_t sl = hash_slot(x0, kSmallHashBits);
            while (atomicCAS(&S.key[sl], kEmpty, x0) != kEmpty) sl = (sl + 1) & (kSmallHash - 1);
            if (PER_NODE) S.pos[sl] = (uint8_t)lane;
        }
        if (h1) {
            uint32_t sl = hash_slot(x1, kSmallHashBits);
            while (atomicCAS(&S.key[sl], kEmpty, x1) != kEmpty) sl = (sl + 1) & (kSmallHash - 1);
            if (PER_NODE) S.pos[sl] = (uint8_t)(64 + lane);
        }
    }
    // rows of t_0 .. t_{te-1}; empty rows are dropped so row starts are distinct.
    // Loads are unconditional (every lane indexes a valid row).
    const int32_t y0 = SLICE ? (lane < te ? x0 - row_lo : 0) : x0;
    const int32_t y1 = SLICE ? (lane + 64 < te ? x1 - row_lo : 0) : x1;
    const int64_t r0 = off[y0], e0r = off[y0 + 1];
    const int64_t r1 = off[y1], e1r = off[y1 + 1];
    const int32_t l0 = lane < te ? (int32_t)(e0r - r0) : 0;
    const int32_t l1 = lane + 64 < te ? (int32_t)(e1r - r1) : 0;
    // rows searched instead of walked: at least a whole step long and longer
    // than sr times the candidates after the target (a - 1 - i >= 1 for
    // every target i < te); a shorter row shares its walk steps with others
    // rows of the dense core tested against their bitmaps instead: at least
    // kCoreMinProbe entries and longer than br times the candidates (chosen
    // first: a test reads one word where a search reads several)
    const bool z0 = CORE && br > 0 && l0 >= kCoreMinProbe && x0 >= clo && l0 > br * (a - 1 - lane);
    const bool z1 = CORE && br > 0 && l1 >= kCoreMinProbe && x1 >= clo && l1 > br * (a - 65 - lane);
    const bool q0 = !z0 && sr != 0 && l0 > 0 && (sr < 0 || (l0 >= kStep && l0 > sr * (a - 1 - lane)));
    const bool q1 = !z1 && sr != 0 && l1 > 0 && (sr < 0 || (l1 >= kStep && l1 > sr * (a - 65 - lane)));
    const int32_t b0 = (q0 || z0) ? 0 : l0, b1 = (q1 || z1) ? 0 : l1;
    const uint64_t m0 = __ballot(b0 > 0), m1 = __ballot(b1 > 0);
    const int n0 = popc64(m0);
    const int32_t inc0 = wave_inclusive_sum(b0);
    const int32_t tot0 = readlane32(inc0, 63);
    const int32_t inc1 = tot0 + wave_inclusive_sum(b1);
    const int32_t total = readlane32(inc1, 63);
    if (b0 > 0) {
        const int j = mbcnt64(m0);
        S.P[j] = inc0 - b0;
        S.base[j] = (idx_t<IDX32>)(r0 - ebase - (int64_t)(inc0 - b0));
        S.tpos[j] = (uint8_t)lane;
    }
    if (b1 > 0) {
        const int j = n0 + mbcnt64(m1);
        S.P[j] = inc1 - b1;
        S.base[j] = (idx_t<IDX32>)(r1 - ebase - (int64_t)(inc1 - b1));
        S.tpos[j] = (uint8_t)(64 + lane);
    }
    const int nt = n0 + popc64(m1);
    if (lane == 0) S.P[nt] = total;
    const uint64_t Q0 = __ballot(q0), Q1 = __ballot(q1);
    int ns = 0;
    const int32_t npairs = (Q0 | Q1) ? search_setup<IDX32>(S, q0, q1, l0, l1, (idx_t<IDX32>)(r0 - ebase),
                                                             (idx_t<IDX32>)(r1 - ebase), Q0, Q1, a, &ns)
                                     : 0;
    wave_lds_sync();

    uint32_t hits = npairs ? search_pairs<PER_NODE, IDX32>(S, rd, npairs, ns, a, x0, x1, samp, ebase) : 0u;
    {
        const uint64_t Z0 = __ballot(z0), Z1 = __ballot(z1);
        if (Z0 | Z1) {
            int32_t zc0 = 0, zc1 = 0;  // per-node counts of the core tests
            const int32_t o0 = z0 ? (int32_t)core_origin(x0, clo, ckw) : 0;
            const int32_t o1 = z1 ? (int32_t)core_origin(x1, clo, ckw) : 0;
            hits += core_rows_small<PER_NODE>(bm, Z0, Z1, o0, o1, a, x0, x1, zc0, zc1);
            // into the position counters before the walk adds to them
            if (PER_NODE && h0) S.cnt[lane] += zc0;
            if (PER_NODE && h1) S.cnt[64 + lane] += zc1;
        }
    }
    const int32_t e_end = ((total + kStep - 1) / kStep) * kStep;
    if (cuckoo)
        hits += walk_steps<kSmallHashBits, PER_NODE, true, true, IDX32, 0, uint8_t>(
            S.key, S.pos, S.P, S.base, S.tpos, S.cnt, S.flag, rd, gcol, nt, total, 0, 0, e_end, 0, a, 0, tv);
    else
        hits += walk_steps<kSmallHashBits, PER_NODE, true, false, IDX32, 0, uint8_t>(
            S.key, S.pos, S.P, S.base, S.tpos, S.cnt, S.flag, rd, gcol, nt, total, 0, 0, e_end, 0, a, 0, tv);
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
    kv[lane] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
    kv[64 + lane] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
    wave_lds_sync();
    return (uint64_t)hits;
}

// CORE: the core's bit tests compiled in (launched only for handles whose
// core has rows long enough to take them; the code costs the other lists'
// walk a few registers).
template <bool PER_NODE, bool IDX32, bool SLICE, bool CORE>
__global__ __launch_bounds__(kSmallWaves * 64) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_count_small(
    const CountDesc *__restrict__ descs, int ndesc, int64_t total_tasks, uint32_t *__restrict__ head, int nworkers,
    unsigned long long *__restrict__ times, int rounds) {
    __shared__ SmallLds<IDX32> lds[kSmallWaves];
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int64_t me = (int64_t)blockIdx.x * kSmallWaves + wave;
    if (times && lane == 0) times[2 * me] = wall_clock64();
    SmallLds<IDX32> &S = lds[wave];
    for (int i = lane; i < kSmallHash; i += 64) S.key[i] = kEmpty;
    for (int i = lane; i < kSmallMax; i += 64) S.cnt[i] = 0;
    for (int i = lane; i < kFlagBytes; i += 64) S.flag[i] = 0;
    wave_lds_sync();

    int64_t c = (int64_t)blockIdx.x * kSmallWaves + wave;
    while (c < total_tasks) {
        const int h = ndesc > 1 ? find_desc(descs, ndesc, c, 0) : 0;
        // source lists (soff / scol) and target rows (off / col) are the same
        // adjacency unless this is a slice launch
        const gptr_t<const int32_t> col = gview(SLICE ? descs[h].scol : descs[h].col);
        const gptr_t<const int64_t> soff = gview(SLICE ? descs[h].soff : descs[h].off);
        const gptr_t<const int64_t> off = gview(descs[h].off);
        int64_t *__restrict__ tv = descs[h].tv;
        const int32_t row_lo = SLICE ? descs[h].row_lo : 0;
        const int64_t lt = c - descs[h].task_base;
        // the scan starts past the task's leading nodes of degree < 2 when the
        // build recorded where they end
        const int32_t v0 = descs[h].start ? descs[h].start[lt] : descs[h].bnd[lt], v1 = descs[h].bnd[lt + 1];
        const int g = descs[h].gid ? descs[h].gid[lt] : 0;
        // rows are addressed from the first entry of the task's graph
        int64_t ebase = 0, mg = descs[h].m;
        if (!SLICE && descs[h].k > 1) {
            ebase = off[descs[h].node_base[g]];
            mg = off[descs[h].node_base[g + 1]] - ebase;
        }
        const ColReader<IDX32> rd(descs[h].col + ebase, mg);
        const int small_max = descs[h].small_max;
        const int32_t sr = uniform32(descs[h].search_ratio);
        // slices hold no samples of their rows
        const gptr_t<const int32_t> samp = gview(SLICE ? (const int32_t *)nullptr : descs[h].samp);
        // nor a core
        const gptr_t<const uint32_t> bm = gview(SLICE || !CORE ? (const uint32_t *)nullptr : descs[h].bm);
        const int32_t br = bm ? uniform32(descs[h].bitmap_ratio) : 0;
        const int32_t clo = uniform32(descs[h].core_lo), cwl = uniform32(descs[h].core_wl);
        const int32_t ckw = uniform32(descs[h].core_kw);
        uint64_t tri = 0;
        for (int32_t s0 = v0; s0 < v1; s0 += 64) {
            const int32_t sv = min(s0 + lane, v1 - 1);
            const int64_t o0 = soff[sv], o1 = soff[sv + 1];
            const int32_t al = s0 + lane < v1 ? (int32_t)(o1 - o0) : 0;
            // targets per source: all entries but the last, or the resident prefix
            const int32_t tl = SLICE ? min(descs[h].tcnt[sv], al - 1) : al - 1;
            const int32_t lab = SLICE ? descs[h].sid[sv] : sv;
            uint64_t work = __ballot(al >= 2 && al <= small_max && tl > 0);
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
                const int32_t te = readlane32(tl, j);
                const int32_t sl = SLICE ? readlane32(lab, j) : s0 + j;
                tri += source_small<PER_NODE, IDX32, SLICE, CORE>(S, rd, col, off, tv, sl, a, te, row_lo, ebase, x0, x1,
                                                            lane, sr, rounds, samp, bm, br, clo, cwl, ckw);
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
    if (times && lane == 0) times[2 * me + 1] = wall_clock64();
}

// ---------------------------------------------------------- one workgroup

// Long lists: one workgroup per list.  Two tiers share this code: lists up to
// 768 entries go to 4-wave workgroups with a ~24 KB LDS table (six per
// compute unit), longer ones to 8-wave workgroups with a ~52 KB table (three
// per compute unit; the kernel is held to 80 registers so that 24 waves fit).
// Lists are handed out longest-rank first (roughly longest first).
// Per-node counts are kept by table slot: CNT 1 one 32-bit counter per slot,
// 2 two 16-bit counters per word.
template <int WAVES, int LMAX, int HBITS, bool IDX32, int CNT>
struct WideLds {
    static constexpr int kCnt = CNT;
    static constexpr int kLmax = LMAX;
    static constexpr int kAndWords = (int)((sizeof(idx_t<IDX32>) * LMAX + 4 * (LMAX + 1) + 4 * (1 << HBITS)) / 4);
    // the walk's row table and hashed list, or (a source of the core met by
    // bitmap AND) the bitmap of its list
    union {
        struct {
            idx_t<IDX32> base[LMAX];
            int32_t P[LMAX + 1];
            int32_t key[1 << HBITS];
        };
        uint32_t vbits[kAndWords];
    };
    int32_t cnt[CNT == 1 ? (1 << HBITS) : (1 << HBITS) / 2];  // per-node counts by slot
    int16_t tpos[LMAX];  // per target row: its target's slot (lists in LDS) or list position
    alignas(4) uint8_t flag[WAVES][kFlagBytes];
    int32_t wsum[WAVES];
    int32_t wcnt[WAVES];
    int32_t wcore[WAVES];
    uint64_t whits[WAVES];
    int64_t item;
    int32_t homeless;  // some key found no place in the two-choice table
};

// Lays out the rows of targets i in [i0, i1) (positions in the source list
// `col` from rs; target t has row t - row_lo of off) into P / base / tpos.
// tpos: the target's slot in the LDS table (TABLE 1: two-choice, 2: linear
// probing) or, with TABLE 0, its list position relative to i0.  Returns (rows,
// total ids).  With br > 0 (a list in LDS, a - 1 - i candidates after target
// i), a target row of the dense core with kCoreMinProbe entries or more that
// is longer than br times its candidates is left out of the walk and listed
// for core_rows_wide instead: core row k (in list order) keeps its target in
// P[LMAX - k], its bitmap origin in base[LMAX - 1 - k] and its slot in
// tpos[LMAX - 1 - k].  The walk's rows and the core rows together are at most
// the targets, fewer than LMAX, so the two ends never meet.
template <int WAVES, int HBITS, bool IDX32, class L>
__device__ __forceinline__ void wide_rows(L &S, gptr_t<const int32_t> col, gptr_t<const int64_t> off, int64_t rs,
                                          int32_t i0, int32_t i1, int32_t row_lo, int64_t ebase, int table,
                                          int32_t a, int32_t br, int32_t clo, int32_t cwl, int32_t ckw,
                                          int32_t *nt_out, int32_t *total_out, int32_t *nc_out) {
    constexpr int kThreadsW = WAVES * 64;
    constexpr int LMAX = L::kLmax;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    int32_t carry_n = 0, carry_sum = 0, carry_c = 0;
    for (int32_t rb = i0; rb < i1; rb += kThreadsW) {
        const int32_t i = rb + (int32_t)threadIdx.x;
        const int32_t x = col[rs + min(i, i1 - 1)], t = x - row_lo;
        const int64_t r = off[t], re = off[t + 1];
        const int32_t len = i < i1 ? (int32_t)(re - r) : 0;
        const bool z = br > 0 && len >= kCoreMinProbe && x >= clo && len > br * (a - 1 - i);
        const int32_t b = z ? 0 : len;
        const int32_t inc = wave_inclusive_sum(b);
        const uint64_t m = __ballot(b > 0);
        const uint64_t mz = __ballot(z);
        if (lane == 63) {
            S.wsum[wave] = inc;
            S.wcnt[wave] = popc64(m);
            S.wcore[wave] = popc64(mz);
        }
        __syncthreads();
        int32_t sb = 0, cb = 0, st = 0, ct = 0, zb = 0, zt = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const int32_t ws = S.wsum[w], wc = S.wcnt[w], wz = S.wcore[w];
            if (w < wave) {
                sb += ws;
                cb += wc;
                zb += wz;
            }
            st += ws;
            ct += wc;
            zt += wz;
        }
        if (b > 0 || z) {
            const int16_t slot = (int16_t)(table == 1   ? cuckoo_slot<HBITS>(S.key, x)
                                           : table == 2 ? linear_slot<HBITS>(S.key, x)
                                                        : (uint32_t)(i - i0));
            if (z) {
                const int k = carry_c + zb + mbcnt64(mz);
                S.P[LMAX - k] = x;
                S.base[LMAX - 1 - k] = (idx_t<IDX32>)core_origin(x, clo, ckw);
                S.tpos[LMAX - 1 - k] = slot;
            } else {
                const int j = carry_n + cb + mbcnt64(m);
                const int32_t p = carry_sum + sb + inc - b;
                S.P[j] = p;
                S.base[j] = (idx_t<IDX32>)(r - ebase - (int64_t)p);
                S.tpos[j] = slot;
            }
        }
        carry_n += ct;
        carry_sum += st;
        carry_c += zt;
        __syncthreads();
    }
    if (threadIdx.x == 0) S.P[carry_n] = carry_sum;
    __syncthreads();
    *nt_out = uniform32(carry_n);
    *total_out = uniform32(carry_sum);
    *nc_out = uniform32(carry_c);
}

// The core rows listed by wide_rows (nc of them): for each, the list entries
// after its target are tested against the target's bitmap.  The list goes in
// chunks of 64 entries, chunk c to wave c mod WAVES; a chunk meets the core
// rows whose target is below its largest entry (a prefix: targets ascend),
// lane j reading the word of L[j] for every row whose target precedes L[j].
// Per-node counts: a row's hits go to its target's slot counter, an entry's
// hits over all rows to its own.  Returns this lane's hits.
template <int WAVES, int HBITS, bool PER_NODE, int PN, class L>
__device__ __forceinline__ uint32_t core_rows_wide(L &S, gptr_t<const int32_t> col, int64_t rs, int32_t a,
                                                   int32_t nc, gptr_t<const uint32_t> bm, bool cuckoo) {
    constexpr int LMAX = L::kLmax;
    const int lane = __lane_id();
    const int wave = uniform32(threadIdx.x >> 6);
    uint32_t hits = 0;
    const int32_t nch = (a + 63) >> 6;
    for (int32_t c = wave; c < nch; c += WAVES) {
        const int32_t j = c * 64 + lane;
        const bool in = j < a;
        const int32_t x = col[rs + min(j, a - 1)];
        const int32_t xmax = readlane32(x, 63);  // the chunk's largest entry (clamped lanes repeat the last)
        int lo = 0, hi = nc;  // rows whose target is below xmax: [0, lo)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (uniform32(S.P[LMAX - mid]) < xmax)
                lo = mid + 1;
            else
                hi = mid;
        }
        const int32_t sw = x >> 5;
        const uint32_t mb = 1u << (x & 31);
        int32_t acc = 0;
        if (!PER_NODE) {
            constexpr int kRowBatch = 8;
            for (int k0 = 0; k0 < lo; k0 += kRowBatch) {
                uint32_t w[kRowBatch];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) {
                    const int k = min(k0 + q, lo - 1);
                    const int32_t u = S.P[LMAX - k];
                    const int32_t org = (int32_t)S.base[LMAX - 1 - k];
                    w[q] = in && x > u && k0 + q < lo ? bm[org + sw] : 0u;
                }
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) acc += (w[q] & mb) != 0u ? 1 : 0;
            }
        } else {
            // kRowBatch rows at a time: their words loaded together, their row
            // counts added by one lane after the ballots
            constexpr int kRowBatch = 8;
            for (int k0 = 0; k0 < lo; k0 += kRowBatch) {
                uint32_t w[kRowBatch];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) {
                    const int k = min(k0 + q, lo - 1);
                    const int32_t u = S.P[LMAX - k];
                    const int32_t org = (int32_t)S.base[LMAX - 1 - k];
                    w[q] = in && x > u && k0 + q < lo ? bm[org + sw] : 0u;
                }
                int rh[kRowBatch];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) {
                    const bool h = (w[q] & mb) != 0u;
                    acc += (int32_t)h;
                    rh[q] = popc64(__ballot(h));
                }
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < kRowBatch; ++q)
                        if (rh[q]) cnt_add<PN>(S.cnt, S.tpos[LMAX - 1 - (k0 + q)], rh[q]);
                }
            }
        }
        hits += (uint32_t)acc;
        if (PER_NODE && acc)
            cnt_add<PN>(S.cnt, cuckoo ? cuckoo_slot<HBITS>(S.key, x) : linear_slot<HBITS>(S.key, x), acc);
    }
    return hits;
}

// This wave's contiguous share of the virtual sequence, in whole steps.
template <int WAVES, int HBITS, bool PER_NODE, bool IDX32, class L>
__device__ __forceinline__ uint64_t wide_windows(L &S, const ColReader<IDX32> &rd, gptr_t<const int32_t> gcol,
                                                 int64_t *__restrict__ tv, int64_t rs, int32_t a, int32_t i0,
                                                 int32_t nt, int32_t total, bool in_lds, bool cuckoo) {
    const int wave = uniform32(threadIdx.x >> 6);  // the same in every lane of the wave
    const int32_t nsteps = (total + kStep - 1) / kStep;
    const int32_t per = (nsteps + WAVES - 1) / WAVES;
    const int32_t s0 = wave * per;
    const int32_t s1 = min(nsteps, s0 + per);
    if (s0 >= s1) return 0;
    const int32_t e_begin = s0 * kStep;
    int lo = 0, hi = nt - 1;  // row holding e_begin: last row whose start is <= it
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (uniform32(S.P[mid]) <= e_begin)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (in_lds && cuckoo)
        return walk_steps<HBITS, PER_NODE, true, true, IDX32, L::kCnt + 1, int16_t>(
            S.key, S.tpos, S.P, S.base, S.tpos, S.cnt, S.flag[wave], rd, gcol, nt, total, lo, e_begin, s1 * kStep, rs,
            a, i0, tv);
    if (in_lds)
        return walk_steps<HBITS, PER_NODE, true, false, IDX32, L::kCnt + 1, int16_t>(
            S.key, S.tpos, S.P, S.base, S.tpos, S.cnt, S.flag[wave], rd, gcol, nt, total, lo, e_begin, s1 * kStep, rs,
            a, i0, tv);
    return walk_steps<HBITS, PER_NODE, false, false, IDX32, L::kCnt + 1, int16_t>(
        S.key, S.tpos, S.P, S.base, S.tpos, S.cnt, S.flag[wave], rd, gcol, nt, total, lo, e_begin, s1 * kStep, rs, a,
        i0, tv);
}

// A source v of the core: every entry of N_v lies in the core too.  N_v is
// a bitmap in LDS (vbits, words from clo >> 5), and two lists meet by AND-ing
// it with core rows word by word: (n - v) / 32 words instead of |N_u| ids,
// fewer by the rows' density.  List entries go to the waves in turn, each
// wave's lanes over consecutive words.
//
// Total only: for each target u, N_v intersect N_u is the AND with row u over
// the labels above u.  Returns this lane's hits.
template <int WAVES, class L>
__device__ __forceinline__ uint32_t core_and_total(L &S, gptr_t<const int32_t> col, int64_t rs, int32_t te,
                                                   gptr_t<const uint32_t> bm, int32_t clo, int32_t cwl, int32_t ckw) {
    const int lane = __lane_id();
    const int wave = uniform32(threadIdx.x >> 6);
    const int32_t wv0 = clo >> 5;
    uint32_t hits = 0;
    for (int32_t i = wave; i < te; i += WAVES) {
        const int32_t u = uniform32(col[rs + i]);
        const int64_t org = core_origin(u, clo, ckw);
        const int32_t w0 = (u + 1) >> 5;
        const uint32_t m0 = ~0u << ((u + 1) & 31);  // labels above u in the first word
        for (int32_t w = w0 + lane; w <= cwl; w += 64) {
            const uint32_t x = bm[org + w] & S.vbits[w - wv0] & (w == w0 ? m0 : ~0u);
            hits += (uint32_t)__popc(x);
        }
    }
    return hits;
}

// Per node: for each entry x of N_v, the AND with the whole row x counts the
// entries of N_v adjacent to x, that is the triangles {v, x, w} found from v,
// which is x's share; every such triangle is found from both of its other
// entries, so v's share is half the sum (the caller halves it).  Adds the
// shares of the entries to tv and returns this lane's part of the sum.
template <int WAVES, class L>
__device__ __forceinline__ uint32_t core_and_per_node(L &S, gptr_t<const int32_t> col, int64_t rs, int32_t a,
                                                      int32_t v, gptr_t<const uint32_t> bm, int32_t clo,
                                                      int32_t cwl, int32_t ckw, int64_t *__restrict__ tv) {
    const int lane = __lane_id();
    const int wave = uniform32(threadIdx.x >> 6);
    const int32_t wv0 = clo >> 5;
    const int32_t w0 = (v + 1) >> 5;  // N_v lies above v
    uint32_t hits = 0;
    for (int32_t i = wave; i < a; i += WAVES) {
        const int32_t x = uniform32(col[rs + i]);
        const int64_t org = core_origin(x, clo, ckw);
        uint32_t t = 0;
        for (int32_t w = w0 + lane; w <= cwl; w += 64) t += (uint32_t)__popc(bm[org + w] & S.vbits[w - wv0]);
        hits += t;
        const uint64_t tx = wave_sum((uint64_t)t);
        if (tx && lane == 0) add_u64(&tv[x], tx);
    }
    return hits;
}

// tier 1: lists in big[0, nmed); tier 2: lists in big[nmed, nbig)
template <bool PER_NODE, bool IDX32, int WAVES, int LMAX, int HBITS, int TIER, bool SLICE>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(WAVES == 8 ? 6 : 1))) void k_count_wide(const CountDesc *__restrict__ descs, int ndesc,
                                                           int64_t total_items, uint32_t *__restrict__ head,
                                                           int lds_max, unsigned long long *__restrict__ times,
                                                           int rounds) {
    constexpr int kThreadsW = WAVES * 64;
    constexpr int kHash = 1 << HBITS;
    // the 4-wave tier counts by slot; the 8-wave tier by slot in 16-bit
    // halves (32-bit counters by slot would take its LDS past what lets three
    // of its workgroups share a CU)
    constexpr int CNT = TIER == 1 ? 1 : 2;
    using L_t = WideLds<WAVES, LMAX, HBITS, IDX32, CNT>;
    __shared__ L_t S;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int cap = min(lds_max, LMAX);
    for (int i = threadIdx.x; i < kHash; i += kThreadsW) S.key[i] = kEmpty;
    for (int i = threadIdx.x; i < (int)(sizeof(S.cnt) / 4); i += kThreadsW) S.cnt[i] = 0;
    for (int i = threadIdx.x; i < WAVES * kFlagBytes; i += kThreadsW) (&S.flag[0][0])[i] = 0;
    if (threadIdx.x == 0) {
        S.item = blockIdx.x;
        S.homeless = 0;
        if (times) times[2 * blockIdx.x] = wall_clock64();
    }
    __syncthreads();

    for (;;) {
        const int64_t item = S.item;
        if (item >= total_items) break;
        const int h = ndesc > 1 ? find_desc(descs, ndesc, item, TIER) : 0;
        // source list in col (= scol of a slice launch), target rows in off / rd
        const gptr_t<const int32_t> col = gview(SLICE ? descs[h].scol : descs[h].col);
        const gptr_t<const int64_t> soff = gview(SLICE ? descs[h].soff : descs[h].off);
        const gptr_t<const int64_t> off = gview(descs[h].off);
        int64_t *__restrict__ tv = descs[h].tv;
        const int32_t row_lo = SLICE ? descs[h].row_lo : 0;
        const int64_t first = TIER == 1 ? 0 : descs[h].nmed;
        const int64_t count = TIER == 1 ? descs[h].nmed : descs[h].nbig - descs[h].nmed;
        const int64_t local = item - (TIER == 1 ? descs[h].med_base : descs[h].large_base);
        const int32_t si = descs[h].big[first + (count - 1 - local)];
        const int64_t rs = soff[si];
        const int32_t a = (int32_t)(soff[si + 1] - rs);
        const int32_t te = SLICE ? min(descs[h].tcnt[si], a - 1) : a - 1;
        const int32_t s = SLICE ? descs[h].sid[si] : si;
        const int g = graph_of(descs[h].node_base, descs[h].k, s);
        // rows are addressed from the first entry of the source's graph
        int64_t ebase = 0, mg = descs[h].m;
        if (!SLICE && descs[h].k > 1) {
            ebase = off[descs[h].node_base[g]];
            mg = off[descs[h].node_base[g + 1]] - ebase;
        }
        const ColReader<IDX32> rd(descs[h].col + ebase, mg);
        // slices hold no core
        const gptr_t<const uint32_t> bm = gview(SLICE ? (const uint32_t *)nullptr : descs[h].bm);
        const int32_t br = bm ? uniform32(descs[h].bitmap_ratio) : 0;
        const int32_t clo = uniform32(descs[h].core_lo), cwl = uniform32(descs[h].core_wl);
        const int32_t ckw = uniform32(descs[h].core_kw);
        uint64_t hits = 0;
        bool halve = false;  // hits counted twice (core AND, per node)
        if (te <= 0) {
            // no resident target (slice launches only)
        } else if (a <= cap) {
            // a source of the core whose list fills 1 / kAndDensity of the labels
            // above it (2 / kAndDensity per node) and whose bitmap fits the LDS:
            // AND of bitmaps
            const bool use_and = br > 0 && s >= clo && ckw <= L_t::kAndWords &&
                                 (int64_t)(PER_NODE ? kAndDensity / 2 : kAndDensity) * a >=
                                     (((int64_t)cwl << 5) | 31) - s;
            halve = use_and && PER_NODE;
            const bool table = !use_and;  // the walk's table
            if (rounds > 0 && table) {
                bool bad = false;
                for (int32_t k = threadIdx.x; k < a && !bad; k += kThreadsW)
                    bad = !cuckoo_place<HBITS>(S.key, col[rs + k], rounds);
                if (__ballot(bad) && lane == 0) S.homeless = 1;
                __syncthreads();
            }
            const bool cuckoo = rounds > 0 && !S.homeless;
            if (!cuckoo && table) {
                if (rounds > 0) {
                    // a key found no place: empty the table and probe linearly instead
                    for (int i = threadIdx.x; i < kHash; i += kThreadsW) S.key[i] = kEmpty;
                    __syncthreads();
                }
                for (int32_t k = threadIdx.x; k < a; k += kThreadsW) {
                    const int32_t x = col[rs + k];
                    uint32_t sl = hash_slot(x, HBITS);
                    while (atomicCAS(&S.key[sl], kEmpty, x) != kEmpty) sl = (sl + 1) & (kHash - 1);
                }
            }
            __syncthreads();
            if (use_and) {
                for (int i = threadIdx.x; i < ckw; i += kThreadsW) S.vbits[i] = 0u;
                __syncthreads();
                for (int32_t k = threadIdx.x; k < a; k += kThreadsW) {
                    const int32_t x = col[rs + k];
                    atomicOr(&S.vbits[(x >> 5) - (clo >> 5)], 1u << (x & 31));
                }
                __syncthreads();
                if (PER_NODE)
                    hits = core_and_per_node<WAVES>(S, col, rs, a, s, bm, clo, cwl, ckw, tv);
                else
                    hits = core_and_total<WAVES>(S, col, rs, te, bm, clo, cwl, ckw);
            } else {
                int32_t nt, total, nc;
                wide_rows<WAVES, HBITS, IDX32>(S, col, off, rs, 0, te, row_lo, ebase, cuckoo ? 1 : 2, a, br, clo,
                                               cwl, ckw, &nt, &total, &nc);
                if (nc > 0)
                    hits = core_rows_wide<WAVES, HBITS, PER_NODE, CNT + 1>(S, col, rs, a, nc, bm, cuckoo);
                hits += wide_windows<WAVES, HBITS, PER_NODE, IDX32>(S, rd, col, tv, rs, a, 0, nt, total, true,
                                                                    cuckoo);
            }
            __syncthreads();
            // counts out (one atomic per non-zero counter), then the table emptied
            if (PER_NODE && CNT == 2) {
                for (int w = threadIdx.x; w < kHash / 2; w += kThreadsW) {
                    const uint32_t c = (uint32_t)S.cnt[w];
                    if (c) {
                        if (c & 0xffffu) add_u64(&tv[S.key[2 * w]], (uint64_t)(c & 0xffffu));
                        if (c >> 16) add_u64(&tv[S.key[2 * w + 1]], (uint64_t)(c >> 16));
                        S.cnt[w] = 0;
                    }
                }
                __syncthreads();
            }
            for (int i = threadIdx.x; i < kHash; i += kThreadsW) {
                if (PER_NODE && CNT == 1) {
                    const int32_t c = S.cnt[i];
                    if (c) {
                        add_u64(&tv[S.key[i]], (uint64_t)c);
                        S.cnt[i] = 0;
                    }
                }
                S.key[i] = kEmpty;
            }
        } else {
            for (int32_t i0 = 0; i0 < te; i0 += cap) {
                const int32_t i1 = min(te, i0 + cap);
                int32_t nt, total, nc;
                wide_rows<WAVES, HBITS, IDX32>(S, col, off, rs, i0, i1, row_lo, ebase, 0, a, 0, 0, 0, 0, &nt,
                                               &total, &nc);
                hits += wide_windows<WAVES, HBITS, PER_NODE, IDX32>(S, rd, col, tv, rs, a, i0, nt, total, false,
                                                                    false);
                __syncthreads();
            }
        }
        const uint64_t wh = wave_sum(hits);
        if (lane == 0) S.whits[wave] = wh;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t H = 0;
            for (int w = 0; w < WAVES; ++w) H += S.whits[w];
            if (halve) H >>= 1;
            if (H) {
                add_u64(&descs[h].totals[g], H);
                if (PER_NODE) add_u64(&tv[s], H);
            }
            S.homeless = 0;
            S.item = (int64_t)gridDim.x + (int64_t)atomicAdd(head, 1u);
        }
        __syncthreads();
    }
    if (times && threadIdx.x == 0) times[2 * blockIdx.x + 1] = wall_clock64();
}

__global__ void k_scatter(const int64_t *__restrict__ tv, const int32_t *__restrict__ perm, int64_t n,
                          int64_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[perm[i]] = tv[i];
}

// Clustering coefficients from the per-node counts: coeff[perm[i]] =
// tv[i] / C(deg[i], 2) (0 below two neighbours) and, per graph, the number of
// paths of length two, sum of C(deg, 2), added into wedges (one atomic per run
// of equal graphs in a wave).
__global__ void k_clustering(const int64_t *__restrict__ tv, const int32_t *__restrict__ deg,
                             const int32_t *__restrict__ perm, int64_t N, const int64_t *__restrict__ node_base,
                             int k, double *__restrict__ coeff, unsigned long long *__restrict__ wedges) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < N; b0 += stride) {
        const int64_t i = b0 + threadIdx.x;
        int64_t pairs = 0;
        int g = -1;
        if (i < N) {
            const int64_t d = deg[i];
            pairs = d * (d - 1) / 2;
            if (coeff) coeff[perm[i]] = pairs > 0 ? (double)tv[i] / (double)pairs : 0.0;
            g = graph_of(node_base, k, i);
        }
        // sum pairs over lanes of the same graph (graphs are label ranges)
        uint64_t sum = (uint64_t)pairs;
#pragma unroll
        for (int dlt = 1; dlt < 64; dlt <<= 1) {
            const uint64_t y = __shfl_up(sum, dlt, 64);
            const int gy = __shfl_up(g, dlt, 64);
            if (__lane_id() >= dlt && gy == g) sum += y;
        }
        const int gn = __shfl_down(g, 1, 64);
        const bool end = __lane_id() == 63 || gn != g;
        if (i < N && end && sum) atomicAdd(&wedges[g], (unsigned long long)sum);
    }
}

__global__ void k_transitivity(const int64_t *__restrict__ totals, const unsigned long long *__restrict__ wedges,
                               int k, double *__restrict__ trans) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < k; g += gridDim.x * blockDim.x)
        trans[g] = wedges[g] ? (double)(3 * totals[g]) / (double)wedges[g] : 0.0;
}

template <bool PER_NODE, bool IDX32, bool SLICE>
void launch_all(CountLaunch &L, int lds_max, hipStream_t s) {
    const int cus = device_cu_count();
    // per-worker timestamps: each launch gets its own slice of L.times
    int64_t used = 0;
    auto times_for = [&](int64_t workers) -> unsigned long long * {
        if (!L.times || used + workers > L.times_cap) return nullptr;
        unsigned long long *p = L.times + 2 * used;
        used += workers;
        return p;
    };
    if (L.total_tasks > 0) {
        // never launch more workers than can be resident at once: a worker that
        // starts late would hold its first task until the end
        int per_cu = 0;
        auto kern = L.core && !SLICE ? k_count_small<PER_NODE, IDX32, SLICE, true>
                                     : k_count_small<PER_NODE, IDX32, SLICE, false>;
        TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kSmallWaves * 64, 0));
        const int64_t resident = (int64_t)std::max(1, per_cu) * cus;
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(L.workers, kSmallWaves), resident));
        unsigned long long *tm = times_for((int64_t)blocks * kSmallWaves);
        L.times_tier[0] = tm ? (int64_t)blocks * kSmallWaves : 0;
        kern<<<blocks, kSmallWaves * 64, 0, s>>>(L.descs, L.ndesc, L.total_tasks, L.heads, blocks * kSmallWaves, tm,
                                                 L.cuckoo_rounds);
        TC_LAUNCH_CHECK();
    }
    if (L.total_med > 0) {
        int per_cu = 0;
        TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_count_wide<PER_NODE, IDX32, kMedWaves, kMedMax, kMedHashBits, 1, SLICE>, kMedWaves * 64, 0));
        const int blocks = (int)std::min<int64_t>((int64_t)std::max(1, per_cu) * cus, L.total_med);
        unsigned long long *tm = times_for(blocks);
        L.times_tier[1] = tm ? blocks : 0;
        k_count_wide<PER_NODE, IDX32, kMedWaves, kMedMax, kMedHashBits, 1, SLICE>
            <<<blocks, kMedWaves * 64, 0, s>>>(L.descs, L.ndesc, L.total_med, L.heads + 1, lds_max, tm,
                                               L.cuckoo_rounds);
        TC_LAUNCH_CHECK();
    }
    if (L.total_large > 0) {
        int per_cu = 0;
        TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_count_wide<PER_NODE, IDX32, kBigWaves, kLdsMax, kBigHashBits, 2, SLICE>, kBigThreads, 0));
        const int blocks = (int)std::min<int64_t>((int64_t)std::max(1, per_cu) * cus, L.total_large);
        unsigned long long *tm = times_for(blocks);
        L.times_tier[2] = tm ? blocks : 0;
        k_count_wide<PER_NODE, IDX32, kBigWaves, kLdsMax, kBigHashBits, 2, SLICE>
            <<<blocks, kBigThreads, 0, s>>>(L.descs, L.ndesc, L.total_large, L.heads + 2, lds_max, tm,
                                            L.cuckoo_rounds);
        TC_LAUNCH_CHECK();
    }
    L.times_used = used;
}

}  // namespace

int max_small_list() { return kSmallMax; }
int max_medium_list() { return kMedMax; }
int max_lds_list() { return kLdsMax; }

int small_kernel_waves_per_cu(bool per_node) {
    static int cached[2] = {0, 0};
    int &c = cached[per_node ? 1 : 0];
    if (!c) {
        int blocks = 0;
        if (per_node)
            TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_count_small<true, false, false, false>,
                                                                kSmallWaves * 64, 0));
        else
            TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_count_small<false, false, false, false>,
                                                                kSmallWaves * 64, 0));
        c = std::max(1, blocks) * kSmallWaves;
    }
    return c;
}

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

int64_t max_timed_workers() {
    // resident small-list waves plus one workgroup tier's resident blocks each
    return (int64_t)device_cu_count() * (8 * kSmallWaves + 16 + 1);
}

void count_launch(CountLaunch &L, hipStream_t s) {
    const int lds_max = L.lds_max < 2 ? kLdsMax : (L.lds_max > kLdsMax ? kLdsMax : L.lds_max);
    // 32-bit row addressing needs every descriptor's adjacency below 2^29
    // entries; TC_FORCE_INDEX64=1 selects the 64-bit path anyway (testing)
    static const bool force64 = [] {
        const char *e = std::getenv("TC_FORCE_INDEX64");
        return e && e[0] == '1';
    }();
    const bool idx32 = !force64 && L.max_m < ((int64_t)1 << 29);
    // TC_CUCKOO_ROUNDS=<r> replaces the eviction limit of the two-choice
    // tables (testing: a small limit sends many lists to the linear fallback)
    static const int env_rounds = [] {
        const char *e = std::getenv("TC_CUCKOO_ROUNDS");
        return e && e[0] ? std::atoi(e) : -1;
    }();
    if (L.cuckoo_rounds > 0 && env_rounds >= 0) L.cuckoo_rounds = env_rounds;
    if (L.slice) {
        // slices are sized below 2^29 entries
        if (L.max_m >= ((int64_t)1 << 29)) throw Error(TC_ERR_TOO_LARGE, "slice of 2^29 or more entries");
        if (L.per_node)
            launch_all<true, true, true>(L, lds_max, s);
        else
            launch_all<false, true, true>(L, lds_max, s);
    } else if (L.per_node) {
        if (idx32)
            launch_all<true, true, false>(L, lds_max, s);
        else
            launch_all<true, false, false>(L, lds_max, s);
    } else {
        if (idx32)
            launch_all<false, true, false>(L, lds_max, s);
        else
            launch_all<false, false, false>(L, lds_max, s);
    }
}

void clustering_epilogue(const int64_t *tv, const int32_t *deg, const int32_t *perm, int64_t N,
                         const int64_t *node_base, int k, const int64_t *totals, double *coeff, double *trans,
                         unsigned long long *wedges, hipStream_t s) {
    fill_zero(wedges, (size_t)std::max(k, 1) * 8, s);
    if (N > 0) {
        const int64_t b = std::min<int64_t>(ceil_div(N, 256 * 4), 1 << 20);
        k_clustering<<<(unsigned)b, 256, 0, s>>>(tv, deg, perm, N, node_base, k, coeff, wedges);
        TC_LAUNCH_CHECK();
    }
    if (trans) {
        k_transitivity<<<(unsigned)ceil_div(std::max(k, 1), 256), 256, 0, s>>>(totals, wedges, k, trans);
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
