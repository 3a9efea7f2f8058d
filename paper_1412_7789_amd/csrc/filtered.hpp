// Device side of the filtered scan: helpers, the candidate filter, the
// walk and the streaming kernel (templates), shared by the kernel library's
// translation units.  Each filtered_*.hip file instantiates the kernels of
// one sampling stride (and, at stride 1, one prefix length), so they compile
// in parallel; kernels.hip holds the other kernels and the launch code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pfac_internal.hpp"

namespace pfac {
namespace dev {

constexpr int kQueueCap = 256;   // per-wave candidate queue (entries)
// Hit records a wave keeps in LDS before it spills further ones to its
// global region.  Global stores in the streaming loop stall it (a later wait
// for the next chunk's loads also waits for them, and the data registers a
// store reads cannot be reused until it is done), so records stay on chip.
constexpr int kLdsHits = 64;
constexpr int kDrain = 64;       // candidates taken per drain (1 per lane; 128 and 192 measured slower)
// A queue holds fewer than kDrain entries before a push round and gains at
// most one per lane in it, so its last entries are never used by the queue:
// the last dword of the first wave's queue holds the block's slot counter.
static_assert(2 * kDrain <= kQueueCap - 4, "queue room");
constexpr int kMaxWaves = 16;    // waves per block at most (1024 threads)
// AC_FILTER_PAIR20 is the default (for texts of 16 MiB and more) at stride 4
// up to this many 4-byte windows (two bits per key), else at stride 2 up to
// kPair2MaxKeys (three bits per key; measured ahead of the other maps up to
// 100,000 windows)
constexpr int32_t kPairMaxKeys = 12000;
constexpr int32_t kPair2MaxKeys = 131072;
// (queue entry, keyword id) pairs a wave's queue holds as its match stage,
// after its count and before the slot counter
constexpr int kWaveStageCap = (kQueueCap - 4) / 2;

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

__device__ __forceinline__ int64_t lmin(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t lmax(int64_t a, int64_t b) { return a > b ? a : b; }

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ unsigned rank_in(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi(unsigned(mask >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(mask), 0u));
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int lane) {
    unsigned lo = __builtin_amdgcn_readlane(unsigned(v), lane);
    unsigned hi = __builtin_amdgcn_readlane(unsigned(v >> 32), lane);
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// Third descriptor word of a raw (untyped, unswizzled) buffer on gfx9-family GPUs.
constexpr int kBufferFlags = 0x00020000;

// Loads through an explicit global-address-space pointer: pointers taken out
// of a by-value struct otherwise lower to flat loads, which also occupy the
// LDS counter and would serialise with the filter lookups.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 global_u32x4;
typedef const __attribute__((address_space(1))) uint32_t global_u32;

__device__ __forceinline__ u32x4 gload16(const uint8_t *p) { return *(global_u32x4 *)(p); }
__device__ __forceinline__ uint32_t gload4(const uint8_t *p) { return *(global_u32 *)(p); }
__device__ __forceinline__ uint32_t gload1(const uint8_t *p) {
    return *(const __attribute__((address_space(1))) uint8_t *)(p);
}
__device__ __forceinline__ void gstore16(uint4 *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    u32x4 v;
    v.x = a;
    v.y = b;
    v.z = c;
    v.w = d;
    *(__attribute__((address_space(1))) u32x4 *)(p) = v;
}

// Orders LDS traffic between lanes of one wave (queue producer -> consumer).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reports every keyword id of final state s at `off` (relative to its text).
// Called from divergent code: the lanes calling it together share one atomic
// per round; lanes with more ids loop more rounds.
__device__ __forceinline__ void emit(const DevAut &A, const ScanArgs &S, int64_t off, int32_t tid, int32_t s) {
    const int32_t k0 = A.out_off[s], k1 = A.out_off[s + 1];
    for (int32_t k = k0; k < k1; ++k) {
        const unsigned long long act = __ballot(1);
        const unsigned rank = rank_in(act);
        const int leader = __ffsll(static_cast<long long>(act)) - 1;
        unsigned long long base = 0;
        if (rank == 0) base = atomicAdd(S.count, static_cast<unsigned long long>(__popcll(act)));
        base = readlane64(base, leader);
        const unsigned long long idx = base + rank - S.count_base;
        if (idx < static_cast<unsigned long long>(S.cap)) {
            S.out_off[idx] = off;
            S.out_pid[idx] = A.out_pid[k];
            if (S.out_tid) S.out_tid[idx] = tid;
        }
        if (S.per_text) atomicAdd(reinterpret_cast<unsigned long long *>(S.per_text + tid), 1ull);
    }
}

// Block-level staging of matches in LDS: one global atomic per block instead
// of one per match.  Matches beyond the stage's capacity go straight out
// through emit().
constexpr int kStageCap = 3072;   // 48 KiB: fits, with the walk's bookkeeping, in the smallest filter's LDS
struct MatchStage {
    int64_t off[kStageCap];
    int32_t pid[kStageCap];
    int32_t tid[kStageCap];
    int32_t n;
    unsigned long long base;
};

__device__ __forceinline__ void emit_staged(const DevAut &A, const ScanArgs &S, MatchStage *st, int64_t off,
                                            int32_t tid, int32_t s) {
    const int32_t k0 = A.out_off[s], k1 = A.out_off[s + 1];
    for (int32_t k = k0; k < k1; ++k) {
        const int32_t i = atomicAdd(&st->n, 1);
        if (i < kStageCap) {
            st->off[i] = off;
            st->pid[i] = A.out_pid[k];
            st->tid[i] = tid;
            if (S.per_text) atomicAdd(reinterpret_cast<unsigned long long *>(S.per_text + tid), 1ull);
        } else {
            // stage full: this id goes out directly (one atomic)
            const unsigned long long idx = atomicAdd(S.count, 1ull) - S.count_base;
            if (idx < static_cast<unsigned long long>(S.cap)) {
                S.out_off[idx] = off;
                S.out_pid[idx] = A.out_pid[k];
                if (S.out_tid) S.out_tid[idx] = tid;
            }
            if (S.per_text) atomicAdd(reinterpret_cast<unsigned long long *>(S.per_text + tid), 1ull);
        }
    }
}

// One keyword id `pid` found at `off` (the caller knows it is the state's only one).
__device__ __forceinline__ void emit_one(const ScanArgs &S, MatchStage *st, int64_t off, int32_t tid, int32_t pid) {
    int32_t i = kStageCap;
    if (st) i = atomicAdd(&st->n, 1);
    if (i < kStageCap) {
        st->off[i] = off;
        st->pid[i] = pid;
        st->tid[i] = tid;
    } else {
        const unsigned long long idx = atomicAdd(S.count, 1ull) - S.count_base;
        if (idx < static_cast<unsigned long long>(S.cap)) {
            S.out_off[idx] = off;
            S.out_pid[idx] = pid;
            if (S.out_tid) S.out_tid[idx] = tid;
        }
    }
    if (S.per_text) atomicAdd(reinterpret_cast<unsigned long long *>(S.per_text + tid), 1ull);
}

// Called by every thread of the block once all its walks are done.
__device__ __forceinline__ void flush_stage(const ScanArgs &S, MatchStage *st) {
    __syncthreads();
    const int32_t n = imin(st->n, kStageCap);
    if (threadIdx.x == 0) st->base = n ? atomicAdd(S.count, static_cast<unsigned long long>(n)) - S.count_base : 0ull;
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long idx = st->base + unsigned(i);
        if (idx < static_cast<unsigned long long>(S.cap)) {
            S.out_off[idx] = st->off[i];
            S.out_pid[idx] = st->pid[i];
            if (S.out_tid) S.out_tid[idx] = st->tid[i];
        }
    }
}

// One Goto transition out of state s on byte b; returns next | final bit, or 0.
__device__ __forceinline__ int32_t step_global(const DevAut &A, const uint8_t *cls, int32_t s, uint32_t b) {
    if (s < A.S_dense) return A.dense[static_cast<int64_t>(s) * A.C + cls[b]];
    const int32_t r = s - A.S_dense;
    const int32_t fc = A.node[2 * r];
    int32_t lo = 0, hi = A.node[2 * r + 1] & 0x7fffffff;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (A.label[fc + mid] < b) lo = mid + 1;
        else hi = mid;
    }
    if (lo < (A.node[2 * r + 1] & 0x7fffffff) && A.label[fc + lo] == b) {
        const int32_t t = fc + lo;
        return t | (A.node[2 * (t - A.S_dense) + 1] & kFinalBit);
    }
    return 0;
}

// 24 x 24-bit product, low 32 bits, unsigned (__umul24 itself returns int,
// whose right shift would sign-extend).
__device__ __forceinline__ uint32_t hash24(uint32_t x, uint32_t mul) {
    return static_cast<uint32_t>(__umul24(x, mul));
}

// Exact prefix lookup for the K-byte prefix x: returns {key, value} of its
// slot -- key = x | next byte << 24, value = state at depth K | has-next bit
// 30 | final bit 31 -- or value 0 when no keyword starts with x.  The table
// holds buckets of four {key, value} slots and x lies in one of its two
// buckets, so both are read at once and no further probing is needed.
constexpr uint32_t kHasNext = 0x40000000u;
constexpr uint32_t kStateMask = 0x3fffffffu;

template <typename LoadBucket>
__device__ __forceinline__ uint2 prefix_state(LoadBucket load, int bits, uint32_t x, uint32_t mul) {
    const int nb = bits - 2;
    const uint32_t b1 = hash24(x, mul) >> (32 - nb);
    uint32_t b2 = hash24(x, kPrefixMul2) >> (32 - nb);
    if (b2 == b1) b2 = b1 ^ 1u;
    u32x4 q[4];
    load(b1, q[0], q[1]);
    load(b2, q[2], q[3]);
    // all four loads go out before the first compare: left alone, the
    // scheduler started comparing the first bucket first, so the second
    // bucket's loads waited for the first's (two round trips, not one)
    __builtin_amdgcn_sched_barrier(0);
    uint2 r = make_uint2(0u, 0u);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (q[i].y != 0u && (q[i].x & 0xFFFFFFu) == x) r = make_uint2(q[i].x, q[i].y);
        if (q[i].w != 0u && (q[i].z & 0xFFFFFFu) == x) r = make_uint2(q[i].z, q[i].w);
    }
    return r;
}

// Text of a candidate offset: [start, end) of the text holding o and its id.
// A batch's text starts come from `loff` when the block has copied them to
// LDS (as offsets from the first text, all below 2^32), else from global
// memory.
__device__ __forceinline__ void locate_text(const ScanArgs &S, const uint32_t *loff, int64_t o, int64_t &tstart,
                                            int64_t &end, int32_t &tid) {
    tstart = 0;
    end = S.n;
    tid = 0;
    if (!S.text_off) return;
    int32_t lo = 0, hi = S.n_texts;   // largest t with start(t) <= o, in [lo, hi)
    if (loff) {
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (int64_t(loff[mid]) <= o) lo = mid;
            else hi = mid;
        }
        tstart = loff[lo];
        end = lmin(int64_t(loff[lo + 1]), S.n);
    } else {
        const int64_t base0 = S.text_off[0];
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (S.text_off[mid] - base0 <= o) lo = mid;
            else hi = mid;
        }
        tstart = S.text_off[lo] - base0;
        end = lmin(S.text_off[lo + 1] - base0, S.n);
    }
    tid = lo;
}

// 16 bytes from p, of any alignment, assembled from five aligned dword loads.
// Every dword address is clamped to at most `last` (the aligned dword holding
// the last readable byte), so no load leaves the buffer; bytes taken from a
// clamped dword are garbage and must be masked by the caller.
__device__ __forceinline__ u32x4 load16_clamped(const uint8_t *p, uintptr_t last) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p) & ~uintptr_t(3);
    const uint32_t sh = uint32_t(reinterpret_cast<uintptr_t>(p) & 3u);
    uint32_t w[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const uintptr_t ai = a + 4u * uintptr_t(i);
        w[i] = gload4(reinterpret_cast<const uint8_t *>(ai < last ? ai : last));
    }
    u32x4 r;
    r.x = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
    r.y = __builtin_amdgcn_alignbyte(w[2], w[1], sh);
    r.z = __builtin_amdgcn_alignbyte(w[3], w[2], sh);
    r.w = __builtin_amdgcn_alignbyte(w[4], w[3], sh);
    return r;
}

// 16 bytes from p, of any alignment, in one load: global memory is accessed
// in the GPU's unaligned access mode, which ROCm enables.  [p, p + 16) must
// be readable.
__device__ __forceinline__ u32x4 load16_any(const uint8_t *p) {
    u32x4 r;
    __builtin_memcpy(&r, (const __attribute__((address_space(1))) uint8_t *)(p), 16);
    return r;
}

// XOR of the first n (0..16) bytes of a and b, 0 when they agree.
__device__ __forceinline__ uint32_t diff16(u32x4 a, u32x4 b, int n) {
    uint32_t d = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = n - 4 * i;    // bytes of word i that count
        const uint32_t keep = m >= 4 ? 0xFFFFFFFFu : (m <= 0 ? 0u : (1u << (8 * m)) - 1u);
        d |= (a[i] ^ b[i]) & keep;
    }
    return d;
}

// Whether text t[0 .. n) equals keyword bytes k[0 .. n) (n <= 64; text[0 ..
// text_n) is the scanned buffer, which holds t[0 .. n)).  The first 32 bytes
// of both are loaded in one round trip, as 16-byte loads of any alignment;
// longer tails take more.  Text bytes within 16 of the buffer's end come
// from clamped dword loads instead.  Keyword bytes may be read up to 79
// bytes past a keyword: the keyword section is followed by at least 256
// bytes of the same allocation.
__device__ __forceinline__ bool equal_bytes(const uint8_t *t, const uint8_t *k, int n, const uint8_t *text,
                                            int64_t text_n) {
    const uintptr_t tend = reinterpret_cast<uintptr_t>(text) + uintptr_t(text_n);
    const uintptr_t tlast = (tend - 1u) & ~uintptr_t(3);
    auto text16 = [&](const uint8_t *p) __attribute__((always_inline)) {
        return reinterpret_cast<uintptr_t>(p) + 16u <= tend ? load16_any(p) : load16_clamped(p, tlast);
    };
    const u32x4 t0 = text16(t), t1 = text16(t + 16);
    const u32x4 k0 = load16_any(k), k1 = load16_any(k + 16);
    uint32_t d = diff16(t0, k0, n) | diff16(t1, k1, n - 16);
    for (int i = 32; d == 0 && i < n; i += 16) d = diff16(text16(t + i), load16_any(k + i), n - i);
    return d == 0;
}

// Position of byte b among the first n (1 .. 16) bytes of v, which are
// distinct, or -1.  Per word, the lowest flag of the zero-byte test marks the
// first byte equal to b exactly (a false flag can only sit above a true one).
__device__ __forceinline__ int find_byte16(u32x4 v, int n, uint32_t b) {
    const uint32_t rep = b * 0x01010101u;
    int at = 16;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        const uint32_t x = v[i] ^ rep;
        const uint32_t z = (x - 0x01010101u) & ~x & 0x80808080u;
        if (z) at = 4 * i + int(__builtin_ctz(z) >> 3);
    }
    return at < n ? at : -1;
}

// The rest of the walk from offset o (relative to the scanned buffer) once
// the exact prefix table gave e = {state at depth K | final bit}.  Each step
// reads the state's 16-byte walk record (tail info): whether a keyword ends
// there, and either a forced path (a unary chain to a leaf with no keyword
// ending in between, whose leaf keyword is then compared with the text
// directly), a unary chain to a deeper state that ends a keyword or
// branches (compared the same way, then the walk goes on from there), or
// the state's children.  A dense state's next state comes from its
// transition row, with the byte's class loaded beside the record; a compact
// state's children are consecutive states with sorted edge labels, found
// among up to 16 labels read in one load.  The walk never compares or steps
// past `end` (the end of o's text).  With REC, rb holds the 8 text bytes
// that follow the prefix (as captured by the streaming kernel), which pick
// the first transitions without waiting for a load; the 32 bytes after the
// prefix are loaded at the start, beside the first record, and serve the
// first compare and the next transitions.  Every keyword starting at o is
// reported, through ids(state) for all keyword ids of a final state or
// one(pid) for a single id.
template <bool REC, typename Ids, typename One>
__device__ __forceinline__ void walk_rest(const DevAut &A, const ScanArgs &S, int64_t o, int64_t end, uint32_t e,
                                          uint2 rb, Ids &&ids, One &&one) {
    const int K = A.K;
    if (o + K > end) return;          // the prefix ran into the next text of a batch
    // The 32 text bytes after the prefix, loaded beside the first walk
    // record: most walks compare them with a forced path's keyword and read
    // no other text.
    const uintptr_t tend = reinterpret_cast<uintptr_t>(S.text) + uintptr_t(S.n);
    const uintptr_t tlast = (tend - 1u) & ~uintptr_t(3);
    auto text16 = [&](int64_t j) __attribute__((always_inline)) {   // 16 bytes from text byte j < S.n
        const uint8_t *p = S.text + j;
        return reinterpret_cast<uintptr_t>(p) + 16u <= tend ? load16_any(p) : load16_clamped(p, tlast);
    };
    u32x4 t0 = {0u, 0u, 0u, 0u}, t1 = t0;
    if (o + K < end) {
        t0 = text16(o + K);
        if (o + K + 16 < S.n) t1 = text16(o + K + 16);
    }
    auto byte_at = [&](int64_t j) -> uint32_t {   // text byte j (o + K <= j < end)
        const int64_t r = j - o - K;
        if (REC && r < 8) return r < 4 ? (rb.x >> (8 * r)) & 0xFFu : (rb.y >> (8 * (r - 4))) & 0xFFu;
        if (r < 32) {
            const u32x4 t = r < 16 ? t0 : t1;
            const int q = int(r & 15);
            const uint32_t w = q < 4 ? t.x : q < 8 ? t.y : q < 12 ? t.z : t.w;
            return (w >> (8 * (q & 3))) & 0xFFu;
        }
        return gload1(S.text + j);
    };
    // whether text bytes o + dd .. o + dd + z equal keyword bytes kw[0 .. z):
    // from the preloaded bytes while the walk is still at the prefix
    auto same = [&](int64_t dd, const uint8_t *kw, int32_t z) -> bool {
        if (dd == K && z <= 32) {
            const u32x4 k0 = load16_any(kw), k1 = load16_any(kw + 16);
            return (diff16(t0, k0, z) | diff16(t1, k1, z - 16)) == 0u;
        }
        return equal_bytes(S.text + o + dd, kw, z, S.text, S.n);
    };
    int32_t s = int32_t(e & kStateMask);
    int64_t d = K;
    while (true) {
        const int4 ti = A.tailinfo[s];
        const bool has_byte = o + d < end;
        const uint32_t b = has_byte ? byte_at(o + d) : 0u;
        const bool dense = s < A.S_dense;
        const uint32_t c = dense && has_byte ? uint32_t(A.cls[b]) : 0u;
        if (ti.w < 0) ids(s);          // a keyword ends at s
        if (ti.x >= 0) {
            // forced path: bytes d .. d + ti.z of the text against the keyword
            const int64_t L = d + ti.z;
            if (o + L > end) return;
            if (!same(d, A.kw_bytes + ti.y, ti.z)) return;
            const int32_t only = ti.w & 0x7fffffff;
            if (only > 0) one(only - 1);
            else ids(ti.x);
            return;
        }
        if (ti.x == -3) {
            // a unary chain of ti.z bytes (no keyword ends inside it) to
            // state ti.w: compared in one pass, like a forced path
            if (o + d + ti.z > end) return;
            if (!same(d, A.kw_bytes + ti.y, ti.z)) return;
            s = ti.w & 0x7fffffff;
            d += ti.z;
            continue;
        }
        if (ti.x == -2 || !has_byte) return;   // a leaf, or the text ends
        if (dense) {
            const int32_t e2 = A.dense[static_cast<int64_t>(s) * A.C + c];
            if (e2 == 0) return;
            s = e2 & 0x7fffffff;
        } else {
            const int32_t fc = ti.y, nc = ti.z;
            int i;
            if (nc <= 16) {
                i = find_byte16(load16_any(A.label + fc), nc, b);
            } else {
                int32_t lo = 0, hi = nc;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (A.label[fc + mid] < b) lo = mid + 1;
                    else hi = mid;
                }
                i = lo < nc && A.label[fc + lo] == b ? lo : -1;
            }
            if (i < 0) return;
            s = fc + i;
        }
        ++d;
    }
}

struct FilterLaunch {
    const uint8_t *base;     // text pointer rounded down to 16 bytes
    int64_t mis;             // text - base
    int64_t V;               // mis + n: end of the text in `base` coordinates
    int64_t n_chunks;        // ceil(V / chunk bytes)
    int64_t c_lo, c_hi;      // interior chunks [c_lo, c_hi): whole chunk + 16 B inside the text
    const uint8_t *filter;   // the filter map this launch stages in LDS
    int32_t hit_cap;         // entries per wave region
    uint4 *hits;             // [waves * hit_cap]: {slot << 12 | position, prefix-table value,
                             //  the 8 text bytes after the prefix}
};

// The filtered kernel's one argument.
struct KArgs {
    DevAut A;
    ScanArgs S;
    FilterLaunch F;
};
typedef const __attribute__((address_space(4))) KArgs *KArgsPtr;

// Slot -> interior chunk of one block (see filtered_kernel).
struct SlotMap {
    int64_t bfirst;    // the block's first chunk
    int64_t nw;        // waves in the grid
    uint32_t wmask;    // waves per block - 1 (a power of two minus one)
    int32_t wlog;      // log2(waves per block)
    __device__ __forceinline__ int64_t chunk(uint32_t slot) const {
        return bfirst + int64_t(slot & wmask) + int64_t(slot >> wlog) * nw;
    }
};

template <int SEGS>
struct ChunkRegs {
    uint32_t d[SEGS][4];
    uint32_t tail;   // first dword after the chunk (halo of the last lane)
};

// Interior chunk: one coalesced 16-byte load per lane and segment, as buffer
// loads from a descriptor based at the chunk (uniform, in SGPRs) with
// per-lane offsets that never change, so issuing the next chunk's loads
// needs no address register that an earlier load might still be writing.
// The loads are non-temporal: the stream passes through the caches without
// pushing out the tables and records that drains and walks read (1 GiB,
// 1000 keywords: 0.178 ms instead of 0.191; the 4096-text batch, whose
// block-wide walk follows the stream closely, 1% slower; a uniform branch
// that kept the default policy for batches cost more than either).
template <int SEGS>
__device__ __forceinline__ void load_interior(const FilterLaunch &F, int64_t c, unsigned lane, ChunkRegs<SEGS> &R) {
    constexpr int64_t CH = int64_t(SEGS) * kSegBytes;
    constexpr int kNonTemporal = 2;     // cache-policy operand of the buffer loads: nt
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(F.base + c * CH), short(0), int(CH + 16), kBufferFlags);
#pragma unroll
    for (int j = 0; j < SEGS; ++j) {
        const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(rsrc, int(lane * 16u + uint32_t(j) * kSegBytes), 0,
                                                              kNonTemporal);
        R.d[j][0] = q.x; R.d[j][1] = q.y; R.d[j][2] = q.z; R.d[j][3] = q.w;
    }
    R.tail = __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(CH), 0, 0);
}

// Chunk that overlaps either end of the text: bytes outside it read as 0.
template <int SEGS>
__device__ __forceinline__ void load_partial(const FilterLaunch &F, int64_t c, unsigned lane, ChunkRegs<SEGS> &R) {
    constexpr int64_t CH = int64_t(SEGS) * kSegBytes;
    auto get4 = [&](int64_t p) {
        uint32_t v = 0;
        for (int b = 0; b < 4; ++b)
            if (p + b >= F.mis && p + b < F.V) v |= uint32_t(F.base[p + b]) << (8 * b);
        return v;
    };
#pragma unroll
    for (int j = 0; j < SEGS; ++j)
#pragma unroll
        for (int w = 0; w < 4; ++w) R.d[j][w] = get4(c * CH + j * kSegBytes + lane * 16 + w * 4);
    R.tail = get4((c + 1) * CH);
}

// Candidate mask of one chunk: bit 16 j + s is set when offset s of the
// lane's 16 bytes in segment j may start a keyword.
//
// Stride 1: the K bytes at offset s hash to a set filter entry.
// Stride 2 and 4: only the 3-byte windows starting at s = STRIDE, 2 STRIDE,
// ..., 16 are tested (s = 16 is the next lane's first bytes), against the
// keywords' windows at positions 1 .. STRIDE; a keyword starting at o has its
// window at position s - o tested for the one sampled s in o + 1 .. o +
// STRIDE, so a positive makes the STRIDE offsets s - STRIDE .. s - 1
// candidates.  Windows at s = 4, 8, 12, 16 are whole registers (the hash
// reads 24 bits), so stride 4 extracts no bytes and stride 2 half as many.
// A bit map is tested without shifting the looked-up bit into place: the
// hash is p = x * mul + c with c = -b mod 32 for destination bit b, so
// rotating the word right by p (mod 32) moves the key's bit (x * mul) mod 32
// to b.  Adding c may carry into the word index; the host sets each key's
// bit in both words that can result.
// PAIR (strides 2 and 4): the window at s is four bytes (the whole register
// d[s / 4] when s is a multiple of 4), tested against the keywords' 4-byte
// windows at positions 1 .. STRIDE: its first three bytes pick the word, and
// the bits (x * mul) mod 32 and (byte 3) mod 32 of that word must both be set;
// at stride 2 also bit (byte 2) mod 32, read from the next sampled window
// (whose low bits are byte 2) at no extra extraction.
template <int K, bool BITMAP, int SEGS, int FLOG2, int STRIDE, bool DUAL, bool PAIR>
__device__ __forceinline__ unsigned long long filter_chunk(const ChunkRegs<SEGS> &R, unsigned lane,
                                                           const uint8_t *sfilt, uint32_t mul) {
    constexpr uint32_t kmask = K >= 3 ? 0xFFFFFFu : ((1u << (8 * K)) - 1u);
    // byte map: 2^FLOG2 entries; bit map: 2^(FLOG2-2) words of 32 bits
    constexpr int shift = BITMAP ? 32 - (FLOG2 - 2) : 32 - FLOG2;
    const uint32_t *fm = reinterpret_cast<const uint32_t *>(sfilt);
    uint32_t mseg[SEGS];
#pragma unroll
    for (int j = 0; j < SEGS; ++j) {
        uint32_t d[5];
        d[0] = R.d[j][0]; d[1] = R.d[j][1]; d[2] = R.d[j][2]; d[3] = R.d[j][3];
        const uint32_t from_next_lane = __builtin_amdgcn_ds_bpermute(int((lane + 1) * 4), int(d[0]));
        const uint32_t from_next_seg = (j + 1 < SEGS) ? __builtin_amdgcn_readlane(R.d[(j + 1) % SEGS][0], 0)
                                                      : R.tail;
        d[4] = lane == 63 ? from_next_seg : from_next_lane;
        uint32_t mj = 0;
        if (STRIDE == 1) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int w = s >> 2, r = s & 3;
                uint32_t x = r == 0 ? d[w] : __builtin_amdgcn_alignbyte(d[w + 1], d[w], uint32_t(r));
                if (K < 3) x &= kmask;
                const uint32_t p = hash24(x, mul);
                uint32_t v;
                if (DUAL) {
                    const uint32_t p2 = hash24(x, kFilterMul2);
                    v = __builtin_amdgcn_ubfe(fm[p >> (shift + 1)], p, 1u) &
                        __builtin_amdgcn_ubfe(fm[(1u << (FLOG2 - 3)) + (p2 >> (shift + 1))], p2, 1u);
                } else if (BITMAP) {
                    v = __builtin_amdgcn_ubfe(fm[p >> shift], p, 1u);
                } else {
                    v = sfilt[p >> shift];
                }
                mj |= v << s;
            }
        } else {
#pragma unroll
            for (int s = STRIDE; s <= 16; s += STRIDE) {
                const int w = s >> 2, r = s & 3;
                const uint32_t x = r == 0 ? d[w] : __builtin_amdgcn_alignbyte(d[w + 1], d[w], uint32_t(r));
                const int b = s - STRIDE;                 // destination bit
                const uint32_t c = uint32_t(32 - b) & 31u;
                const uint32_t p = hash24(x, mul) + c;
                if (PAIR) {
                    const uint32_t p0 = hash24(x, mul);
                    const uint32_t w1 = fm[p0 >> shift];
                    uint32_t v = __builtin_amdgcn_alignbit(w1, w1, p0) & __builtin_amdgcn_alignbit(w1, w1, x >> 24);
                    if (STRIDE == 2) {
                        // third bit: (byte 2) mod 32, the low bits of the next sampled window
                        const int s2 = s + 2, w2 = s2 >> 2;
                        const uint32_t x2 = s2 > 16 ? d[4] >> 16
                                          : (s2 & 3) ? __builtin_amdgcn_alignbyte(d[w2 + 1], d[w2], 2u) : d[w2];
                        v &= __builtin_amdgcn_alignbit(w1, w1, x2);
                    }
                    mj |= (v & 1u) << b;
                } else if (BITMAP) {
                    uint32_t v;
                    if (DUAL) {
                        // two maps of 2^(FLOG2 - 3) words, independent hashes: both bits must be set
                        const uint32_t p2 = hash24(x, kFilterMul2) + c;
                        const uint32_t w1 = fm[p >> (shift + 1)];
                        const uint32_t w2 = fm[(1u << (FLOG2 - 3)) + (p2 >> (shift + 1))];
                        v = __builtin_amdgcn_alignbit(w1, w1, p) & __builtin_amdgcn_alignbit(w2, w2, p2);
                    } else {
                        const uint32_t w1 = fm[p >> shift];
                        v = __builtin_amdgcn_alignbit(w1, w1, p);
                    }
                    mj = (v & (1u << b)) | (mj & ~(1u << b));
                } else {
                    mj |= uint32_t(sfilt[p >> shift]) << b;
                }
            }
            // a positive at bit b covers the offsets b .. b + STRIDE - 1
            if (STRIDE == 2) mj |= mj << 1;
            if (STRIDE == 4) mj = __umul24(mj, 15u);
        }
        mseg[j] = mj;
    }
    // bit 16 j + s: segment j, byte s
    const uint32_t lo = SEGS >= 2 ? (mseg[0] | (mseg[1 % SEGS] << 16)) : mseg[0];
    const uint32_t hi = SEGS >= 4 ? (mseg[2 % SEGS] | (mseg[3 % SEGS] << 16)) : 0u;
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// A condition every lane of the wave agrees on, marked as such for the
// compiler, so that branching on it needs no exec-mask bookkeeping.  The
// ballot keeps the lane mask in scalar registers (a readfirstlane would first
// write it to a VGPR, whose reuse could wait for a load still in flight).
__device__ __forceinline__ bool uniform(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }
// A value every lane holds, moved to scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// The kernel's argument block, read where it lies.  The empty asm hides the
// pointer's origin from the compiler, so the fields read through it are
// loaded here and not all at the kernel's entry, from where they would stay
// live (and spill) across the streaming loop.
__device__ __forceinline__ const KArgs *kernel_args() {
    KArgsPtr p = (KArgsPtr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return (const KArgs *)p;   // still known to be constant memory: read with scalar loads
}

// Exact prefix lookup through the LDS copy of the prefix table when it has
// one, else through global memory.
__device__ __forceinline__ uint2 probe_prefix(bool in_lds, const uint32_t *sptab, const uint32_t *gptab, int bits,
                                              uint32_t x, uint32_t mul) {
    if (in_lds)
        return prefix_state([&](uint32_t b, u32x4 &lo, u32x4 &hi) {
            lo = reinterpret_cast<const u32x4 *>(sptab)[2 * b];
            hi = reinterpret_cast<const u32x4 *>(sptab)[2 * b + 1];
        }, bits, x, mul);
    return prefix_state([&](uint32_t b, u32x4 &lo, u32x4 &hi) {
        lo = gload16(reinterpret_cast<const uint8_t *>(gptab + 8 * b));
        hi = gload16(reinterpret_cast<const uint8_t *>(gptab + 8 * b + 4));
    }, bits, x, mul);
}

// Streaming kernel of the filtered policy.
//
// Work is dealt out in slots: slot i of block b is interior chunk c_lo + b W
// + (i mod W) + (i div W) nw (W waves per block, nw waves in the grid, so a
// step of the grid still reads one contiguous stretch of text).  Each wave
// starts with slots `wave` and `wave + W` and takes every further slot from
// a counter in LDS, one slot ahead of need.  Waves of one block progress at
// very different rates (the SIMDs favour older waves), and with a fixed
// share per wave the block would wait for its slowest one.
//
// Candidate offsets wait in a per-wave LDS queue; a drain takes kDrain of
// them at once (each lane loads the prefix window of kDrain / 64 candidates
// with independent loads, then looks the prefix up in the exact prefix table)
// and appends the surviving prefixes, with the 8 text bytes after them, to
// the wave's hit region with plain stores.  The chunk loop has no walk,
// atomic in global memory, call or other dependent global access.  A wave
// whose region has no room for another drain leaves the loop and goes on in
// a slow mode: it scans the rest of its slots one chunk at a time and walks
// every hit as soon as the prefix table confirms it.  So does every wave with
// the partial chunks at the text's ends.  Finally each wave (one text) or the
// whole block (a batch) walks the stored hits.
template <int K, bool BITMAP, int SEGS, int FLOG2, int STRIDE, bool DUAL, bool PAIR>
__global__ __launch_bounds__(1024) void filtered_kernel(const KArgs) {
    __shared__ __align__(16) uint8_t sfilt[1 << FLOG2];
    __shared__ __align__(16) uint32_t squeue[kMaxWaves * kQueueCap];
    // Beside a 64 KiB filter, a copy of the prefix table (8192 slots) fits
    // too; beside a 128 KiB one only the queues and the hit records do.
    constexpr int PT_SLOTS = FLOG2 >= 17 ? 0 : 8192;
    constexpr int kHitBytes = kMaxWaves * kLdsHits * 16;
    __shared__ __align__(16) uint32_t sxtra[(2 * PT_SLOTS * 4 + kHitBytes) / 4];
    uint32_t *const sptab = sxtra;                                        // [2 * PT_SLOTS]
    uint4 *const shits = reinterpret_cast<uint4 *>(sxtra + 2 * PT_SLOTS);  // [waves * kLdsHits]
    constexpr int64_t CH = int64_t(SEGS) * kSegBytes;
    constexpr int PER_LANE = kDrain / kWave;
    const int waves_per_block = int(blockDim.x) / kWave;
    const int wlog = __builtin_ctz(unsigned(waves_per_block));   // W is a power of two
    const unsigned lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    uint32_t *q = squeue + wave * kQueueCap;
    const int64_t w = int64_t(blockIdx.x) * waves_per_block + wave;
    const int64_t nw = int64_t(gridDim.x) * waves_per_block;
    uint32_t &snext = squeue[kQueueCap - 1];              // next slot to hand out
    int hcount = 0;                    // hits stored in this wave's region
    int qlen = 0;

    // Queues the candidate offsets of mask m (chunk slot k), draining the
    // queue whenever it holds kDrain entries.  Returns false, leaving the
    // bits not yet queued in m, if `drain` refuses to run.
    auto push = [&](unsigned long long &m, uint32_t k, auto &&drain) __attribute__((always_inline)) {
        while (true) {
            if (qlen >= kDrain && !drain(kDrain)) return false;
            const unsigned long long act = __ballot(m != 0);
            if (act == 0) return true;
            if (m) {
                const int b = __ffsll(static_cast<long long>(m)) - 1;
                q[qlen + int(rank_in(act))] = (k << 12) | uint32_t((b >> 4) * kSegBytes + int(lane) * 16 + (b & 15));
                m &= m - 1;
            }
            qlen += __popcll(act);
        }
    };
    // The newest `take` queue entries, one per lane (lanes past `take`
    // repeat the first one, so every load made from them is valid).
    auto pop = [&](int take, uint32_t (&ent)[PER_LANE]) __attribute__((always_inline)) {
        wave_sync();
#pragma unroll
        for (int r = 0; r < PER_LANE; ++r) {
            const int i = int(lane) + r * kWave;
            ent[r] = q[qlen - take + (i < take ? i : 0)];
        }
        wave_sync();
        qlen -= take;
    };

    // Where the streaming loop stopped: every slot from `cur` on is left to
    // the slow mode (none if cur_ok is false), cur's candidates not yet
    // queued in `rest`, and lane 0's `ahead` holding the slot after nxt
    // (taken when nxt is a chunk of the text).
    bool slow = false;
    bool cur_ok = false;
    uint32_t cur = 0, nxt = 0, ahead = 0;
    unsigned long long rest = 0;

    // ---- set-up and streaming: the fields they read, and no others ----
    {
        const KArgs *P1 = kernel_args();
        const FilterLaunch F = P1->F;
        const uint8_t *text = P1->S.text;
        const uint32_t *gptab = P1->A.ptab;
        const int ptab_bits = P1->A.ptab_bits;
        const uint32_t mul = P1->A.hash_mul;
        const bool pt_lds = FLOG2 < 17 && ptab_bits <= 13;
        // Tables to LDS, two loads in flight per thread.  Every block reads
        // the same lines, so the blocks of one XCD (blockIdx mod 8) start at
        // different ones (n16 is a power of two).
        auto stage = [&](const uint4 *src, uint4 *dst, int n16) __attribute__((always_inline)) {
            const int rot = (int(blockIdx.x >> 3) * 1024) & (n16 - 1);
            for (int i0 = int(threadIdx.x); i0 < n16; i0 += 2 * int(blockDim.x)) {
                const int i1 = i0 + int(blockDim.x);
                const uint4 v0 = src[(i0 + rot) & (n16 - 1)];
                uint4 v1;
                if (i1 < n16) v1 = src[(i1 + rot) & (n16 - 1)];
                dst[(i0 + rot) & (n16 - 1)] = v0;
                if (i1 < n16) dst[(i1 + rot) & (n16 - 1)] = v1;
            }
        };
        stage(reinterpret_cast<const uint4 *>(F.filter), reinterpret_cast<uint4 *>(sfilt), (1 << FLOG2) / 16);
        if (pt_lds) stage(reinterpret_cast<const uint4 *>(gptab), reinterpret_cast<uint4 *>(sptab), (2 << ptab_bits) / 4);
        SlotMap M;
        M.bfirst = F.c_lo + int64_t(blockIdx.x) * waves_per_block;
        M.nw = nw;
        M.wmask = uint32_t(waves_per_block - 1);
        M.wlog = wlog;
        if (threadIdx.x == 0) snext = uint32_t(2 * waves_per_block);
        __syncthreads();

        uint4 *hits = F.hits + w * F.hit_cap;
        uint4 *lhits = shits + wave * kLdsHits;
        // Streaming-loop drain of the newest `take` entries (interior chunks
        // only: there o + 16 <= n, so the aligned 16 bytes from (o & ~3) lie
        // in the text and give the prefix and the 8 bytes after it).  Refuses
        // when the region might not hold its hits.
        auto drain_store = [&](int take) __attribute__((always_inline)) {
            if (hcount + kDrain > kLdsHits + F.hit_cap) return false;
            uint32_t ent[PER_LANE];
            pop(take, ent);
            u32x4 win[PER_LANE];
            uint32_t sh[PER_LANE];
#pragma unroll
            for (int r = 0; r < PER_LANE; ++r) {
                const int64_t o = M.chunk(ent[r] >> 12) * CH + int64_t(ent[r] & 4095u) - F.mis;
                const uintptr_t a = reinterpret_cast<uintptr_t>(text + o);
                sh[r] = uint32_t(a & 3u);
                const uint8_t *pa = reinterpret_cast<const uint8_t *>(a & ~uintptr_t(3));
                win[r].x = gload4(pa);
                win[r].y = gload4(pa + 4);
                win[r].z = gload4(pa + 8);
                win[r].w = gload4(pa + 12);
            }
#pragma unroll
            for (int r = 0; r < PER_LANE; ++r) {
                const uint32_t y0 = __builtin_amdgcn_alignbyte(win[r].y, win[r].x, sh[r]);
                const uint32_t y1 = __builtin_amdgcn_alignbyte(win[r].z, win[r].y, sh[r]);
                const uint32_t y2 = __builtin_amdgcn_alignbyte(win[r].w, win[r].z, sh[r]);
                const uint32_t x = K >= 3 ? (y0 & 0xFFFFFFu) : (y0 & ((1u << (8 * K)) - 1u));
                const uint32_t rb0 = __builtin_amdgcn_alignbyte(y1, y0, uint32_t(K));
                const uint32_t rb1 = __builtin_amdgcn_alignbyte(y2, y1, uint32_t(K));
                uint32_t e = 0;
                if (int(lane) + r * kWave < take) {
                    const uint2 kv = probe_prefix(pt_lds, sptab, gptab, ptab_bits, x, mul);
                    e = kv.y;
                    // a non-final prefix state whose only child's byte differs
                    // from the text's next byte ends the walk at the prefix
                    if ((e & kHasNext) && !(e >> 31) && (kv.x >> 24) != (rb0 & 0xFFu)) e = 0u;
                }
                const unsigned long long hit = __ballot(e != 0u);
                if (hit == 0) continue;
                if (e != 0u) {
                    const int at = hcount + int(rank_in(hit));
                    if (at < kLdsHits) lhits[at] = make_uint4(ent[r], e, rb0, rb1);
                    else gstore16(hits + (at - kLdsHits), ent[r], e, rb0, rb1);
                }
                hcount += __popcll(hit);
            }
            return true;
        };

        // Interior chunks, two register sets in turn so that the next chunk's
        // loads are in flight while this one is filtered.  The next chunk's
        // loads are issued unconditionally (the last step reloads its own
        // chunk): with a fixed number of loads between a chunk's loads and
        // its first use, the compiler waits for that chunk only.
        ChunkRegs<SEGS> ra, rb;
        const int64_t c_hi = uniform64(F.c_hi);
        cur = uint32_t(wave);
        nxt = uint32_t(wave + waves_per_block);
        cur_ok = uniform(M.chunk(cur) < c_hi);
        if (cur_ok) load_interior<SEGS>(F, M.chunk(cur), lane, ra);
        // One half step: issue the next chunk's loads into `into` (or reload
        // the current one), take the slot after nxt from the block's counter
        // (lane 0), filter and queue the current chunk held in `regs`, then
        // move on.  The counter's divergent branch joins right after the
        // atomic, so the loop's back edge merges only uniform conditions.
        // Returns false when the loop must end (slow mode, or no slot left).
        auto half = [&](ChunkRegs<SEGS> &regs, ChunkRegs<SEGS> &into) __attribute__((always_inline)) {
            const bool nxt_ok = uniform(M.chunk(nxt) < c_hi);
            load_interior<SEGS>(F, M.chunk(nxt_ok ? nxt : cur), lane, into);
            if (lane == 0 && nxt_ok) ahead = atomicAdd(&snext, 1u);
            rest = filter_chunk<K, BITMAP, SEGS, FLOG2, STRIDE, DUAL, PAIR>(regs, lane, sfilt, mul);
            if (!uniform(push(rest, cur, drain_store))) { slow = true; return false; }
            // slots held by a wave only grow, and so do their chunks: once
            // one is past the end, so is every later one
            cur = nxt;
            cur_ok = nxt_ok;
            nxt = __builtin_amdgcn_readfirstlane(ahead);
            return cur_ok;
        };
        while (cur_ok) {
            if (!half(ra, rb)) break;
            if (!half(rb, ra)) break;
        }
        while (!slow && qlen > 0)
            if (!drain_store(imin(qlen, kDrain))) slow = true;
    }

    // ---- slow mode, partial chunks, walks and output ----
    const KArgs *P2 = kernel_args();
    const DevAut A = P2->A;
    const ScanArgs S = P2->S;
    const FilterLaunch F = P2->F;
    SlotMap M;
    M.bfirst = F.c_lo + int64_t(blockIdx.x) * waves_per_block;
    M.nw = nw;
    M.wmask = uint32_t(waves_per_block - 1);
    M.wlog = wlog;
    const bool pt_lds = FLOG2 < 17 && A.ptab_bits <= 13;
    const uint32_t mul = A.hash_mul;
    uint4 *hits = F.hits + w * F.hit_cap;
    auto offset_of = [&](uint32_t ent) __attribute__((always_inline)) {
        return M.chunk(ent >> 12) * CH + int64_t(ent & 4095u) - F.mis;
    };

    {
        int64_t pchunk = -1;         // a partial chunk's number, else -1 (entries hold slots)
        // Drain that probes with byte loads and walks the hits right here.
        auto drain_walk = [&](int take) __attribute__((always_inline)) {
            uint32_t ent[PER_LANE];
            pop(take, ent);
            for (int r = 0; r < PER_LANE; ++r) {
                if (int(lane) + r * kWave >= take) continue;
                const int64_t o = (pchunk >= 0 ? pchunk : M.chunk(ent[r] >> 12)) * CH + int64_t(ent[r] & 4095u) - F.mis;
                uint32_t x = 0;
                for (int j = 0; j < K; ++j) x |= gload1(S.text + o + j) << (8 * j);
                const uint2 kv = probe_prefix(pt_lds, sptab, A.ptab, A.ptab_bits, x, mul);
                if (kv.y == 0u) continue;
                int64_t tstart, end;
                int32_t tid;
                locate_text(S, nullptr, o, tstart, end, tid);
                walk_rest<false>(A, S, o, end, kv.y, make_uint2(0u, 0u),
                                 [&](int32_t st) { emit(A, S, o - tstart, tid, st); },
                                 [&](int32_t pid) { emit_one(S, nullptr, o - tstart, tid, pid); });
            }
            return true;
        };
        if (slow) {
            // the rest of cur's candidates, then cur's successors, one chunk
            // at a time
            (void)push(rest, cur, drain_walk);
            uint32_t sl = nxt;
            uint32_t after = __builtin_amdgcn_readfirstlane(ahead);
            bool ok = cur_ok && M.chunk(sl) < F.c_hi;
            while (ok) {
                ChunkRegs<SEGS> r;
                load_interior<SEGS>(F, M.chunk(sl), lane, r);
                unsigned long long m = filter_chunk<K, BITMAP, SEGS, FLOG2, STRIDE, DUAL, PAIR>(r, lane, sfilt, mul);
                (void)push(m, sl, drain_walk);
                sl = after;
                ok = M.chunk(sl) < F.c_hi;
                if (ok) {
                    uint32_t t = 0;
                    if (lane == 0) t = atomicAdd(&snext, 1u);
                    after = __builtin_amdgcn_readfirstlane(t);
                }
            }
            while (qlen > 0) drain_walk(imin(qlen, kDrain));
        }
        // chunks overlapping an end of the text, [0, p0) and [p1, n_chunks),
        // filtered with byte loads
        const int64_t p0 = lmin(F.c_lo, F.n_chunks);
        const int64_t p1 = lmax(F.c_hi, F.c_lo);
        const int64_t n_partial = p0 + (F.n_chunks - p1);
        for (int64_t i = w; i < n_partial; i += nw) {
            pchunk = i < p0 ? i : p1 + (i - p0);
            ChunkRegs<SEGS> r;
            load_partial<SEGS>(F, pchunk, lane, r);
            unsigned long long m = filter_chunk<K, BITMAP, SEGS, FLOG2, STRIDE, DUAL, PAIR>(r, lane, sfilt, mul);
            for (int b = 0; b < SEGS * 16; ++b) {
                // keep offsets o with 0 <= o and o + K <= n
                const int64_t o = pchunk * CH + (b >> 4) * kSegBytes + int64_t(lane) * 16 + (b & 15) - F.mis;
                if (o < 0 || o + K > S.n) m &= ~(1ull << b);
            }
            (void)push(m, 0, drain_walk);
            while (qlen > 0) drain_walk(imin(qlen, kDrain));
        }
    }

    const int64_t r0 = int64_t(blockIdx.x) * waves_per_block;
    if (!S.text_off) {
        // One text: the wave walks its own stored hits as soon as its
        // streaming is done, while the block's other waves still stream.
        // Its (now empty) queue holds the matches: q[0] counts them, then
        // (queue entry, keyword id) pairs; the block stores them after its
        // barrier with one global atomic.  Matches beyond the stage's room go
        // out directly.
        wave_sync();
        if (lane == 0) q[0] = 0u;
        // the hit records were stored by other lanes of this wave
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        wave_sync();
        for (int i = int(lane); i < hcount; i += kWave) {
            uint4 rec;
            if (i < kLdsHits) {
                rec = shits[wave * kLdsHits + i];
            } else {
                const u32x4 g = gload16(reinterpret_cast<const uint8_t *>(hits + (i - kLdsHits)));
                rec = make_uint4(g.x, g.y, g.z, g.w);
            }
            const int64_t o = offset_of(rec.x);
            auto put = [&](int32_t pid) __attribute__((always_inline)) {
                const uint32_t at = atomicAdd(&q[0], 1u);
                if (at < uint32_t(kWaveStageCap)) {
                    q[2 + 2 * at] = rec.x;
                    q[3 + 2 * at] = uint32_t(pid);
                } else {
                    emit_one(S, nullptr, o, 0, pid);
                }
            };
            walk_rest<true>(A, S, o, S.n, rec.y, make_uint2(rec.z, rec.w),
                            [&](int32_t st) {
                                for (int32_t k = A.out_off[st], k1 = A.out_off[st + 1]; k < k1; ++k) put(A.out_pid[k]);
                            },
                            put);
        }
        __syncthreads();
        // every wave's matches are staged: one atomic reserves the block's
        // output range, the filter's LDS holds the waves' prefix sums
        int32_t *wpre = reinterpret_cast<int32_t *>(sfilt);                                // [waves + 1]
        unsigned long long *wbase = reinterpret_cast<unsigned long long *>(sfilt + 128);
        if (threadIdx.x == 0) {
            int32_t t = 0;
            for (int j = 0; j < waves_per_block; ++j) {
                wpre[j] = t;
                t += imin(int32_t(squeue[j * kQueueCap]), kWaveStageCap);
            }
            wpre[waves_per_block] = t;
            *wbase = t ? atomicAdd(S.count, static_cast<unsigned long long>(t)) - S.count_base : 0ull;
        }
        __syncthreads();
        const int32_t total = wpre[waves_per_block];
        const unsigned long long base = *wbase;
        for (int32_t i = int32_t(threadIdx.x); i < total; i += int32_t(blockDim.x)) {
            int j = 0;
            while (wpre[j + 1] <= i) ++j;
            const uint32_t *pr = squeue + j * kQueueCap + 2 + 2 * (i - wpre[j]);
            const uint32_t ent = pr[0];
            const unsigned long long idx = base + unsigned(i);
            if (idx < static_cast<unsigned long long>(S.cap)) {
                S.out_off[idx] = offset_of(ent);
                S.out_pid[idx] = int32_t(pr[1]);
            }
        }
    } else {
        // A batch: the block walks the hits its waves stored, spread over all
        // its threads (one flat index over the waves' regions), once every
        // wave is done.  The filter and queues are then free, so their LDS
        // holds the match stage (one global atomic per block) and the
        // batch's text starts for the walks' text lookups.
        // Each wave leaves its hit count in its own (empty) queue; after the
        // barrier the stage and the prefix sums of the counts go where the
        // filter was.
        if (lane == 0) q[0] = uint32_t(hcount);
        // The text starts go to LDS after the barrier; a batch of up to
        // kPreTexts starts per thread reads them now, into registers, while
        // the block's slowest waves still stream.
        constexpr int kPreTexts = 8;
        const bool pre_ok = S.n_texts < kPreTexts * int(blockDim.x) && S.n < (int64_t(1) << 32);
        int64_t pre[kPreTexts];
        int64_t pre_base = 0;
        if (pre_ok) {
            pre_base = S.text_off[0];
#pragma unroll
            for (int k = 0; k < kPreTexts; ++k) {
                const int i = int(threadIdx.x) + k * int(blockDim.x);
                pre[k] = i <= S.n_texts ? S.text_off[i] : 0;
            }
        }
        __syncthreads();
        static_assert((sizeof(MatchStage) + 15) / 16 * 16 + (2 * kMaxWaves + 1) * 4 <= (1u << FLOG2),
                      "the walk's stage must fit where the filter was");
        MatchStage *st = reinterpret_cast<MatchStage *>(sfilt);
        int32_t *wfirst = reinterpret_cast<int32_t *>(sfilt + (sizeof(MatchStage) + 15) / 16 * 16);   // [waves + 1]
        if (threadIdx.x == 0) {
            wfirst[0] = 0;
            for (int j = 0; j < waves_per_block; ++j) wfirst[j + 1] = wfirst[j] + int32_t(squeue[j * kQueueCap]);
            st->n = 0;
        }
        __syncthreads();
        const int32_t total = wfirst[waves_per_block];
        // The text starts (as offsets from the first text) are copied to LDS
        // when they fit, beside the stage or where the prefix table was.
        constexpr int kStageEnd = ((sizeof(MatchStage) + 15) / 16 * 16 + (2 * kMaxWaves + 1) * 4 + 15) / 16 * 16;
        constexpr int kLdsTexts = FLOG2 >= 17 ? ((1 << FLOG2) - kStageEnd) / 4 : 2 * PT_SLOTS;
        static_assert(kLdsTexts >= 4096, "room for the text starts of a batch of 4096 texts");
        uint32_t *lds_off = FLOG2 >= 17 ? reinterpret_cast<uint32_t *>(sfilt + kStageEnd) : sptab;
        const uint32_t *loff = nullptr;
        if (total > 0 && S.n_texts < kLdsTexts && S.n < (int64_t(1) << 32)) {
            if (pre_ok) {
#pragma unroll
                for (int k = 0; k < kPreTexts; ++k) {
                    const int i = int(threadIdx.x) + k * int(blockDim.x);
                    if (i <= S.n_texts) lds_off[i] = uint32_t(pre[k] - pre_base);
                }
            } else {
                const int64_t base0 = S.text_off[0];
                for (int i = int(threadIdx.x); i <= S.n_texts; i += int(blockDim.x))
                    lds_off[i] = uint32_t(S.text_off[i] - base0);
            }
            __syncthreads();
            loff = lds_off;
        }
        for (int32_t i = int32_t(threadIdx.x); i < total; i += int32_t(blockDim.x)) {
            int j = 0;
            while (wfirst[j + 1] <= i) ++j;          // wave (region) of flat index i
            const int k = i - wfirst[j];
            const uint4 rec = k < kLdsHits ? shits[j * kLdsHits + k] : F.hits[(r0 + j) * F.hit_cap + (k - kLdsHits)];
            const int64_t o = offset_of(rec.x);
            int64_t tstart, end;
            int32_t tid;
            locate_text(S, loff, o, tstart, end, tid);
            walk_rest<true>(A, S, o, end, rec.y, make_uint2(rec.z, rec.w),
                            [&](int32_t s2) { emit_staged(A, S, st, o - tstart, tid, s2); },
                            [&](int32_t pid) { emit_one(S, st, o - tstart, tid, pid); });
        }
        flush_stage(S, st);
    }

    // The last block to finish hands the count to the host, once every
    // block's matches are stored: the barrier waits for this block's stores,
    // the release fence makes them visible to the device before the block
    // counts itself done, and the last block's acquire fence pairs with the
    // other blocks' release fences.
    if (S.host_count) __syncthreads();
    if (S.host_count && threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long t = atomicAdd(S.done, 1ull);
        if (t == S.done_base + gridDim.x - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const unsigned long long c = atomicAdd(S.count, 0ull);
            auto *hc = (__attribute__((address_space(1))) unsigned long long *)(S.host_count);
            hc[0] = c;
            __threadfence_system();
            hc[1] = S.host_seq;      // the count is in place
            __threadfence_system();
        }
    }
}


using FilteredFn = void (*)(const KArgs);

template <int K, bool BM, int FLOG2, int STRIDE, bool DUAL = false, bool PAIR = false>
FilteredFn pick_segs(int segs) {
    switch (segs) {
        case 1: return filtered_kernel<K, BM, 1, FLOG2, STRIDE, DUAL, PAIR>;
        case 2: return filtered_kernel<K, BM, 2, FLOG2, STRIDE, DUAL, PAIR>;
        default: return filtered_kernel<K, BM, 4, FLOG2, STRIDE, DUAL, PAIR>;
    }
}

template <int K, int STRIDE>
FilteredFn pick_filter(int kind, int segs) {
    switch (kind) {
        case AC_FILTER_BYTES17: return pick_segs<K, false, 17, STRIDE>(segs);
        case AC_FILTER_BITS20: return pick_segs<K, true, 17, STRIDE>(segs);
        case AC_FILTER_BYTES16: return pick_segs<K, false, 16, STRIDE>(segs);
        case AC_FILTER_DUAL19: return pick_segs<K, true, 17, STRIDE, true>(segs);
        case AC_FILTER_PAIR20:
            // strides 2 and 4 only (resolve_launch never pairs it with stride 1)
            if constexpr (STRIDE == 2 || STRIDE == 4) return pick_segs<K, true, 17, STRIDE, false, true>(segs);
            else return nullptr;
        default: return pick_segs<K, true, 16, STRIDE>(segs);
    }
}

}  // namespace dev

// The filtered kernel of each stride (and prefix length), by filter kind and
// segments per chunk; nullptr for a combination that does not exist.
dev::FilteredFn pick_filtered_s1k1(int kind, int segs);
dev::FilteredFn pick_filtered_s1k2(int kind, int segs);
dev::FilteredFn pick_filtered_s1k3(int kind, int segs);
dev::FilteredFn pick_filtered_s2(int kind, int segs);
dev::FilteredFn pick_filtered_s4(int kind, int segs);

}  // namespace pfac
