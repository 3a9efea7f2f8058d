// HIP kernels (gfx950) of the failure-less Aho-Corasick matcher.
//
// The method (paper, Section II; Fig. 3 "N", Fig. 5): every byte offset o of
// the text starts a walk of the Goto trie at the root, follows T[o], T[o+1],
// ... while transitions exist, and reports every keyword whose state it
// enters.  No failure links are used.  Two kernels compute it:
//
// filtered_kernel (default).  A wave owns a 1-4 KiB chunk of text per step:
//   each lane holds 16 contiguous bytes per 1 KiB segment in VGPRs (one
//   coalesced 16-byte load; the 2-byte halo comes from the next lane), and
//   for each of its 16 offsets tests the first K = min(3, shortest keyword)
//   bytes against a hashed filter of the keywords' K-byte prefixes held in
//   LDS.  An offset whose prefix is not in the filter cannot start a keyword
//   (its walk dies within K steps without reaching a final state), so only
//   the rare candidate offsets are queued (wave ballot + prefix count into a
//   per-wave LDS queue) and walked, 64 at a time, through the transition
//   table in global memory (L2-resident rows; dense rows for shallow states,
//   compact child lists for deep ones).
//
// direct_kernel (plain PFAC).  A block stages its text tile plus a halo of
//   (longest keyword - 1) bytes in LDS and walks every offset from the root
//   through the dense table, itself in LDS when it fits.
//
// Both emit matches with a wave ballot: one atomic per wave reserves output
// slots, each lane writes at its rank.  The returned count is exact even when
// the output buffer is too small (only `cap` entries are written).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "filtered.hpp"

namespace pfac {

using namespace dev;

namespace {

// ---------------------------------------------------------------------------
struct DirectLaunch {
    int64_t tile;          // offsets per block
    int32_t table_bytes;   // dense table bytes staged in LDS (0 = global)
    int32_t halo;          // longest keyword - 1
};

template <bool TABLE_LDS>
__global__ __launch_bounds__(1024) void direct_kernel(const DevAut A, const ScanArgs S, const DirectLaunch L) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t *scls = smem;
    int32_t *stab = reinterpret_cast<int32_t *>(smem + 256);
    uint8_t *stext = smem + 256 + (TABLE_LDS ? L.table_bytes : 0);
    if (threadIdx.x < 64) reinterpret_cast<uint32_t *>(scls)[threadIdx.x] =
        reinterpret_cast<const uint32_t *>(A.cls)[threadIdx.x];
    if (TABLE_LDS) {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.dense);
        uint4 *dst = reinterpret_cast<uint4 *>(stab);
        for (int i = threadIdx.x; i < L.table_bytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    const int64_t t0 = int64_t(blockIdx.x) * L.tile;
    const int64_t t1 = lmin(t0 + L.tile, S.n);
    const int64_t h1 = lmin(t1 + L.halo, S.n);
    for (int64_t i = threadIdx.x; i < h1 - t0; i += blockDim.x) stext[i] = S.text[t0 + i];
    __syncthreads();
    for (int64_t o = t0 + threadIdx.x; o < t1; o += blockDim.x) {
        int32_t s = 0;
        for (int64_t j = o; j < h1; ++j) {
            const uint32_t b = stext[j - t0];
            int32_t e;
            if (TABLE_LDS) e = stab[s * A.C + scls[b]];
            else e = step_global(A, scls, s, b);
            if (e == 0) break;
            s = e & 0x7fffffff;
            if (e < 0) emit(A, S, o, 0, s);
        }
    }
}

__global__ void zero_kernel(unsigned long long *count, unsigned long long *done, int64_t *per_text, int32_t n_texts) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) *count = 0ull;
    if (i == 0 && done) *done = 0ull;
    if (per_text && i < n_texts) per_text[i] = 0;
}

// Achievable-bandwidth probe: every lane streams 16-byte words and folds them
// into one value, written once per wave so the loads cannot be dropped.  The
// loads are non-temporal, as the scan's stream loads are.
__global__ __launch_bounds__(256) void probe_read_kernel(const uint8_t *buf, int64_t n16, uint32_t *out) {
    uint32_t acc = 0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const u32x4 v = __builtin_nontemporal_load((const global_u32x4 *)(buf + i * 16));
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    for (int d = 32; d >= 1; d >>= 1) acc ^= __shfl_xor(acc, d);
    if (lane_id() == 0 && acc == 0x9E3779B9u) *out = acc;   // practically never taken
}

// strides 2 and 4 exist for K = 3 only
FilteredFn pick_filtered(int K, int kind, int segs, int stride) {
    if (stride == 4) return pick_filtered_s4(kind, segs);
    if (stride == 2) return pick_filtered_s2(kind, segs);
    if (K == 1) return pick_filtered_s1k1(kind, segs);
    if (K == 2) return pick_filtered_s1k2(kind, segs);
    return pick_filtered_s1k3(kind, segs);
}

int64_t filtered_lds(const FilterGeom &g) {
    const int64_t pt_slots = g.bytes > (64 << 10) ? 0 : 8192;
    return g.bytes + int64_t(kMaxWaves) * kQueueCap * 4 + pt_slots * 8 + int64_t(kMaxWaves) * kLdsHits * 16;
}

// Launch geometry of the filtered policy for a text of n bytes at `addr`.
struct FilteredGeom {
    FilterLaunch F;
    int64_t grid, waves;
};

FilteredGeom filtered_geom(const ac_automaton *a, const uint8_t *text, int64_t n, const ac_launch &cfg) {
    FilteredGeom G{};
    FilterLaunch &F = G.F;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(text);
    F.base = reinterpret_cast<const uint8_t *>(addr & ~uintptr_t(15));
    F.mis = int64_t(addr & 15);
    F.V = F.mis + n;
    const int64_t CH = int64_t(cfg.segs) * kSegBytes;
    F.n_chunks = (F.V + CH - 1) / CH;
    F.c_lo = F.mis > 0 ? 1 : 0;
    F.c_hi = F.V >= 16 ? (F.V - 16) / CH : 0;
    F.filter = a->dfilter[stride_set(cfg.stride) * kNumFilterKinds + cfg.filter - 1];
    const int waves = cfg.block / kWave;
    const int64_t interior = std::max<int64_t>(0, F.c_hi - F.c_lo);
    const int64_t want = (std::max<int64_t>(interior, 1) + waves - 1) / waves;
    const int64_t cap = int64_t(a->cu_count) * cfg.grid_per_cu;
    G.grid = std::max<int64_t>(1, std::min(want, cap));
    G.waves = G.grid * waves;
    return G;
}

// Launch through hipExtLaunchKernel when start/stop events are wanted (they
// are then taken from the kernel's own dispatch packet), else hipLaunchKernel.
hipError_t launch_timed(const void *fn, dim3 grid, dim3 block, void **args, size_t lds, hipStream_t stream,
                        hipEvent_t start, hipEvent_t stop) {
    if (start || stop) return hipExtLaunchKernel(fn, grid, block, args, lds, stream, start, stop, 0);
    return hipLaunchKernel(fn, grid, block, args, lds, stream);
}

std::mutex g_attr_mu;

void allow_lds(const void *fn, int64_t bytes) {
    // Raise the dynamic-LDS limit of a kernel once (160 KiB per CU on gfx950).
    std::lock_guard<std::mutex> lk(g_attr_mu);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

}  // namespace

void resolve_launch(const ac_automaton *a, int64_t len, bool batch, ac_launch &cfg) {
    const Plan &P = a->host;
    if (cfg.policy == AC_POLICY_AUTO) cfg.policy = AC_POLICY_FILTERED;
    if (batch) cfg.policy = AC_POLICY_FILTERED;
    if (cfg.policy == AC_POLICY_FILTERED) {
        // Sampling stride and map, chosen by the number of keys the map must
        // hold.  A stride of s divides the probes by s but holds s windows per
        // keyword and makes s candidates per positive; the dual map spends a
        // second hash and LDS read per probe to square the false-positive
        // rate, and the 4-byte-window map sets two bits (three at stride 2)
        // of one word per key, which cuts false positives without a second
        // LDS read.
        // Measured on MI355X (ms per GiB, two segments): 1000 printable
        // keywords 0.193 with the 4-byte-window map at stride 4, 0.214 with
        // it at stride 2, 0.217 with one 2^20-bit map at stride 2, 0.269
        // dual at stride 2; 20000 byte keywords (29958 4-byte windows at
        // stride 2) 0.275 with the 4-byte-window map at stride 2, 0.284 dual
        // at stride 2, 0.437 with the 4-byte-window map at stride 4, 0.567
        // with one 2^20-bit map at stride 2 (the stride-2 map has since
        // gained its third bit: 0.245).  On 256 MiB of random bytes, 20000
        // keywords of 8..64 bytes (39999 windows): 0.071 ms with the
        // 4-byte-window map at stride 2, 0.078 dual at stride 2, 0.099 with
        // a 2^20-bit map at stride 1; 50000 such keywords (99998 windows):
        // 0.126 with the 4-byte-window map at stride 2, 0.132 dual at stride
        // 1, 0.149 dual at stride 2.
        const bool auto_filter = cfg.filter < AC_FILTER_BYTES17 || cfg.filter > AC_FILTER_PAIR20;
        const bool auto_stride = cfg.stride != 1 && cfg.stride != 2 && cfg.stride != 4;
        const bool small_text = len < (int64_t(16) << 20);
        if (auto_stride) {
            if (auto_filter && !small_text && P.pair4 && P.n_quads4 <= kPairMaxKeys) {
                cfg.stride = 4;
                cfg.filter = AC_FILTER_PAIR20;
            } else if (P.sampled && (P.n_windows2 <= 65536 ||
                                     (auto_filter && !small_text && P.pair2 && P.n_quads2 <= kPair2MaxKeys))) {
                cfg.stride = 2;
                if (auto_filter && !small_text && P.pair2 && P.n_quads2 <= kPair2MaxKeys) cfg.filter = AC_FILTER_PAIR20;
            } else {
                cfg.stride = 1;
            }
        }
        if (cfg.stride == 4 && !P.sampled4) cfg.stride = P.sampled ? 2 : 1;
        if (cfg.stride == 2 && !P.sampled) cfg.stride = 1;
        // the 4-byte-window map exists at stride 4 only
        if (cfg.filter == AC_FILTER_PAIR20 && !((cfg.stride == 4 && P.pair4) || (cfg.stride == 2 && P.pair2)))
            cfg.filter = AC_FILTER_AUTO;
        if (cfg.filter < AC_FILTER_BYTES17 || cfg.filter > AC_FILTER_PAIR20) {
            // keys in the filter: prefixes (stride 1) or windows (strides 2, 4)
            const int64_t keys = cfg.stride == 4 ? P.n_windows4 : cfg.stride == 2 ? P.n_windows2 : P.n_prefixes;
            if (small_text) cfg.filter = keys > 1500 ? AC_FILTER_BITS19 : AC_FILTER_BYTES16;
            else if (keys <= 1500) cfg.filter = AC_FILTER_BYTES17;
            else if (keys <= 8192) cfg.filter = AC_FILTER_BITS20;
            else if (cfg.stride == 2 || keys > 20000) cfg.filter = AC_FILTER_DUAL19;
            else cfg.filter = AC_FILTER_BITS20;
        }
        FilterGeom g = filter_geom(cfg.filter);
        if (filtered_lds(g) > a->lds_per_block) {
            // the 128 KiB maps need a 160 KiB LDS; fall back to the 64 KiB ones
            if (cfg.filter == AC_FILTER_BYTES17) cfg.filter = AC_FILTER_BYTES16;
            if (cfg.filter == AC_FILTER_BITS20 || cfg.filter == AC_FILTER_DUAL19 || cfg.filter == AC_FILTER_PAIR20)
                cfg.filter = AC_FILTER_BITS19;
            g = filter_geom(cfg.filter);
        }
        if (cfg.block != 256 && cfg.block != 512 && cfg.block != 1024) cfg.block = 1024;
        // Texts under 32 MiB take one segment per wave step, which spreads
        // them over more waves (measured on MI355X: a 1 MiB scan in 11 us
        // instead of 19 with four segments).  Above that, two (1 GiB on
        // MI355X: 1000 keywords, 4-byte-window map at stride 4, 0.192 ms at
        // two and 0.200 at four; the dual map's four-segment kernel spills
        // registers), except for the 4-byte-window map at stride 2 with up
        // to 65,536 windows on texts of 256 MiB and more, where four halve
        // the per-step work of a filter-bound loop with few drains (20000
        // byte keywords, 29974 windows: 1 GiB 0.221 ms at four and 0.241 at
        // two, 256 MiB 0.070 and 0.075; 20000 keywords of 8..64 bytes, 39999
        // windows: 1 GiB 0.234 and 0.252; 50000 such keywords, 99998
        // windows, whose many drains favour two: 0.625 and 0.597).
        if (cfg.segs != 1 && cfg.segs != 2 && cfg.segs != 4) {
            cfg.segs = len < (int64_t(32) << 20) ? 1 : 2;
            if (cfg.filter == AC_FILTER_PAIR20 && cfg.stride == 2 && P.n_quads2 <= 65536 && len >= (int64_t(256) << 20))
                cfg.segs = 4;
        }
        const int64_t fit = std::max<int64_t>(1, a->lds_per_cu / filtered_lds(g));
        if (cfg.grid_per_cu <= 0 || cfg.grid_per_cu > fit) cfg.grid_per_cu = int32_t(fit);
    } else {
        if (cfg.block != 256 && cfg.block != 512 && cfg.block != 1024) cfg.block = 256;
        const int64_t table_bytes = int64_t(P.S_dense) * P.C * 4;
        const bool fits = P.S_dense == P.S && table_bytes + 256 + 8192 + P.max_len + 64 <= a->lds_per_block;
        if (cfg.table_in_lds == 1 && !fits) cfg.table_in_lds = 2;
        if (cfg.table_in_lds != 1 && cfg.table_in_lds != 2) cfg.table_in_lds = fits ? 1 : 2;
    }
}

int launch_probe_read(const uint8_t *buf, int64_t n, uint32_t *out, hipStream_t stream, std::string &err) {
    if (n <= 0) return AC_OK;
    int dev = 0, cus = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n16 = n / 16;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n16 + 255) / 256, int64_t(cus) * 8));
    probe_read_kernel<<<unsigned(grid), 256, 0, stream>>>(buf, n16, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { err = std::string("probe launch: ") + hipGetErrorString(e); return AC_EHIP; }
    return AC_OK;
}

int launch_zero(unsigned long long *count, unsigned long long *done, int64_t *per_text, int32_t n_texts,
                hipStream_t stream, std::string &err) {
    const int32_t threads = 256;
    const int32_t blocks = std::max<int32_t>(1, (std::max<int32_t>(n_texts, 1) + threads - 1) / threads);
    zero_kernel<<<blocks, threads, 0, stream>>>(count, done, per_text, n_texts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { err = std::string("zero_kernel launch: ") + hipGetErrorString(e); return AC_EHIP; }
    return AC_OK;
}

int64_t scan_regions(const ac_automaton *a, const uint8_t *text, int64_t n, const ac_launch &cfg) {
    if (cfg.policy != AC_POLICY_FILTERED || n <= 0) return 0;
    return filtered_geom(a, text, n, cfg).waves;
}

int64_t widest_scan_regions(int cu_count, int64_t lds_per_cu) {
    // a filtered launch has at most (LDS per CU / the smallest filter's LDS)
    // blocks per CU, each of at most kMaxWaves waves
    return int64_t(cu_count) * std::max<int64_t>(1, lds_per_cu / filtered_lds(filter_geom(AC_FILTER_BITS19))) *
           kMaxWaves;
}

int launch_scan(const ac_automaton *a, const ScanArgs &S, const ac_launch &cfg, const HitScratch &hs,
                hipStream_t stream, std::string &err, const KernelTiming *timing, int64_t *blocks) {
    if (blocks) *blocks = 0;
    const KernelTiming none;
    const KernelTiming &T = timing ? *timing : none;
    if (S.n <= 0) return AC_OK;
    const Plan &P = a->host;
    hipError_t e = hipSuccess;
    if (cfg.policy == AC_POLICY_FILTERED) {
        FilteredGeom G = filtered_geom(a, S.text, S.n, cfg);
        FilterLaunch &F = G.F;
        if (!hs.hits || hs.regions < G.waves || hs.cap < kDrain) {
            err = "scan scratch too small for the launch";
            return AC_EINVAL;
        }
        F.hits = hs.hits;
        F.hit_cap = hs.cap;
        const int64_t interior = std::max<int64_t>(0, F.c_hi - F.c_lo);
        // queue entries hold (slot << 12 | position): a block's slots must fit 20 bits
        if (interior / G.grid + 2 * (cfg.block / kWave) >= (int64_t(1) << 20)) {
            err = "text too large for one launch";
            return AC_EINVAL;
        }
        FilteredFn fn = pick_filtered(P.K, cfg.filter, cfg.segs, cfg.stride);
        if (!fn) { err = "no kernel for this filter and stride"; return AC_EINVAL; }
        KArgs KA{a->dev, S, F};
        void *fargs[] = {&KA};
        e = launch_timed(reinterpret_cast<const void *>(fn), dim3(unsigned(G.grid)), dim3(unsigned(cfg.block)), fargs, 0,
                         stream, T.scan0, T.scan1);
        if (blocks && e == hipSuccess) *blocks = G.grid;
        if (e != hipSuccess) { err = std::string("scan launch: ") + hipGetErrorString(e); return AC_EHIP; }
    } else if (cfg.policy == AC_POLICY_DIRECT) {
        if (S.text_off) { err = "direct policy does not scan batches"; return AC_ENOTSUP; }
        DirectLaunch L;
        L.tile = 8192;
        L.halo = P.max_len - 1;
        const bool lds_table = cfg.table_in_lds == 1;
        L.table_bytes = lds_table ? int32_t((int64_t(P.S_dense) * P.C * 4 + 15) / 16 * 16) : 0;
        const int64_t lds = 256 + L.table_bytes + L.tile + L.halo + 16;
        const int64_t grid = (S.n + L.tile - 1) / L.tile;
        if (lds > a->lds_per_block) { err = "direct policy: tile and table exceed LDS"; return AC_ENOTSUP; }
        auto fn = lds_table ? direct_kernel<true> : direct_kernel<false>;
        allow_lds(reinterpret_cast<const void *>(fn), lds);
        DevAut A = a->dev;
        ScanArgs SA = S;
        void *dargs[] = {&A, &SA, &L};
        e = launch_timed(reinterpret_cast<const void *>(fn), dim3(unsigned(grid)), dim3(unsigned(cfg.block)), dargs,
                         size_t(lds), stream, T.scan0, T.scan1);
    } else {
        err = "unknown policy";
        return AC_EINVAL;
    }
    if (e != hipSuccess) { err = std::string("scan launch: ") + hipGetErrorString(e); return AC_EHIP; }
    return AC_OK;
}

}  // namespace pfac
