// C ABI of the failure-less Aho-Corasick matcher: argument checks, device
// upload of a built automaton, per-stream count buffers, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <system_error>
#include <utility>
#include <vector>

#include "pfac_internal.hpp"

using namespace pfac;

namespace {

thread_local std::string g_err;
thread_local float g_scan_ms = -1.0f;
thread_local float g_stream_ms = -1.0f, g_walk_ms = -1.0f;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(const char *what, hipError_t e) {
    return fail(AC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// One device count word and one pinned host word per (device, stream),
// allocated on first use and kept until the stream's scratch is released.
// The synchronous calls never clear the device word: it only grows, the
// pinned word holds its value after the last such call, and a scan numbers
// its matches from that value on (ScanArgs::count_base).  A batch call that
// asks for per-text counts clears it along with them (one clearing kernel).
// The filtered policy's hit regions are sized for the widest launch when the
// slot is created and never change afterwards, so a HIP graph that captured
// their address stays valid.
struct CountSlot {
    unsigned long long *d = nullptr;           // [0] match count, [1] finished blocks
    unsigned long long *h = nullptr;           // pinned: [0] count, [1] sequence number of the last report
    unsigned long long seq = 0;                // last sequence number handed to a scan
    unsigned long long done_total = 0;         // value of d[1] after the last synchronous call
    bool stale = false;                        // a failed call may have left *d != *h
    hipEvent_t ev[2] = {nullptr, nullptr};   // kernel timing: scan start, stop
    HitScratch hs;                             // hit regions of the filtered policy
    // ac_match_dispatch's device staging, grown to the largest call
    uint8_t *d_text = nullptr;
    int64_t text_cap = 0;
    int64_t *d_off = nullptr;
    int32_t *d_pid = nullptr;
    int64_t match_cap = 0;
};
std::mutex g_slots_mu;
std::map<std::pair<int, hipStream_t>, CountSlot> g_slots;

void free_slot(CountSlot &s) {
    if (s.d) (void)hipFree(s.d);
    if (s.h) (void)hipHostFree(s.h);
    for (hipEvent_t ev : s.ev)
        if (ev) (void)hipEventDestroy(ev);
    if (s.hs.hits) (void)hipFree(s.hs.hits);
    for (void *p : {static_cast<void *>(s.d_text), static_cast<void *>(s.d_off), static_cast<void *>(s.d_pid)})
        if (p) (void)hipFree(p);
    s = CountSlot();
}

// Grows the slot's dispatch staging to `text` bytes and `matches` entries.
int ensure_staging(CountSlot &s, int64_t text, int64_t matches) {
    hipError_t e = hipSuccess;
    if (text > s.text_cap) {
        const int64_t cap = std::max<int64_t>(text, 2 * s.text_cap);
        if (s.d_text) (void)hipFree(s.d_text);
        s.d_text = nullptr;
        s.text_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&s.d_text), size_t(cap))) != hipSuccess)
            return fail(AC_ENOMEM, std::string("hipMalloc(dispatch text): ") + hipGetErrorString(e));
        s.text_cap = cap;
    }
    if (matches > s.match_cap) {
        if (s.d_off) (void)hipFree(s.d_off);
        if (s.d_pid) (void)hipFree(s.d_pid);
        s.d_off = nullptr;
        s.d_pid = nullptr;
        s.match_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&s.d_off), size_t(matches) * 8)) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void **>(&s.d_pid), size_t(matches) * 4)) != hipSuccess)
            return fail(AC_ENOMEM, std::string("hipMalloc(dispatch matches): ") + hipGetErrorString(e));
        s.match_cap = matches;
    }
    return AC_OK;
}

// The slot of (device, stream), created on first use with hit regions for
// `regions` waves (the widest launch on the device); the pointer stays valid
// until the slot is released.
int count_slot(int device, hipStream_t stream, CountSlot **out, int64_t regions) {
    std::lock_guard<std::mutex> lk(g_slots_mu);
    auto key = std::make_pair(device, stream);
    auto it = g_slots.find(key);
    if (it != g_slots.end()) {
        *out = &it->second;
        return it->second.hs.regions >= regions ? AC_OK
                                                : fail(AC_EINVAL, "stream scratch has fewer hit regions than the launch");
    }
    CountSlot s;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&s.d), 2 * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail("hipMalloc(count)", e);
    // coherent: the scan kernel stores the count here itself
    e = hipHostMalloc(reinterpret_cast<void **>(&s.h), 2 * sizeof(unsigned long long), hipHostMallocCoherent);
    if (e != hipSuccess) { free_slot(s); return hip_fail("hipHostMalloc(count)", e); }
    s.h[0] = s.h[1] = 0;
    s.stale = true;                            // cleared by the first call
    for (auto &ev : s.ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) { free_slot(s); return hip_fail("hipEventCreate", e); }
    e = hipMalloc(reinterpret_cast<void **>(&s.hs.hits), size_t(regions) * kHitCap * sizeof(uint4));
    if (e != hipSuccess) { free_slot(s); return fail(AC_ENOMEM, std::string("hipMalloc(hit regions): ") + hipGetErrorString(e)); }
    s.hs.regions = regions;
    s.hs.cap = kHitCap;
    CountSlot &slot = g_slots[key];
    slot = s;
    *out = &slot;
    return AC_OK;
}

// The calling stream's slot, with hit regions for any launch on a's device.
int slot_for(const ac_automaton *a, hipStream_t stream, CountSlot **out) {
    return count_slot(a->device, stream, out, widest_scan_regions(a->cu_count, a->lds_per_cu));
}

int64_t pad256(int64_t x) { return (x + 255) / 256 * 256; }

// Compute units and LDS bytes (per block, per CU) of device `dev`.
int device_props(int dev, int *cus, int64_t *lds_block, int64_t *lds_cu) {
    int c = 0, lds = 0, lds_optin = 0, per_cu = 0;
    hipError_t e;
    if ((e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail("hipDeviceGetAttribute(cu)", e);
    if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
        return hip_fail("hipDeviceGetAttribute(lds)", e);
    if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) {
        lds_optin = 0;
        (void)hipGetLastError();
    }
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess) {
        per_cu = 0;
        (void)hipGetLastError();
    }
    *cus = std::max(1, c);
    *lds_block = std::max(lds, lds_optin);
    *lds_cu = std::max<int64_t>(per_cu, *lds_block);
    return AC_OK;
}

int upload(ac_automaton *a) {
    const Plan &P = a->host;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    a->device = dev;
    int rc = device_props(dev, &a->cu_count, &a->lds_per_block, &a->lds_per_cu);
    if (rc) return rc;

    // section layout (each section 256-byte aligned and padded)
    struct Sec { const void *src; int64_t bytes; int64_t at; };
    Sec cls{P.cls, 256, 0};
    Sec filt[kNumFilters];
    Sec dense{P.dense.data(), int64_t(P.dense.size()) * 4, 0};
    Sec node{P.node.data(), int64_t(P.node.size()) * 4, 0};
    Sec label{P.label.data(), int64_t(P.label.size()), 0};
    Sec ooff{P.out_off.data(), int64_t(P.out_off.size()) * 4, 0};
    Sec opid{P.out_pid.data(), int64_t(P.out_pid.size()) * 4, 0};
    Sec ptab{P.ptab.data(), int64_t(P.ptab.size()) * 4, 0};
    Sec tail{P.tail.data(), int64_t(P.tail.size()) * 4, 0};
    Sec tinfo{P.tailinfo.data(), int64_t(P.tailinfo.size()) * 4, 0};
    Sec kwb{P.kw_bytes.data(), int64_t(P.kw_bytes.size()), 0};
    Sec kwo{P.kw_off.data(), int64_t(P.kw_off.size()) * 4, 0};
    int64_t at = 0;
    auto place = [&](Sec &s) { s.at = at; at += pad256(std::max<int64_t>(s.bytes, 1)); };
    place(cls);
    for (int k = 0; k < kNumFilters; ++k) {
        filt[k] = Sec{P.filter[k].data(), int64_t(P.filter[k].size()), 0};
        place(filt[k]);
    }
    place(dense); place(node); place(label); place(ooff); place(opid);
    place(ptab); place(tail); place(tinfo); place(kwb); place(kwo);
    a->dbytes = at;
    std::vector<uint8_t> staging(size_t(at), 0);
    auto copy = [&](const Sec &s) { if (s.bytes) std::memcpy(staging.data() + s.at, s.src, size_t(s.bytes)); };
    copy(cls); for (auto &f : filt) copy(f); copy(dense); copy(node); copy(label); copy(ooff); copy(opid);
    copy(ptab); copy(tail); copy(tinfo); copy(kwb); copy(kwo);
    e = hipMalloc(&a->dmem, size_t(at));
    if (e != hipSuccess) { a->dmem = nullptr; return fail(AC_ENOMEM, std::string("hipMalloc(automaton): ") + hipGetErrorString(e)); }
    e = hipMemcpy(a->dmem, staging.data(), size_t(at), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail("hipMemcpy(automaton)", e);
    uint8_t *b = static_cast<uint8_t *>(a->dmem);
    DevAut &D = a->dev;
    D.cls = b + cls.at;
    for (int k = 0; k < kNumFilters; ++k) a->dfilter[k] = b + filt[k].at;
    D.dense = reinterpret_cast<const int32_t *>(b + dense.at);
    D.node = reinterpret_cast<const int32_t *>(b + node.at);
    D.label = b + label.at;
    D.out_off = reinterpret_cast<const int32_t *>(b + ooff.at);
    D.out_pid = reinterpret_cast<const int32_t *>(b + opid.at);
    D.ptab = reinterpret_cast<const uint32_t *>(b + ptab.at);
    D.tailinfo = reinterpret_cast<const int4 *>(b + tinfo.at);
    D.kw_bytes = b + kwb.at;
    D.ptab_bits = P.ptab_bits;
    D.C = P.C;
    D.S_dense = P.S_dense;
    D.K = P.K;
    D.hash_mul = P.hash_mul;
    return AC_OK;
}

void fill_info(const Plan &P, ac_info_t *o) {
    std::memset(o, 0, sizeof(*o));
    o->n_patterns = P.n_patterns;
    o->n_states = P.S;
    o->n_classes = P.C;
    o->min_len = P.min_len;
    o->max_len = P.max_len;
    o->prefix_len = P.K;
    o->n_dense_states = P.S_dense;
    o->dense_depth = P.dense_depth;
    o->n_prefixes = P.n_prefixes;
    o->n_windows2 = P.sampled ? P.n_windows2 : 0;
    o->n_windows4 = P.sampled4 ? P.n_windows4 : 0;
    o->n_quads4 = P.pair4 ? P.n_quads4 : 0;
    o->n_quads2 = P.pair2 ? P.n_quads2 : 0;
    o->dense_bytes = int64_t(P.dense.size()) * 4;
    o->compact_bytes = int64_t(P.node.size()) * 4 + int64_t(P.label.size());
    o->output_bytes = int64_t(P.out_off.size() + P.out_pid.size()) * 4;
    o->prefix_table_bytes = int64_t(P.ptab.size()) * 4;
    o->tail_bytes = int64_t(P.tail.size() + P.tailinfo.size()) * 4 + int64_t(P.kw_bytes.size()) +
                    int64_t(P.kw_off.size()) * 4;
    for (const auto &f : P.filter) o->filter_bytes += int64_t(f.size());
    o->device_bytes = 256 + o->dense_bytes + o->compact_bytes + o->output_bytes + o->filter_bytes +
                      o->prefix_table_bytes + o->tail_bytes;
    o->build_ms = P.build_ms;
}

int check_launch(const ac_launch *l) {
    if (!l) return AC_OK;
    if (l->policy < AC_POLICY_AUTO || l->policy > AC_POLICY_DIRECT) return fail(AC_EINVAL, "ac_launch: bad policy");
    if (l->filter < AC_FILTER_AUTO || l->filter > AC_FILTER_PAIR20) return fail(AC_EINVAL, "ac_launch: bad filter");
    if (l->block != 0 && l->block != 256 && l->block != 512 && l->block != 1024)
        return fail(AC_EINVAL, "ac_launch: block must be 256, 512 or 1024");
    if (l->segs != 0 && l->segs != 1 && l->segs != 2 && l->segs != 4)
        return fail(AC_EINVAL, "ac_launch: segs must be 1, 2 or 4");
    if (l->grid_per_cu < 0 || l->grid_per_cu > 64) return fail(AC_EINVAL, "ac_launch: bad grid_per_cu");
    if (l->flags & ~AC_LAUNCH_TIME_SCAN) return fail(AC_EINVAL, "ac_launch: unknown flags");
    if (l->stride < 0 || l->stride > 4 || l->stride == 3) return fail(AC_EINVAL, "ac_launch: stride must be 0, 1, 2 or 4");
    return AC_OK;
}

int device_matches(const ac_automaton *a) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    if (dev != a->device) return fail(AC_EINVAL, "automaton was built on another device than the current one");
    return AC_OK;
}

// Enqueue zero + scan for one text or a batch.
int length_bucket(int64_t n) {
    int b = 0;
    while (n >= 4) { n >>= 2; ++b; }
    return b;
}

// Whether a launch leaves every choice to the library (NULL or all zero but
// for the flags).
bool all_auto(const ac_launch *l) {
    return !l || (l->policy == 0 && l->filter == 0 && l->block == 0 && l->segs == 0 && l->grid_per_cu == 0 &&
                  l->table_in_lds == 0 && l->stride == 0);
}

ac_launch resolved(const ac_automaton *a, const ScanArgs &S, const ac_launch *launch, bool batch) {
    ac_launch cfg{};
    if (launch) cfg = *launch;
    if (all_auto(launch)) {
        // a choice measured by ac_tune / ac_tune_batch for this length, if any
        std::lock_guard<std::mutex> lk(a->tune_mu);
        const auto &tuned = batch ? a->tuned_batch : a->tuned;
        auto it = tuned.find(length_bucket(S.n));
        if (it != tuned.end()) {
            const int32_t flags = cfg.flags;
            cfg = it->second;
            cfg.flags = flags;
        }
    }
    resolve_launch(a, S.n, batch, cfg);
    return cfg;
}

// Enqueue the scan of one text or a batch.  `clear` first zeroes *d_count
// (and the batch's per-text counts); otherwise matches are numbered from
// S.count_base.
int enqueue(const ac_automaton *a, ScanArgs S, const ac_launch &cfg, bool batch, bool clear,
            unsigned long long *d_count, const HitScratch &hs, hipStream_t stream,
            const KernelTiming *timing = nullptr, int64_t *blocks = nullptr) {
    S.count = d_count;
    std::string err;
    if (clear) {
        S.count_base = 0;
        S.done_base = 0;
        int rc = launch_zero(d_count, S.done, S.per_text, batch ? S.n_texts : 0, stream, err);
        if (rc) return fail(rc, err);
    }
    int rc = launch_scan(a, S, cfg, hs, stream, err, timing, blocks);
    return rc ? fail(rc, err) : AC_OK;
}

int64_t sync_count(const ac_automaton *a, ScanArgs S, const ac_launch *launch, bool batch, hipStream_t stream) {
    if (batch && launch && launch->policy == AC_POLICY_DIRECT) return fail(AC_ENOTSUP, "batches use the filtered policy");
    const ac_launch cfg = resolved(a, S, launch, batch);
    CountSlot *slot = nullptr;
    int rc = slot_for(a, stream, &slot);
    if (rc) return rc;
    const bool timed = launch && (launch->flags & AC_LAUNCH_TIME_SCAN) && S.n > 0;
    g_scan_ms = g_stream_ms = g_walk_ms = -1.0f;
    KernelTiming T;
    if (timed) {
        T.scan0 = slot->ev[0];
        T.scan1 = slot->ev[1];
    }
    // a batch with per-text counts clears the word (its counts need a
    // clearing kernel anyway); any other call numbers on from the word
    const bool clear = (batch && S.per_text) || slot->stale;
    const unsigned long long base = clear ? 0ull : *slot->h;
    S.count_base = base;
    if (S.n == 0 && !clear) return 0;              // nothing to scan, nothing to clear
    slot->stale = true;
    // the filtered policy's last block stores the count into the pinned word
    const bool reported = cfg.policy == AC_POLICY_FILTERED && S.n > 0;
    S.done = slot->d + 1;                          // cleared with the count
    if (clear) slot->done_total = 0;
    S.done_base = slot->done_total;
    S.host_count = reported ? slot->h : nullptr;
    S.host_seq = ++slot->seq;
    int64_t blocks = 0;
    rc = enqueue(a, S, cfg, batch, clear, slot->d, slot->hs, stream, timed ? &T : nullptr, &blocks);
    if (rc) return rc;
    hipError_t e = hipSuccess;
    if (!reported) {
        e = hipMemcpyAsync(slot->h, slot->d, sizeof(unsigned long long), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return hip_fail("hipMemcpyAsync(count)", e);
    }
    if (reported && !timed) {
        // The count is final once the last block has stored it with this
        // call's sequence number; every match and per-text count is written
        // by then.  Waiting on the word skips the stream's completion path.
        // The stream is polled now and then, so a failed launch or a kernel
        // that ended without reporting ends the wait too.
        for (uint64_t spin = 1; __atomic_load_n(&slot->h[1], __ATOMIC_ACQUIRE) != S.host_seq; ++spin) {
#if defined(__x86_64__)
            __builtin_ia32_pause();
#endif
            if (spin % 65536 != 0) continue;
            e = hipStreamQuery(stream);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return hip_fail("hipStreamQuery", e);
            if (__atomic_load_n(&slot->h[1], __ATOMIC_ACQUIRE) != S.host_seq)
                return fail(AC_EHIP, "scan finished without reporting its count");
            break;
        }
    } else {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail("hipStreamSynchronize", e);
    }
    if (reported) slot->done_total += uint64_t(blocks);
    slot->stale = false;
    if (timed) {
        float ms = -1.0f;
        if ((e = hipEventElapsedTime(&ms, T.scan0, T.scan1)) != hipSuccess) return hip_fail("hipEventElapsedTime", e);
        g_scan_ms = g_stream_ms = ms;
        g_walk_ms = 0.0f;
    }
    return int64_t(__atomic_load_n(&slot->h[0], __ATOMIC_ACQUIRE) - base);
}

int check_single(const ac_automaton *a, const uint8_t *d_text, int64_t len, const ac_matches *m) {
    if (!a) return fail(AC_EINVAL, "ac_match: NULL automaton");
    if (len < 0) return fail(AC_EINVAL, "ac_match: negative length");
    if (len > 0 && !d_text) return fail(AC_EINVAL, "ac_match: NULL text");
    if (m) {
        if (m->capacity < 0) return fail(AC_EINVAL, "ac_match: negative capacity");
        if (m->capacity > 0 && (!m->offset || !m->pattern_id)) return fail(AC_EINVAL, "ac_match: NULL match arrays");
    }
    return device_matches(a);
}

ScanArgs single_args(const uint8_t *d_text, int64_t len, const ac_matches *m) {
    ScanArgs S{};
    S.text = d_text;
    S.n = len;
    if (m && m->capacity > 0) {
        S.out_off = m->offset;
        S.out_pid = m->pattern_id;
        S.cap = m->capacity;
    }
    return S;
}

int check_batch(const ac_automaton *a, const uint8_t *d_texts, const int64_t *d_off, int32_t n_texts,
                int64_t total, const ac_batch_matches *m) {
    if (!a) return fail(AC_EINVAL, "ac_match_batch: NULL automaton");
    if (n_texts < 0) return fail(AC_EINVAL, "ac_match_batch: negative text count");
    if (total < 0) return fail(AC_EINVAL, "ac_match_batch: negative total bytes");
    if (n_texts > 0 && !d_off) return fail(AC_EINVAL, "ac_match_batch: NULL offsets");
    if (total > 0 && !d_texts) return fail(AC_EINVAL, "ac_match_batch: NULL texts");
    if (m) {
        if (m->capacity < 0) return fail(AC_EINVAL, "ac_match_batch: negative capacity");
        if (m->capacity > 0 && (!m->offset || !m->pattern_id || !m->text_id))
            return fail(AC_EINVAL, "ac_match_batch: NULL match arrays");
    }
    return device_matches(a);
}

ScanArgs batch_args(const uint8_t *d_texts, const int64_t *d_off, int32_t n_texts, int64_t total,
                    const ac_batch_matches *m) {
    ScanArgs S{};
    S.text = d_texts;
    S.n = n_texts > 0 ? total : 0;
    S.text_off = d_off;
    S.n_texts = n_texts;
    if (m) {
        if (m->capacity > 0) {
            S.out_off = m->offset;
            S.out_pid = m->pattern_id;
            S.out_tid = m->text_id;
            S.cap = m->capacity;
        }
        S.per_text = m->per_text_count;
    }
    return S;
}

int check_host(const void *h, const uint8_t *text, int64_t len, int64_t *off, int32_t *pid, int64_t cap,
               const char *who) {
    if (!h) return fail(AC_EINVAL, std::string(who) + ": NULL automaton");
    if (len < 0) return fail(AC_EINVAL, std::string(who) + ": negative length");
    if (len > 0 && !text) return fail(AC_EINVAL, std::string(who) + ": NULL text");
    if (cap < 0) return fail(AC_EINVAL, std::string(who) + ": negative capacity");
    if (cap > 0 && (!off || !pid)) return fail(AC_EINVAL, std::string(who) + ": NULL match arrays");
    return AC_OK;
}

int64_t host_match_checked(const Plan &P, const uint8_t *text, int64_t len, int64_t *off, int32_t *pid,
                           int64_t cap, int32_t n_threads) {
    try {
        return host_match(P, text, len, off, pid, cap, n_threads);
    } catch (const std::bad_alloc &) {
        return fail(AC_ENOMEM, "CPU matcher: out of host memory");
    } catch (const std::system_error &e) {
        return fail(AC_ENOMEM, std::string("CPU matcher: cannot start threads: ") + e.what());
    }
}

// GPU side of the dispatch: host text -> device, scan, matches -> host.
int64_t gpu_round_trip(const ac_automaton *a, const uint8_t *text, int64_t len, int64_t *off, int32_t *pid,
                       int64_t cap, hipStream_t stream) {
    if (len == 0) return 0;
    CountSlot *slot = nullptr;
    int rc = slot_for(a, stream, &slot);
    if (rc) return rc;
    if ((rc = ensure_staging(*slot, len, std::max<int64_t>(cap, 1)))) return rc;
    hipError_t e = hipMemcpyAsync(slot->d_text, text, size_t(len), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail("hipMemcpyAsync(dispatch text)", e);
    ScanArgs S{};
    S.text = slot->d_text;
    S.n = len;
    if (cap > 0) {
        S.out_off = slot->d_off;
        S.out_pid = slot->d_pid;
        S.cap = cap;
    }
    const int64_t count = sync_count(a, S, nullptr, false, stream);
    if (count < 0) return count;
    const int64_t put = std::min(count, cap);
    if (put > 0) {
        if ((e = hipMemcpyAsync(off, slot->d_off, size_t(put) * 8, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipMemcpyAsync(pid, slot->d_pid, size_t(put) * 4, hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return hip_fail("hipMemcpyAsync(dispatch matches)", e);
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail("hipStreamSynchronize", e);
    }
    return count;
}

// Times every choice of the filtered policy (stride, filter map, segments)
// on S, three runs each (the first warms up), and records the fastest for
// single texts or batches of S's length bucket.
int tune(ac_automaton *a, const ScanArgs &S, bool batch, hipStream_t stream, ac_launch *out) {
    const Plan &P = a->host;
    std::vector<ac_launch> cands;
    for (int stride : {1, 2, 4}) {
        if ((stride == 2 && !P.sampled) || (stride == 4 && !P.sampled4)) continue;
        for (int filter = AC_FILTER_BYTES17; filter <= AC_FILTER_PAIR20; ++filter)
            for (int segs : {1, 2, 4}) {
                ac_launch c{};
                c.policy = AC_POLICY_FILTERED;
                c.filter = filter;
                c.segs = segs;
                c.stride = stride;
                cands.push_back(c);
            }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail("hipEventCreate", e);
    int rc = AC_OK;
    float best_ms = 1e30f;
    ac_launch best{};
    for (const ac_launch &c0 : cands) {
        ac_launch cfg = c0;
        resolve_launch(a, S.n, batch, cfg);
        if (cfg.filter != c0.filter || cfg.stride != c0.stride) continue;   // not available here
        float ms_sum = 0.0f;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
            CountSlot *slot = nullptr;
            if ((rc = slot_for(a, stream, &slot))) break;
            KernelTiming T;
            T.scan0 = e0;
            T.scan1 = e1;
            ScanArgs SA = S;
            SA.done = slot->d + 1;
            slot->stale = true;                  // the next synchronous call clears the count
            if ((rc = enqueue(a, SA, cfg, batch, true, slot->d, slot->hs, stream, &T))) break;
            if ((e = hipStreamSynchronize(stream)) != hipSuccess) { rc = hip_fail("hipStreamSynchronize", e); break; }
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_fail("hipEventElapsedTime", e); break; }
            if (rep > 0) ms_sum += ms;
        }
        if (rc) break;
        if (ms_sum < best_ms) {
            best_ms = ms_sum;
            best = c0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(a->tune_mu);
        (batch ? a->tuned_batch : a->tuned)[length_bucket(S.n)] = best;
    }
    if (out) {
        *out = best;
        resolve_launch(a, S.n, batch, *out);
    }
    return AC_OK;
}

int build_common(const uint8_t *bytes, const int64_t *offsets, int32_t n, const ac_build_opts *opts,
                 ac_automaton **out) {
    if (!out) return fail(AC_EINVAL, "ac_build: NULL output pointer");
    *out = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    ac_automaton *a = new (std::nothrow) ac_automaton();
    if (!a) return fail(AC_ENOMEM, "ac_build: out of host memory");
    std::string err;
    int rc;
    try {
        rc = compile_plan(bytes, offsets, n, opts, a->host, err);
    } catch (const std::bad_alloc &) {
        rc = AC_ENOMEM;
        err = "ac_build: out of host memory";
    }
    if (rc) { delete a; return fail(rc, err); }
    rc = upload(a);
    if (rc) { if (a->dmem) (void)hipFree(a->dmem); delete a; return rc; }
    a->host.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = a;
    return AC_OK;
}

}  // namespace

int pfac::report_error(int code, const std::string &msg) { return fail(code, msg); }

int pfac::reserve_stream_scratch(hipStream_t stream, int64_t *device_bytes) {
    int dev = 0, cus = 1;
    int64_t lds_block = 0, lds_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    int rc = device_props(dev, &cus, &lds_block, &lds_cu);
    if (rc) return rc;
    CountSlot *slot = nullptr;
    rc = count_slot(dev, stream, &slot, widest_scan_regions(cus, lds_cu));
    if (!rc && device_bytes)
        *device_bytes = 2 * int64_t(sizeof(unsigned long long)) + slot->hs.regions * slot->hs.cap * int64_t(sizeof(uint4));
    return rc;
}

void pfac::release_stream_scratch(hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_slots_mu);
    auto it = g_slots.find(std::make_pair(dev, stream));
    if (it == g_slots.end()) return;
    free_slot(it->second);
    g_slots.erase(it);
}

namespace {

// ---- the allocation-free scan's scratch ----------------------------------
// Hit regions of ac_match_async_noalloc: a fixed device array that each GPU
// holds for the life of the process (16 MiB: 4096 waves x 256 records of
// 16 bytes, the widest launch on a 256-CU MI355X).  In host code `scratch`
// only names the array; its device address, one per GPU, comes from
// hipGetSymbolAddress with that GPU current.
constexpr int64_t kStaticScratchBytes = int64_t(16) << 20;
// fewest records per region the scan accepts: two drains' worth
constexpr int64_t kNoallocMinCap = 128;
static __device__ __align__(256) uint4 scratch[kStaticScratchBytes / sizeof(uint4)];
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
uint4 *g_static_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (set on the first call there).
int static_scratch(int dev, uint4 **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(AC_EINVAL, "ac_match_async_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail("hipGetSymbolAddress(scratch)", e);
        if (!p) return fail(AC_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_static_ptr[dev] = static_cast<uint4 *>(p);
    }
    *out = g_static_ptr[dev];
    return AC_OK;
}

}  // namespace

extern "C" {

int ac_match_async_noalloc(const ac_automaton *a, const uint8_t *d_text, int64_t len, const ac_matches *matches,
                           const ac_launch *launch, int64_t *d_count, hipStream_t stream) {
    int rc = check_single(a, d_text, len, matches);
    if (rc) return rc;
    if ((rc = check_launch(launch))) return rc;
    if (!d_count) return fail(AC_EINVAL, "ac_match_async_noalloc: NULL count pointer");
    const ScanArgs S = single_args(d_text, len, matches);
    const ac_launch cfg = resolved(a, S, launch, false);
    HitScratch hs;
    if (cfg.policy == AC_POLICY_FILTERED && len > 0) {
        const int64_t regions = scan_regions(a, S.text, S.n, cfg);
        const int64_t cap = std::min<int64_t>(kHitCap, kStaticScratchBytes / int64_t(sizeof(uint4)) / regions);
        if (cap < kNoallocMinCap)
            return fail(AC_EINVAL, "ac_match_async_noalloc: the launch needs " + std::to_string(regions) +
                                       " hit regions of at least " + std::to_string(kNoallocMinCap) +
                                       " records; the static scratch holds " +
                                       std::to_string(kStaticScratchBytes) + " bytes");
        if ((rc = static_scratch(a->device, &hs.hits))) return rc;
        hs.regions = regions;
        hs.cap = int32_t(cap);
    }
    return enqueue(a, S, cfg, false, true, reinterpret_cast<unsigned long long *>(d_count), hs, stream);
}

const char *ac_last_error(void) { return g_err.c_str(); }

float ac_last_scan_ms(void) { return g_scan_ms; }

void ac_last_scan_split(float *stream_ms, float *walk_ms) {
    if (stream_ms) *stream_ms = g_stream_ms;
    if (walk_ms) *walk_ms = g_walk_ms;
}

int ac_release_stream(hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    pfac::release_stream_scratch(stream);
    return AC_OK;
}

int ac_probe_read(const uint8_t *d_buf, int64_t n, uint32_t *d_out, hipStream_t stream) {
    if (!d_buf || !d_out || n < 0 || (n % 16) || (reinterpret_cast<uintptr_t>(d_buf) % 16))
        return fail(AC_EINVAL, "ac_probe_read: buffer must be 16-byte aligned and a multiple of 16 bytes");
    std::string err;
    int rc = launch_probe_read(d_buf, n, d_out, stream, err);
    return rc ? fail(rc, err) : AC_OK;
}

int ac_build_csr(const uint8_t *bytes, const int64_t *offsets, int32_t n_patterns, const ac_build_opts *opts,
                 ac_automaton **out) {
    return build_common(bytes, offsets, n_patterns, opts, out);
}

int ac_build(const uint8_t *const *patterns, const int64_t *lengths, int32_t n_patterns,
             const ac_build_opts *opts, ac_automaton **out) {
    if (n_patterns <= 0) return fail(AC_EINVAL, "ac_build: need at least one keyword");
    if (!patterns || !lengths) return fail(AC_EINVAL, "ac_build: NULL keyword arrays");
    std::vector<int64_t> offs(size_t(n_patterns) + 1, 0);
    for (int32_t i = 0; i < n_patterns; ++i) {
        if (lengths[i] <= 0) return fail(AC_EINVAL, "ac_build: keyword " + std::to_string(i) + " is empty");
        if (!patterns[i]) return fail(AC_EINVAL, "ac_build: NULL keyword pointer");
        offs[size_t(i) + 1] = offs[size_t(i)] + lengths[i];
    }
    std::vector<uint8_t> flat;
    try {
        flat.resize(size_t(offs.back()));
    } catch (const std::bad_alloc &) {
        return fail(AC_ENOMEM, "ac_build: out of host memory");
    }
    for (int32_t i = 0; i < n_patterns; ++i)
        std::memcpy(flat.data() + offs[size_t(i)], patterns[i], size_t(lengths[i]));
    return build_common(flat.data(), offs.data(), n_patterns, opts, out);
}

void ac_free(ac_automaton *a) {
    if (!a) return;
    if (a->dmem) (void)hipFree(a->dmem);
    delete a;
}

int ac_info(const ac_automaton *a, ac_info_t *out) {
    if (!a || !out) return fail(AC_EINVAL, "ac_info: NULL argument");
    fill_info(a->host, out);
    out->device_bytes = a->dbytes;
    return AC_OK;
}

int ac_default_launch(const ac_automaton *a, int64_t len, ac_launch *out) {
    if (!a || !out) return fail(AC_EINVAL, "ac_default_launch: NULL argument");
    ScanArgs S{};
    S.n = len;
    *out = resolved(a, S, nullptr, false);
    return AC_OK;
}

int64_t ac_match_ex(const ac_automaton *a, const uint8_t *d_text, int64_t len, const ac_matches *matches,
                    const ac_launch *launch, hipStream_t stream) {
    int rc = check_single(a, d_text, len, matches);
    if (rc) return rc;
    if ((rc = check_launch(launch))) return rc;
    return sync_count(a, single_args(d_text, len, matches), launch, false, stream);
}

int ac_tune(ac_automaton *a, const uint8_t *d_text, int64_t len, hipStream_t stream, ac_launch *out) {
    int rc = check_single(a, d_text, len, nullptr);
    if (rc) return rc;
    if (len <= 0) return fail(AC_EINVAL, "ac_tune: empty sample");
    return tune(a, single_args(d_text, len, nullptr), false, stream, out);
}

int ac_tune_batch(ac_automaton *a, const uint8_t *d_texts, const int64_t *d_text_offsets, int32_t n_texts,
                  int64_t total_bytes, hipStream_t stream, ac_launch *out) {
    int rc = check_batch(a, d_texts, d_text_offsets, n_texts, total_bytes, nullptr);
    if (rc) return rc;
    if (n_texts <= 0 || total_bytes <= 0) return fail(AC_EINVAL, "ac_tune_batch: empty sample");
    return tune(a, batch_args(d_texts, d_text_offsets, n_texts, total_bytes, nullptr), true, stream, out);
}

int64_t ac_match(const ac_automaton *a, const uint8_t *d_text, int64_t len, const ac_matches *matches,
                 hipStream_t stream) {
    return ac_match_ex(a, d_text, len, matches, nullptr, stream);
}

int ac_match_async(const ac_automaton *a, const uint8_t *d_text, int64_t len, const ac_matches *matches,
                   const ac_launch *launch, int64_t *d_count, hipStream_t stream) {
    int rc = check_single(a, d_text, len, matches);
    if (rc) return rc;
    if ((rc = check_launch(launch))) return rc;
    if (!d_count) return fail(AC_EINVAL, "ac_match_async: NULL count pointer");
    const ScanArgs S = single_args(d_text, len, matches);
    const ac_launch cfg = resolved(a, S, launch, false);
    CountSlot *slot = nullptr;
    if ((rc = slot_for(a, stream, &slot))) return rc;
    return enqueue(a, S, cfg, false, true, reinterpret_cast<unsigned long long *>(d_count), slot->hs, stream);
}

int64_t ac_match_batch(const ac_automaton *a, const uint8_t *d_texts, const int64_t *d_text_offsets,
                       int32_t n_texts, int64_t total_bytes, const ac_batch_matches *matches,
                       const ac_launch *launch, hipStream_t stream) {
    int rc = check_batch(a, d_texts, d_text_offsets, n_texts, total_bytes, matches);
    if (rc) return rc;
    if ((rc = check_launch(launch))) return rc;
    return sync_count(a, batch_args(d_texts, d_text_offsets, n_texts, total_bytes, matches), launch, true,
                      stream);
}

int ac_match_batch_async(const ac_automaton *a, const uint8_t *d_texts, const int64_t *d_text_offsets,
                         int32_t n_texts, int64_t total_bytes, const ac_batch_matches *matches,
                         const ac_launch *launch, int64_t *d_count, hipStream_t stream) {
    int rc = check_batch(a, d_texts, d_text_offsets, n_texts, total_bytes, matches);
    if (rc) return rc;
    if ((rc = check_launch(launch))) return rc;
    if (!d_count) return fail(AC_EINVAL, "ac_match_batch_async: NULL count pointer");
    if (launch && launch->policy == AC_POLICY_DIRECT) return fail(AC_ENOTSUP, "batches use the filtered policy");
    const ScanArgs S = batch_args(d_texts, d_text_offsets, n_texts, total_bytes, matches);
    const ac_launch cfg = resolved(a, S, launch, true);
    CountSlot *slot = nullptr;
    if ((rc = slot_for(a, stream, &slot))) return rc;
    return enqueue(a, S, cfg, true, true, reinterpret_cast<unsigned long long *>(d_count), slot->hs, stream);
}

// ---- CPU matcher and CPU/GPU dispatch ------------------------------------------
int64_t ac_match_host(const ac_automaton *a, const uint8_t *text, int64_t len, int64_t *offset,
                      int32_t *pattern_id, int64_t capacity, int32_t n_threads) {
    int rc = check_host(a, text, len, offset, pattern_id, capacity, "ac_match_host");
    if (rc) return rc;
    return host_match_checked(a->host, text, len, offset, pattern_id, capacity, n_threads);
}

int64_t ac_plan_match_host(const ac_plan *p, const uint8_t *text, int64_t len, int64_t *offset,
                           int32_t *pattern_id, int64_t capacity, int32_t n_threads) {
    int rc = check_host(p, text, len, offset, pattern_id, capacity, "ac_plan_match_host");
    if (rc) return rc;
    return host_match_checked(p->p, text, len, offset, pattern_id, capacity, n_threads);
}

int64_t ac_match_dispatch(const ac_automaton *a, const uint8_t *text, int64_t len, int64_t *offset,
                          int32_t *pattern_id, int64_t capacity, hipStream_t stream, int32_t *ran_on) {
    int rc = check_host(a, text, len, offset, pattern_id, capacity, "ac_match_dispatch");
    if (rc) return rc;
    if (len < a->dispatch_bytes.load(std::memory_order_relaxed)) {
        if (ran_on) *ran_on = AC_RAN_CPU;
        return host_match_checked(a->host, text, len, offset, pattern_id, capacity, 0);
    }
    if ((rc = device_matches(a))) return rc;
    if (ran_on) *ran_on = AC_RAN_GPU;
    return gpu_round_trip(a, text, len, offset, pattern_id, capacity, stream);
}

int ac_set_dispatch_threshold(ac_automaton *a, int64_t bytes) {
    if (!a) return fail(AC_EINVAL, "ac_set_dispatch_threshold: NULL automaton");
    a->dispatch_bytes.store(bytes < 0 ? kDefaultDispatchBytes : bytes, std::memory_order_relaxed);
    return AC_OK;
}

int64_t ac_dispatch_threshold(const ac_automaton *a) {
    if (!a) return fail(AC_EINVAL, "ac_dispatch_threshold: NULL automaton");
    return a->dispatch_bytes.load(std::memory_order_relaxed);
}

int ac_calibrate_dispatch(ac_automaton *a, const uint8_t *sample, int64_t len, hipStream_t stream,
                          int64_t *threshold) {
    int rc = check_host(a, sample, len, nullptr, nullptr, 0, "ac_calibrate_dispatch");
    if (rc) return rc;
    if (len < 512) return fail(AC_EINVAL, "ac_calibrate_dispatch: sample shorter than 512 bytes");
    if ((rc = device_matches(a))) return rc;
    // prefixes of 512 B x 2^k: medians of 7 runs each way (after one warm-up)
    const int64_t top = std::min<int64_t>(len, int64_t(64) << 20);
    std::vector<int64_t> off;
    std::vector<int32_t> pid;
    auto median_ms = [&](auto &&run) -> double {
        std::vector<double> t;
        for (int r = 0; r < 8; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            const int64_t c = run();
            const auto t1 = std::chrono::steady_clock::now();
            if (c < 0) return -1.0;
            if (r) t.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        std::sort(t.begin(), t.end());
        return t[t.size() / 2];
    };
    int64_t found = -1;
    for (int64_t n = 512; n <= top; n *= 2) {
        const int64_t cap = a->host.n_patterns > 0 ? n * 4 + 64 : 64;
        off.resize(size_t(cap));
        pid.resize(size_t(cap));
        const double cpu = median_ms([&] { return host_match_checked(a->host, sample, n, off.data(), pid.data(), cap, 0); });
        const double gpu = median_ms([&] { return gpu_round_trip(a, sample, n, off.data(), pid.data(), cap, stream); });
        if (cpu < 0 || gpu < 0) return AC_EHIP;
        if (gpu < cpu) {
            found = n;
            break;
        }
        if (n > top / 2) break;
    }
    // the GPU never won within the sample: everything up to it stays on the CPU
    if (found < 0) found = top * 2;
    a->dispatch_bytes.store(found, std::memory_order_relaxed);
    if (threshold) *threshold = found;
    return AC_OK;
}

// ---- host-side inspection -----------------------------------------------------
int ac_compile(const uint8_t *bytes, const int64_t *offsets, int32_t n_patterns, const ac_build_opts *opts,
               ac_plan **out) {
    if (!out) return fail(AC_EINVAL, "ac_compile: NULL output pointer");
    *out = nullptr;
    ac_plan *p = new (std::nothrow) ac_plan();
    if (!p) return fail(AC_ENOMEM, "ac_compile: out of host memory");
    std::string err;
    int rc;
    try {
        rc = compile_plan(bytes, offsets, n_patterns, opts, p->p, err);
    } catch (const std::bad_alloc &) {
        rc = AC_ENOMEM;
        err = "ac_compile: out of host memory";
    }
    if (rc) { delete p; return fail(rc, err); }
    *out = p;
    return AC_OK;
}

int ac_plan_info(const ac_plan *p, ac_info_t *out) {
    if (!p || !out) return fail(AC_EINVAL, "ac_plan_info: NULL argument");
    fill_info(p->p, out);
    return AC_OK;
}

int64_t ac_plan_export(const ac_plan *p, int32_t table, void *dst, int64_t dst_bytes) {
    if (!p) return fail(AC_EINVAL, "ac_plan_export: NULL plan");
    const Plan &P = p->p;
    const void *src = nullptr;
    int64_t bytes = 0;
    switch (table) {
        case AC_TABLE_CLASS_MAP: src = P.cls; bytes = 256; break;
        case AC_TABLE_DENSE: src = P.dense.data(); bytes = int64_t(P.dense.size()) * 4; break;
        case AC_TABLE_NODE: src = P.node.data(); bytes = int64_t(P.node.size()) * 4; break;
        case AC_TABLE_LABEL: src = P.label.data(); bytes = int64_t(P.label.size()); break;
        case AC_TABLE_OUT_OFF: src = P.out_off.data(); bytes = int64_t(P.out_off.size()) * 4; break;
        case AC_TABLE_OUT_PID: src = P.out_pid.data(); bytes = int64_t(P.out_pid.size()) * 4; break;
        case AC_TABLE_DEPTH: src = P.depth.data(); bytes = int64_t(P.depth.size()) * 4; break;
        case AC_TABLE_PREFIX: src = P.ptab.data(); bytes = int64_t(P.ptab.size()) * 4; break;
        case AC_TABLE_TAIL: src = P.tail.data(); bytes = int64_t(P.tail.size()) * 4; break;
        case AC_TABLE_TAIL_INFO: src = P.tailinfo.data(); bytes = int64_t(P.tailinfo.size()) * 4; break;
        default:
            if (table > AC_TABLE_FILTER_BASE && table <= AC_TABLE_FILTER_BASE + kNumFilters) {
                const auto &f = P.filter[table - AC_TABLE_FILTER_BASE - 1];
                src = f.data();
                bytes = int64_t(f.size());
                break;
            }
            return fail(AC_EINVAL, "ac_plan_export: unknown table");
    }
    if (!dst) return bytes;
    if (dst_bytes < bytes) return fail(AC_EINVAL, "ac_plan_export: destination too small");
    if (bytes) std::memcpy(dst, src, size_t(bytes));
    return bytes;
}

uint32_t ac_plan_hash(const ac_plan *p, uint32_t x) {
    if (!p) return 0;
    const uint32_t kmask = p->p.K >= 3 ? 0xFFFFFFu : ((1u << (8 * p->p.K)) - 1u);
    return prefix_hash(x & kmask, p->p.hash_mul);
}

uint32_t ac_plan_hash2(const ac_plan *p, uint32_t x) {
    if (!p) return 0;
    const uint32_t kmask = p->p.K >= 3 ? 0xFFFFFFu : ((1u << (8 * p->p.K)) - 1u);
    return prefix_hash(x & kmask, kFilterMul2);
}

void ac_plan_prefix_buckets(const ac_plan *p, uint32_t x, uint32_t *b1, uint32_t *b2) {
    if (!p || !b1 || !b2) return;
    prefix_buckets(x & 0xFFFFFFu, p->p.hash_mul, p->p.ptab_bits, *b1, *b2);
}

void ac_plan_free(ac_plan *p) { delete p; }

}  // extern "C"
