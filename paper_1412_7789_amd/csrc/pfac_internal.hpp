// Internal structures shared by the host builder, the launch code and the
// HIP kernels of the failure-less Aho-Corasick matcher.
#pragma once

#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "pfac.h"

namespace pfac {

constexpr int kWave = 64;
constexpr int kSegBytes = 1024;          // bytes one wave loads per segment (64 lanes x 16 B)
constexpr int kMaxPrefix = 3;            // bytes hashed by the candidate filter
constexpr uint32_t kDefaultHashMul = 0x9E3779u;   // odd 24-bit multiplier
constexpr uint32_t kPrefixMul2 = 0x5BD1E5u;       // second bucket of the prefix table
constexpr int64_t kDefaultDenseBudget = 64ll << 20;
constexpr int32_t kFinalBit = int32_t(0x80000000u);
// ac_match_dispatch's CPU/GPU crossover before ac_calibrate_dispatch or
// ac_set_dispatch_threshold sets one (measured on MI355X with its host CPU:
// 1000 printable keywords, text in pinned host memory)
constexpr int64_t kDefaultDispatchBytes = int64_t(8) << 10;

// Filter geometry: index bits taken from the top of the 32-bit product.
struct FilterGeom {
    int kind;        // AC_FILTER_*
    bool bitmap;     // false: one byte per entry; true: one bit per entry
    int index_bits;  // log2(entries) of one map
    int shift;       // product >> shift gives the byte (byte map) or word (bit map) index
    int64_t bytes;   // LDS bytes
    bool dual;       // two bit maps with independent hashes, both must be set
    bool pair;       // two bits per key in one word (4-byte keys), both must be set
};

inline FilterGeom filter_geom(int kind) {
    switch (kind) {
        case AC_FILTER_BYTES17: return {kind, false, 17, 32 - 17, 1ll << 17, false, false};
        case AC_FILTER_BITS20:  return {kind, true, 20, 32 - 15, 1ll << 17, false, false};
        case AC_FILTER_BYTES16: return {kind, false, 16, 32 - 16, 1ll << 16, false, false};
        case AC_FILTER_BITS19:  return {kind, true, 19, 32 - 14, 1ll << 16, false, false};
        case AC_FILTER_DUAL19:  return {kind, true, 19, 32 - 14, 1ll << 17, true, false};
        case AC_FILTER_PAIR20:  return {kind, true, 20, 32 - 15, 1ll << 17, false, true};
        default: return {0, false, 0, 0, 0, false, false};
    }
}
constexpr int kNumFilterKinds = 6;
constexpr uint32_t kFilterMul2 = 0x7FEB35u;       // hash of the second map of AC_FILTER_DUAL19
// Filter sets, kNumFilterKinds maps each: stride 1 tests every offset against
// the keywords' K-byte prefixes; stride 2 tests the windows starting at every
// second offset against the 3-byte windows at keyword positions 1 and 2
// (built when K = 3 and every keyword has >= 5 bytes); stride 4 every fourth
// one against positions 1 .. 4 (keywords of >= 7 bytes).  The
// AC_FILTER_PAIR20 map of strides 2 and 4 holds the 4-byte windows at those
// positions instead (keywords of >= 6 and >= 8 bytes); it is empty at stride 1.
constexpr int kNumFilters = 3 * kNumFilterKinds;   // strides 1, 2 and 4
// Filter set of a sampling stride: 0 (stride 1), 1 (stride 2), 2 (stride 4).
constexpr int stride_set(int stride) { return stride == 4 ? 2 : stride - 1; }

// Host-side build result (the "plan").  States are numbered breadth first,
// so the children of a state are contiguous and sorted by byte, and every
// state of depth <= dense_depth precedes every deeper state.
struct Plan {
    int32_t n_patterns = 0;
    std::vector<int64_t> kw_len;
    int32_t S = 0;                 // states, root = 0
    int32_t C = 0;                 // classes
    uint8_t cls[256] = {};
    int32_t min_len = 0, max_len = 0, K = 0;
    std::vector<int32_t> depth, first_child, n_child;
    std::vector<uint8_t> label;
    std::vector<int32_t> out_off, out_pid;
    int32_t S_dense = 0, dense_depth = 0;
    std::vector<int32_t> dense;    // [S_dense * C]
    std::vector<int32_t> node;     // [2 * (S - S_dense)]
    uint32_t hash_mul = kDefaultHashMul;
    int32_t n_prefixes = 0;
    int32_t n_windows2 = 0;        // distinct 3-byte windows at keyword positions 1 and 2
    bool sampled = false;          // the stride-2 filters exist
    int32_t n_windows4 = 0;        // distinct 3-byte windows at keyword positions 1 .. 4
    bool sampled4 = false;         // the stride-4 filters exist
    int32_t n_quads4 = 0;          // distinct 4-byte windows at keyword positions 1 .. 4
    bool pair4 = false;            // the stride-4 AC_FILTER_PAIR20 map exists
    int32_t n_quads2 = 0;          // distinct 4-byte windows at keyword positions 1 and 2
    bool pair2 = false;            // the stride-2 AC_FILTER_PAIR20 map exists
    std::vector<uint8_t> filter[kNumFilters];   // indexed by stride_set(stride) * kNumFilterKinds + kind - 1
    int32_t ptab_bits = 0;
    std::vector<uint32_t> ptab;    // [2 << ptab_bits]: buckets of 4 {key, value} slots
    std::vector<int32_t> tail;     // [S]: leaf of a forced path, or -1
    std::vector<int32_t> tailinfo; // [4 S]: {leaf or -1, kw_bytes position, remaining bytes, 0}
    std::vector<uint8_t> kw_bytes; // keywords back to back
    std::vector<int32_t> kw_off;   // [n + 1]
    double build_ms = 0.0;
};

// Kernel-side view of a device automaton (passed by value).  It holds only
// what the walks read: every field is a kernel argument kept in scalar
// registers, so the filter maps (one of which a launch stages in LDS) travel
// in the launch's own arguments instead.
struct DevAut {
    const uint8_t *cls;
    const int32_t *dense;
    const int32_t *node;
    const uint8_t *label;
    const int32_t *out_off;
    const int32_t *out_pid;
    const uint32_t *ptab;          // exact prefix table (global copy)
    const int4 *tailinfo;
    const uint8_t *kw_bytes;
    int32_t C, S_dense, K;
    int32_t ptab_bits;
    uint32_t hash_mul;
};

// Arguments of one scan launch.
struct ScanArgs {
    const uint8_t *text;           // first byte of the (packed) text
    int64_t n;                     // bytes
    const int64_t *text_off;       // batch: device int64[n_texts + 1]; nullptr = single text
    int32_t n_texts;
    int64_t *out_off;              // match offsets (relative to its text)
    int32_t *out_pid;
    int32_t *out_tid;              // batch only
    int64_t cap;                   // 0 = count only
    unsigned long long *count;
    unsigned long long count_base; // value of *count before this scan: match i goes to index i - base
    int64_t *per_text;             // batch only, may be null
    // Optional report of the count to the host: the streaming kernel's last
    // block to finish (*done reaching done_base + blocks) stores *count into
    // host_count[0], a pinned host word, and then host_seq into host_count[1],
    // so the host can wait for the word instead of the stream.
    // host_count == nullptr: no report.
    unsigned long long *done;
    unsigned long long done_base;
    unsigned long long *host_count;
    unsigned long long host_seq;
};

}  // namespace pfac

struct ac_plan {
    pfac::Plan p;
};

struct ac_automaton {
    pfac::Plan host;               // tables kept for ac_info and launch decisions
    int device = 0;
    void *dmem = nullptr;          // one device allocation for every table
    int64_t dbytes = 0;
    pfac::DevAut dev{};
    const uint8_t *dfilter[pfac::kNumFilters] = {};   // device filter maps, by stride_set * kinds + kind - 1
    int cu_count = 0;
    int64_t lds_per_block = 0;
    int64_t lds_per_cu = 0;
    // launch choices measured by ac_tune, by text-length bucket (floor(log4 len))
    mutable std::mutex tune_mu;
    std::map<int, ac_launch> tuned;
    std::map<int, ac_launch> tuned_batch;  // the same for batches, by total length
    // texts shorter than this go to the CPU matcher in ac_match_dispatch
    std::atomic<int64_t> dispatch_bytes{pfac::kDefaultDispatchBytes};
};

namespace pfac {
// plan.cpp
int compile_plan(const uint8_t *bytes, const int64_t *offsets, int32_t n,
                 const ac_build_opts *opts, Plan &out, std::string &err);
uint32_t prefix_hash(uint32_t x, uint32_t mul);
// The two candidate buckets (of 4 slots) of prefix x in a table of 2^bits slots.
void prefix_buckets(uint32_t x, uint32_t mul, int bits, uint32_t &b1, uint32_t &b2);
// Per-stream scratch of the filtered policy: one hit region per streaming
// wave of the widest launch.
struct HitScratch {
    uint4 *hits = nullptr;         // [regions * cap]
    int64_t regions = 0;
    int32_t cap = 0;
};
constexpr int32_t kHitCap = 1024;

// host_match.cpp: every (offset, keyword id) of text[0, n) found on host
// threads (n_threads <= 0: chosen by length); writes up to cap of them and
// returns how many there are.
int64_t host_match(const Plan &P, const uint8_t *text, int64_t n, int64_t *off, int32_t *pid, int64_t cap,
                   int32_t n_threads);

// kernels.hip
int64_t scan_regions(const ac_automaton *a, const uint8_t *text, int64_t n, const ac_launch &cfg);
// Hit regions of the widest filtered launch on a device.
int64_t widest_scan_regions(int cu_count, int64_t lds_per_cu);
// Start/stop events of the scan kernel (the filtered policy's streaming
// kernel or the direct kernel), taken from its own dispatch packet so that
// they time the kernel alone; null = untimed.
struct KernelTiming {
    hipEvent_t scan0 = nullptr, scan1 = nullptr;
};
// *blocks (if given) receives the number of blocks of the scan kernel (0
// when nothing was launched).
int launch_scan(const ac_automaton *a, const ScanArgs &args, const ac_launch &cfg, const HitScratch &hs,
                hipStream_t stream, std::string &err, const KernelTiming *timing = nullptr,
                int64_t *blocks = nullptr);
int launch_zero(unsigned long long *count, unsigned long long *done, int64_t *per_text, int32_t n_texts,
                hipStream_t stream, std::string &err);
void resolve_launch(const ac_automaton *a, int64_t len, bool batch, ac_launch &cfg);

// Sets the calling thread's ac_last_error() message; returns `code`.
int report_error(int code, const std::string &msg);

// Creates the (current device, stream) scratch now, so that later scans on
// the stream allocate nothing; *device_bytes (if given) receives its device
// memory in bytes.
int reserve_stream_scratch(hipStream_t stream, int64_t *device_bytes = nullptr);
// Frees the (current device, stream) scratch; the stream must be idle and is
// about to be destroyed.
void release_stream_scratch(hipStream_t stream);
int launch_probe_read(const uint8_t *buf, int64_t n, uint32_t *out, hipStream_t stream, std::string &err);
}  // namespace pfac
