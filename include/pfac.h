/*
 * pfac.h -- C ABI of the MI355X (gfx950) failure-less Aho-Corasick matcher.
 *
 * Problem (paper, Section II): locate all occurrences of any of a finite set
 * of keywords in a text.  The matcher uses the failure-less parallel form of
 * Aho-Corasick that the paper evaluates on the GPU (Section II, Fig. 3 "N" and
 * Fig. 5): every byte offset of the text starts its own walk of the Goto trie
 * from the root, the walk stops at the first missing transition, and every
 * keyword equal to T[o .. j] for a state passed by the walk from o is reported
 * at offset o.  Unlike the PFAC variant the paper describes, keywords nested in
 * longer ones ("sub patterns", Section II) are all reported, so the result is
 *
 *     R = { (o, p) : T[o .. o + |k_p|) == k_p },
 *
 * an unordered set of (start offset, keyword id) pairs.  Keyword ids are the
 * input indices 0 .. n-1.  Bytes are raw unsigned 0..255, compared exactly.
 *
 * Memory: the library owns automata (device memory, freed by ac_free).  The
 * caller owns every text and match buffer passed in; those are DEVICE
 * pointers (e.g. torch tensors on the GPU).  Every function returning int or
 * int64_t returns a negative AC_E* code on error and records a message for
 * ac_last_error() in the calling thread.
 *
 * Streams: every GPU call is stream-ordered on the hipStream_t passed in
 * (0 = the null stream).  Calls on different streams may run concurrently; an
 * automaton is read-only after ac_build.  Two host threads must not drive the
 * same stream at once.
 */
#ifndef PFAC_H
#define PFAC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define AC_OK        0
#define AC_EINVAL   (-1)  /* bad argument: empty keyword, n <= 0, NULL pointer  */
#define AC_ENOMEM   (-2)  /* host or device allocation failed                   */
#define AC_EHIP     (-3)  /* a HIP runtime call failed                          */
#define AC_ENOTSUP  (-4)  /* option combination not supported                   */

typedef struct ac_automaton ac_automaton;   /* device automaton, immutable     */
typedef struct ac_plan ac_plan;             /* host-side build result          */

/* ---- build ---------------------------------------------------------------- */
typedef struct {
    /* Upper bound on the bytes of dense transition rows.  States are numbered
     * breadth first; the shallowest states whose rows fit get dense int32
     * rows, deeper ones a compact child-list layout.  0 = 64 MiB. */
    int64_t dense_budget_bytes;
    /* 24-bit odd multiplier of the prefix hash used by the candidate filter;
     * 0 = default.  Any value gives the same matches. */
    uint32_t hash_multiplier;
    int32_t reserved[7];
} ac_build_opts;

/*
 * Build an automaton from n_patterns keywords (host memory: patterns[i] points
 * at lengths[i] bytes).  Steps (paper Section II, Fig. 5): Goto trie over the
 * keywords, breadth-first state numbering, Output lists (keyword ids per
 * state), alphabet compression (byte -> class, unused bytes -> a dead class),
 * dense/compact transition layout, candidate filter over each keyword's first
 * min(3, shortest keyword) bytes, then one upload to the current device.
 * Errors: AC_EINVAL (n_patterns <= 0, NULL pointer, empty keyword),
 * AC_ENOMEM, AC_EHIP.  On success *out owns device memory until ac_free.
 */
int ac_build(const uint8_t *const *patterns, const int64_t *lengths, int32_t n_patterns,
             const ac_build_opts *opts, ac_automaton **out);

/* Same, with keywords packed as bytes[offsets[i] .. offsets[i+1]) (host). */
int ac_build_csr(const uint8_t *bytes, const int64_t *offsets, int32_t n_patterns,
                 const ac_build_opts *opts, ac_automaton **out);

void ac_free(ac_automaton *a);

/* ---- match ---------------------------------------------------------------- */
typedef struct {
    int64_t *offset;      /* device [capacity]: start offset of each match     */
    int32_t *pattern_id;  /* device [capacity]: keyword id of each match       */
    int64_t capacity;     /* entries available in both arrays                  */
} ac_matches;

/* Kernel choice; zero-initialise for the library's defaults. */
#define AC_POLICY_AUTO      0
#define AC_POLICY_FILTERED  1  /* prefix-filter every offset, walk candidates   */
#define AC_POLICY_DIRECT    2  /* walk every offset from the root (plain PFAC)  */

#define AC_FILTER_AUTO      0
#define AC_FILTER_BYTES17   1  /* 2^17-entry byte map, 128 KiB of LDS           */
#define AC_FILTER_BITS20    2  /* 2^20-bit map, 128 KiB of LDS                  */
#define AC_FILTER_BYTES16   3  /* 2^16-entry byte map, 64 KiB of LDS            */
#define AC_FILTER_BITS19    4  /* 2^19-bit map, 64 KiB of LDS                   */
#define AC_FILTER_DUAL19    5  /* two 2^19-bit maps with independent hashes,   */
                               /* 128 KiB of LDS; both bits must be set         */
#define AC_FILTER_PAIR20    6  /* strides 2 and 4: a 2^20-bit map (128 KiB of   */
                               /* LDS) keyed by the keywords' 4-byte windows at */
                               /* positions 1 .. stride, two bits per key in    */
                               /* one word (three at stride 2): all must be     */
                               /* set; needs every keyword >= stride + 4 bytes  */

typedef struct {
    int32_t policy;         /* AC_POLICY_*                                        */
    int32_t filter;         /* AC_FILTER_* (FILTERED policy)                      */
    int32_t block;          /* threads per block: 256, 512 or 1024; 0 = auto     */
    int32_t segs;           /* 1 KiB segments per wave step: 1, 2 or 4; 0 = auto */
    int32_t grid_per_cu;    /* resident blocks per compute unit; 0 = auto        */
    int32_t table_in_lds;   /* DIRECT: -1/0 = auto, 1 = force LDS, 2 = global     */
    int32_t flags;          /* AC_LAUNCH_* bits                                   */
    int32_t stride;         /* FILTERED: 1 = test every offset's prefix; 2 = test
                             * the 3-byte windows starting at every second offset
                             * against the keywords' windows at positions 1 and 2
                             * (needs every keyword >= 5 bytes), a positive test at
                             * s making s - 2 and s - 1 candidates; 4 = every
                             * fourth window against the windows at positions
                             * 1 .. 4 (keywords >= 7 bytes), a positive at s making
                             * s - 4 .. s - 1 candidates; 0 = auto               */
    int32_t reserved[4];
} ac_launch;

/* Time the scan's kernels with HIP events taken from their own dispatch
 * packets (start and end of each kernel, no launch gaps); a synchronous call
 * then leaves the durations for ac_last_scan_ms() / ac_last_scan_split() in
 * the calling thread. */
#define AC_LAUNCH_TIME_SCAN 1

/*
 * The scan (Section II's problem; the parallel "N" side of Fig. 3, one walk of
 * the Fig. 5 trie per offset): every occurrence in d_text[0 .. len) (device).
 * Writes up to
 * matches->capacity (offset, pattern_id) pairs in unspecified order and
 * returns the TRUE number of matches |R| (>= 0), also when it exceeds the
 * capacity; then an unspecified subset of `capacity` matches is written and
 * the caller may retry with a larger buffer.  matches == NULL counts only.
 * len == 0 returns 0.  d_text may have any alignment.
 * The call is stream-ordered on `stream` and returns once the count is
 * final: the filtered scan's last block reports it to pinned host memory
 * after every match is written (the kernel may still be retiring; work
 * enqueued later on `stream` runs after it).  The direct policy synchronises
 * the stream instead.  The library keeps per-(device, stream) scratch (a
 * count word, a pinned host word and the filtered policy's hit regions,
 * 16 KiB for each wave of the widest launch the device allows: 64 MiB on a
 * 256-CU MI355X), allocated on the stream's first call and kept, unchanged,
 * until ac_release_stream or the end of the process; calls on one stream
 * must come from one thread at a time.  Errors: AC_EINVAL (NULL
 * automaton, NULL text with len > 0, len < 0, capacity < 0, NULL arrays with
 * capacity > 0), AC_ENOMEM, AC_EHIP.
 */
int64_t ac_match(const ac_automaton *a, const uint8_t *d_text, int64_t len,
                 const ac_matches *matches, hipStream_t stream);

/* ac_match with an explicit kernel choice (NULL = defaults). */
int64_t ac_match_ex(const ac_automaton *a, const uint8_t *d_text, int64_t len,
                    const ac_matches *matches, const ac_launch *launch, hipStream_t stream);

/*
 * Asynchronous form: enqueues the scan on `stream` and writes the match count
 * to d_count (device int64) without synchronising; returns AC_OK or an error.
 * It clears d_count with a kernel (no memset).  Only the first call on a
 * stream allocates (the stream's scratch, sized for any text); after one
 * call on the stream it may be captured in a HIP graph.  Replays of captured
 * scans that share a stream's scratch must not overlap.
 */
int ac_match_async(const ac_automaton *a, const uint8_t *d_text, int64_t len,
                   const ac_matches *matches, const ac_launch *launch,
                   int64_t *d_count, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * scan as ac_match_async, with the filtered policy's hit regions taken from a
 * fixed array in the library's device code instead of per-stream scratch.
 * The call makes no hipMalloc, hipFree or other allocating call, on any call,
 * including the first on a device (which only looks up the array's address
 * there).  The array holds 16 MiB per GPU for the life of the process: 256
 * records of 16 bytes for each of the 4096 waves of the widest launch on a
 * 256-CU MI355X; a launch whose waves would get fewer than 128 records each
 * is rejected with AC_EINVAL (a wave whose records run out finishes its
 * share walking hits as it finds them, which is slower, never wrong).  Every
 * call on one GPU uses that GPU's one array, so two such calls must not
 * overlap on a GPU (serialise them on one stream, or wait between them);
 * overlapping calls race on the array and their results are undefined.
 * Matches, count, launch choices and errors are those of ac_match_async.
 */
int ac_match_async_noalloc(const ac_automaton *a, const uint8_t *d_text, int64_t len,
                           const ac_matches *matches, const ac_launch *launch,
                           int64_t *d_count, hipStream_t stream);

/* ---- batches -------------------------------------------------------------- */
typedef struct {
    int32_t *text_id;         /* device [capacity]                              */
    int64_t *offset;          /* device [capacity]: offset within its text      */
    int32_t *pattern_id;      /* device [capacity]                              */
    int64_t capacity;
    int64_t *per_text_count;  /* device [n_texts] or NULL: matches per text     */
} ac_batch_matches;

/*
 * The scan of ac_match over many texts at once (each text is its own
 * instance of Section II's problem): n_texts texts packed back to back, text t is
 * d_texts[d_text_offsets[t] - d_text_offsets[0] .. d_text_offsets[t+1] - d_text_offsets[0])
 * where d_text_offsets (device int64[n_texts + 1], non-decreasing) is read by
 * the kernel.  A match never spans two texts.  One launch scans the whole
 * batch.  total_bytes must equal d_text_offsets[n_texts] - d_text_offsets[0]
 * (the host sizes the launch from it without reading device memory); launch
 * may be NULL (defaults, or the choice ac_tune_batch recorded).  Returns the
 * true total count as ac_match does; per_text_count, if given, receives exact
 * per-text counts (it is cleared by the call, with one small clearing kernel
 * before the scan; without it the call launches the scan kernel alone).
 * Errors: AC_EINVAL, AC_ENOTSUP (launch->policy == AC_POLICY_DIRECT), AC_EHIP.
 */
int64_t ac_match_batch(const ac_automaton *a, const uint8_t *d_texts,
                       const int64_t *d_text_offsets, int32_t n_texts, int64_t total_bytes,
                       const ac_batch_matches *matches, const ac_launch *launch,
                       hipStream_t stream);

/* Asynchronous, graph-capturable batch form (count to d_count, no sync). */
int ac_match_batch_async(const ac_automaton *a, const uint8_t *d_texts,
                         const int64_t *d_text_offsets, int32_t n_texts, int64_t total_bytes,
                         const ac_batch_matches *matches, const ac_launch *launch,
                         int64_t *d_count, hipStream_t stream);

/* ---- CPU matcher and CPU/GPU dispatch --------------------------------------- */
/*
 * The paper measures where a GPU starts to beat a serial CPU matcher on the
 * same input and concludes that an application should switch processing
 * units automatically around that size (Section IV, Fig. 6-8; Section V).
 *
 * ac_match_host: the same match set R as ac_match, computed on host threads
 * by the failure-less walk over the automaton's own tables (text, offset and
 * pattern_id are HOST memory).  n_threads <= 0 lets the library choose (one
 * thread below 1 MiB).  Returns |R| and writes up to `capacity` matches in
 * unspecified order, like ac_match.  Errors: AC_EINVAL, AC_ENOMEM.
 * ac_plan_match_host: the same on a host-only build (no GPU needed).
 */
int64_t ac_match_host(const ac_automaton *a, const uint8_t *text, int64_t len, int64_t *offset,
                      int32_t *pattern_id, int64_t capacity, int32_t n_threads);
int64_t ac_plan_match_host(const ac_plan *p, const uint8_t *text, int64_t len, int64_t *offset,
                           int32_t *pattern_id, int64_t capacity, int32_t n_threads);

#define AC_RAN_CPU 1
#define AC_RAN_GPU 2
/*
 * Host text in, host matches out, on whichever unit finishes first: texts
 * shorter than the automaton's dispatch threshold go to ac_match_host, the
 * others are copied to the device (per-stream staging, grown as needed),
 * scanned and their matches copied back, all on `stream`, which the call
 * synchronises.  *ran_on (may be NULL) receives AC_RAN_CPU or AC_RAN_GPU.
 * Returns |R| as ac_match does.  Errors: AC_EINVAL, AC_ENOMEM, AC_EHIP.
 */
int64_t ac_match_dispatch(const ac_automaton *a, const uint8_t *text, int64_t len, int64_t *offset,
                          int32_t *pattern_id, int64_t capacity, hipStream_t stream, int32_t *ran_on);
/* Sets the dispatch threshold in bytes (negative: the built-in 8 KiB). */
int ac_set_dispatch_threshold(ac_automaton *a, int64_t bytes);
int64_t ac_dispatch_threshold(const ac_automaton *a);
/*
 * Measures the crossover on prefixes of a host sample (512 B, 1 KiB, ...,
 * up to min(len, 64 MiB)): the median of 7 timed calls each way, the CPU
 * matcher against the GPU round trip of ac_match_dispatch, and sets the
 * threshold to the first size where the GPU is faster (twice the largest
 * size tried if it never is).  *threshold (may be NULL) receives it.
 * Synchronises `stream`.  Errors: AC_EINVAL (len < 512), AC_ENOMEM, AC_EHIP.
 */
int ac_calibrate_dispatch(ac_automaton *a, const uint8_t *sample, int64_t len, hipStream_t stream,
                          int64_t *threshold);

/* ---- introspection ---------------------------------------------------------- */
typedef struct {
    int32_t n_patterns;
    int32_t n_states;        /* trie states, root included                      */
    int32_t n_classes;       /* alphabet classes (dense row width)              */
    int32_t min_len, max_len;
    int32_t prefix_len;      /* bytes hashed by the candidate filter            */
    int32_t n_dense_states;  /* states [0, n_dense_states) have dense rows      */
    int32_t dense_depth;     /* every state of depth <= dense_depth is dense    */
    int32_t n_prefixes;      /* distinct keyword prefixes of prefix_len bytes   */
    int32_t n_windows2;      /* distinct 3-byte windows at positions 1 and 2 (0 = stride 2 unavailable) */
    int64_t dense_bytes, compact_bytes, output_bytes, filter_bytes, device_bytes;
    double build_ms;         /* host build + upload time                        */
    int64_t prefix_table_bytes;  /* exact prefix -> state table                 */
    int64_t tail_bytes;      /* forced-path leaves + keyword bytes               */
    int32_t n_windows4;      /* distinct 3-byte windows at positions 1 .. 4 (0 = stride 4 unavailable) */
    int32_t n_quads4;        /* distinct 4-byte windows at positions 1 .. 4 (0 = no stride-4 AC_FILTER_PAIR20) */
    int32_t n_quads2;        /* distinct 4-byte windows at positions 1 and 2 (0 = no stride-2 AC_FILTER_PAIR20) */
    int32_t reserved[1];
} ac_info_t;

int ac_info(const ac_automaton *a, ac_info_t *out);

/* Kernel choice the library makes for a text of `len` bytes by default
 * (a choice recorded by ac_tune for that length, else the built-in rule). */
int ac_default_launch(const ac_automaton *a, int64_t len, ac_launch *out);

/*
 * Autotuner: times every choice of the filtered policy (sampling stride,
 * filter map, segments per chunk) on d_text[0 .. len) (device; a sample of
 * the texts to come), three runs each, and records the fastest for texts of
 * similar length (the same floor(log4 len)).  Later single-text calls whose
 * launch is NULL or leaves every choice at 0 use it.  *out (may be NULL)
 * receives the choice.  Synchronises `stream`; every choice computes the same
 * matches.  Errors: AC_EINVAL (NULL automaton or text, len <= 0), AC_EHIP.
 */
int ac_tune(ac_automaton *a, const uint8_t *d_text, int64_t len, hipStream_t stream, ac_launch *out);

/* The same for batches: times every choice on one batch (arguments as in
 * ac_match_batch) and records the fastest for batches of a similar total
 * length, which later ac_match_batch / ac_match_batch_async calls with a
 * NULL or all-zero launch use.  Errors: AC_EINVAL (empty batch), AC_EHIP. */
int ac_tune_batch(ac_automaton *a, const uint8_t *d_texts, const int64_t *d_text_offsets, int32_t n_texts,
                  int64_t total_bytes, hipStream_t stream, ac_launch *out);

const char *ac_last_error(void);

/* Scan-kernel milliseconds of this thread's last synchronous call made with
 * AC_LAUNCH_TIME_SCAN (negative if none or if the text was empty): from the
 * start of the first scan kernel to the end of the last one. */
float ac_last_scan_ms(void);

/* The same call's split: *stream_ms = the scan kernel (the filtered
 * policy's streaming kernel, which also walks the candidate offsets it keeps,
 * or the direct kernel), *walk_ms = time in separate walk kernels (0: the
 * walks run inside the scan kernel); both negative if no timed call was made. */
void ac_last_scan_split(float *stream_ms, float *walk_ms);

/*
 * Frees the scratch the library keeps for `stream` on the current device
 * (count words, the pinned host word, hit regions and ac_match_dispatch's
 * staging), for a caller about to destroy the stream.  The stream must be
 * idle (no scan of this library still queued on it) and no other thread may
 * be calling the library on it.  A later call on the stream allocates the
 * scratch again.  Returns AC_OK (also when the stream had none) or AC_EHIP.
 */
int ac_release_stream(hipStream_t stream);

/* ---- measurement probe -------------------------------------------------------- */
/*
 * Reads d_buf[0 .. n) (device, 16-byte aligned, n a multiple of 16) once with
 * coalesced 16-byte loads and folds it into *d_out (device uint32), so that
 * the achievable HBM read bandwidth can be timed beside the scan.  Async on
 * `stream`.  Errors: AC_EINVAL (misaligned or NULL), AC_EHIP.
 */
int ac_probe_read(const uint8_t *d_buf, int64_t n, uint32_t *d_out, hipStream_t stream);

/* ---- host-side build, for inspection (no GPU needed) ------------------------ */
/*
 * ac_compile runs every host step of ac_build (trie, numbering, outputs,
 * classes, layouts, filters) without touching a GPU.  ac_plan_info fills the
 * same fields as ac_info (device_bytes = bytes ac_build would upload).
 * ac_plan_export copies one table into host memory `dst` of `dst_bytes`
 * and returns the bytes the table needs (call with dst = NULL to size it):
 *   AC_TABLE_CLASS_MAP  uint8[256]         byte -> class
 *   AC_TABLE_DENSE      int32[n_dense*C]   next state | final bit 31, 0 = dead
 *   AC_TABLE_NODE       int32[2*(S-n_dense)] first child, child count | final bit 31
 *   AC_TABLE_LABEL      uint8[S]           byte on the edge into each state
 *   AC_TABLE_OUT_OFF    int32[S+1]         CSR offsets into AC_TABLE_OUT_PID
 *   AC_TABLE_OUT_PID    int32[...]         keyword ids ending at each state
 *   AC_TABLE_DEPTH      int32[S]           trie depth of each state
 *   AC_TABLE_PREFIX     uint32[2*slots]    buckets of 4 {key, value} slots: key = prefix |
 *                                          next byte << 24, value = state | has-next 1<<30 |
 *                                          final 1<<31 (0 = empty slot); a prefix lies in
 *                                          one of the two buckets ac_plan_prefix_buckets gives
 *   AC_TABLE_TAIL       int32[S]           leaf reached by a forced path, or -1
 *   AC_TABLE_TAIL_INFO  int32[4*S]         per state, one walk step's record: {leaf,
 *                                          keyword-byte position of the first byte below
 *                                          the state, bytes to the leaf, the leaf's only
 *                                          keyword id + 1 or 0} for a forced path;
 *                                          {-3, keyword-byte position, bytes to c, c} when
 *                                          a unary chain of 2+ bytes with no keyword
 *                                          ending inside leads to a state c that ends a
 *                                          keyword or branches; {-2, 0, 0, 0} at a leaf;
 *                                          {-1, first child, child count, 0} otherwise;
 *                                          bit 31 of the last field set when a keyword
 *                                          ends at the state
 *   AC_TABLE_FILTER_BASE + k   filter map of kind k = AC_FILTER_* (stride 1),
 *                              k = 6 + AC_FILTER_* (stride 2, may be empty),
 *                              k = 12 + AC_FILTER_* (stride 4, may be empty);
 *                              AC_FILTER_DUAL19: map A (first 64 KiB, hashed as
 *                              ac_plan_hash) then map B (ac_plan_hash2).  A key
 *                              with hash h owns bit h mod 32 of word (or byte)
 *                              h >> shift; the stride-2 and stride-4 maps also
 *                              set it at index (h + 31) >> shift.
 *                              AC_FILTER_PAIR20 (strides 2 and 4): the 4-byte
 *                              window x owns bits h mod 32 and (x >> 24) mod 32
 *                              of word h >> 17, h = ac_plan_hash(x), and at
 *                              stride 2 also bit (x >> 16) mod 32
 */
#define AC_TABLE_CLASS_MAP  1
#define AC_TABLE_DENSE      2
#define AC_TABLE_NODE       3
#define AC_TABLE_LABEL      4
#define AC_TABLE_OUT_OFF    5
#define AC_TABLE_OUT_PID    6
#define AC_TABLE_DEPTH      7
#define AC_TABLE_PREFIX     8
#define AC_TABLE_TAIL       9
#define AC_TABLE_TAIL_INFO  10
#define AC_TABLE_FILTER_BASE 100

int ac_compile(const uint8_t *bytes, const int64_t *offsets, int32_t n_patterns,
               const ac_build_opts *opts, ac_plan **out);
int ac_plan_info(const ac_plan *p, ac_info_t *out);
int64_t ac_plan_export(const ac_plan *p, int32_t table, void *dst, int64_t dst_bytes);
/* Filter hash of a prefix value x (prefix bytes little-endian), as the kernel computes it. */
uint32_t ac_plan_hash(const ac_plan *p, uint32_t x);
/* The second filter hash (map B of AC_FILTER_DUAL19). */
uint32_t ac_plan_hash2(const ac_plan *p, uint32_t x);
/* The two buckets (of 4 slots) of the exact prefix table that may hold prefix x. */
void ac_plan_prefix_buckets(const ac_plan *p, uint32_t x, uint32_t *b1, uint32_t *b2);
void ac_plan_free(ac_plan *p);

#ifdef __cplusplus
}
#endif
#endif /* PFAC_H */
