/*
 * pfac_serve.h -- request server over the failure-less Aho-Corasick matcher.
 *
 * Serving form of the paper's data-parallel scan (Section II, Fig. 3 "N"):
 * many independent requests (host text + one of several resident keyword
 * automata) arrive over time; the server copies their texts into HBM, scans
 * every request in one launch of the batch kernel together with the other
 * requests for the same automaton that are waiting, and hands each request
 * its exact match set (the set R of ac_match) in host memory.
 *
 *   AC_SERVE_BATCHED  continuous batching: while batches are in flight on
 *                     some streams, arrivals wait in a queue and form the
 *                     next batch on the next free stream.
 *   AC_SERVE_FIFO     the plain way: one stream, one launch per request, in
 *                     arrival order.
 *
 * Admission: every request is charged its text bytes plus its match buffer
 * (16 bytes per reserved match) against hbm_budget_bytes, after the
 * registered automata's device bytes and the server's own device buffers
 * (per stream: the scan's scratch and text and match buffers sized for
 * max_batch_bytes; they grow, and are charged more, if a single request is
 * larger; ac_server_stats.resident_bytes reports them).  The oldest waiting
 * request is always served first (no overtaking across automata); when its
 * charge does not fit the budget left by the batches in flight it waits
 * ("admission wait").
 *
 * Threads: the server owns one engine thread that makes every HIP call of
 * the server (streams of default priority, created on the device current at
 * ac_server_create).  ac_server_submit / wait / poll / release may be called
 * from any thread.  Errors are negative AC_* codes (pfac.h); the message is
 * in ac_last_error() of the calling thread.
 */
#ifndef PFAC_SERVE_H
#define PFAC_SERVE_H

#include "pfac.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ac_server ac_server;

#define AC_SERVE_BATCHED 0
#define AC_SERVE_FIFO 1

typedef struct {
    int32_t mode;              /* AC_SERVE_BATCHED (default) or AC_SERVE_FIFO            */
    int32_t n_streams;         /* batches in flight at once; 0 = 3 (FIFO: always 1)      */
    int64_t hbm_budget_bytes;  /* 0 = 32 GiB                                             */
    int64_t max_batch_bytes;   /* text bytes per batch; 0 = 256 MiB (a longer request is */
                               /* served alone)                                          */
    int32_t max_batch_texts;   /* requests per batch; 0 = 4096                           */
    int32_t matches_per_kib;   /* match slots reserved per KiB of text; 0 = 4 (at least  */
                               /* 256 per request); more matches cost one re-scan        */
    int32_t reserved[6];
} ac_server_opts;

/* Creates a server on the current device.  opts may be NULL (defaults).
 * Errors: AC_EINVAL (bad option), AC_ENOMEM, AC_EHIP. */
int ac_server_create(const ac_server_opts *opts, ac_server **out);

/* Waits for every submitted request, stops the engine, frees the server's
 * memory (not the automata). */
void ac_server_destroy(ac_server *s);

/* Registers a built automaton (not owned: it must outlive the server) and
 * charges its device bytes against the budget.  Returns its id (>= 0).
 * Errors: AC_EINVAL (NULL, other device, budget exceeded). */
int ac_server_add_automaton(ac_server *s, const ac_automaton *a);

/* Queues one request: scan host text[0 .. len) with automaton `automaton`.
 * The text must stay valid and unchanged until the request completes; pinned
 * memory (hipHostMalloc) is copied asynchronously, pageable memory through
 * HIP's staging.  Returns the request id (>= 0).  Errors: AC_EINVAL (bad id,
 * len < 0, NULL text with len > 0, a charge larger than the whole budget
 * left after the automata). */
int64_t ac_server_submit(ac_server *s, int32_t automaton, const uint8_t *text, int64_t len);

/* Result of a completed request.  The arrays are host memory owned by the
 * server until ac_server_release; matches are in unspecified order. */
typedef struct {
    int32_t status;            /* AC_OK, or the error that failed the request     */
    int32_t batch_requests;    /* requests in the launch that served it            */
    int64_t count;             /* exact number of matches                          */
    const int64_t *offset;     /* [count] start offsets within the request's text  */
    const int32_t *pattern_id; /* [count]                                          */
    int64_t submit_ns;         /* steady-clock ns at ac_server_submit              */
    int64_t done_ns;           /* steady-clock ns when the result became visible   */
} ac_request_result;

/* Blocks until `request` completes and fills *out.  AC_EINVAL for an unknown
 * or released id. */
int ac_server_wait(ac_server *s, int64_t request, ac_request_result *out);

/* Non-blocking: 1 and *out filled when complete, 0 while pending. */
int ac_server_poll(ac_server *s, int64_t request, ac_request_result *out);

/* Frees a completed request's result (no-op for unknown ids). */
void ac_server_release(ac_server *s, int64_t request);

/*
 * Open-loop replay of a request trace for measurement: from the calling
 * thread, submits request i at (start + arrival_ns[i]) on the steady clock
 * (arrival_ns non-decreasing, relative to the call), then waits for all.
 * latency_ns[i] = time the result became visible - scheduled arrival;
 * count[i] = its match count.  Results are released.  Returns AC_OK or the
 * first error.
 */
int ac_server_replay(ac_server *s, int32_t n, const int32_t *automaton, const uint8_t *const *text,
                     const int64_t *len, const int64_t *arrival_ns, int64_t *latency_ns, int64_t *count);

typedef struct {
    int64_t requests;          /* completed                                         */
    int64_t batches;           /* launches                                          */
    int64_t text_bytes;        /* bytes scanned                                     */
    int64_t admission_waits;   /* times the oldest request waited for budget        */
    int64_t rescans;           /* batches scanned again for lack of match slots     */
    int64_t peak_charged;      /* largest budget charge: automata + resident +
                                  requests in flight (bytes)                        */
    int64_t max_batch_requests;
    int64_t resident_bytes;    /* device bytes of the server's own buffers          */
    int64_t reserved[3];
} ac_server_stats;

int ac_server_get_stats(const ac_server *s, ac_server_stats *out);

/* ---- host-side rules, exposed for tests (no GPU needed) ---------------------- */

/* Budget charge of a request of len bytes under opts (NULL = defaults). */
int64_t ac_serve_charge(const ac_server_opts *opts, int64_t len);

/*
 * The batch-formation rule: given the waiting requests in arrival order
 * (automaton ids, lengths) and the budget left, writes the indices of the
 * next batch (ascending) to picked[] and returns how many.  The batch starts
 * with the oldest request and takes, in order, the later ones for the same
 * automaton while the text, request-count and budget limits hold.  Returns 0
 * when the oldest request's charge exceeds free_budget (admission wait).
 */
int32_t ac_serve_plan(const ac_server_opts *opts, int32_t n_waiting, const int32_t *automaton,
                      const int64_t *len, int64_t free_budget, int32_t *picked);

#ifdef __cplusplus
}
#endif
#endif /* PFAC_SERVE_H */
