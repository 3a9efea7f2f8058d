// Request server over the matcher: admission against an HBM budget, batch
// formation, one engine thread that drives several streams, and an open-loop
// trace replayer.  Every scan goes through ac_match_batch_async, so a served
// request gets exactly the match set a standalone ac_match would give it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pfac_internal.hpp"
#include "pfac_serve.h"

namespace {

using pfac::report_error;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Opts {
    int32_t mode = AC_SERVE_BATCHED;
    int32_t n_streams = 3;
    int64_t budget = int64_t(32) << 30;
    int64_t max_batch_bytes = int64_t(256) << 20;
    int32_t max_batch_texts = 4096;
    int32_t matches_per_kib = 4;
};

int resolve_opts(const ac_server_opts *o, Opts &r) {
    r = Opts();
    if (!o) return AC_OK;
    if (o->mode != AC_SERVE_BATCHED && o->mode != AC_SERVE_FIFO)
        return report_error(AC_EINVAL, "ac_server_opts: bad mode");
    if (o->n_streams < 0 || o->n_streams > 16) return report_error(AC_EINVAL, "ac_server_opts: n_streams in 0..16");
    if (o->hbm_budget_bytes < 0 || o->max_batch_bytes < 0 || o->max_batch_texts < 0 || o->matches_per_kib < 0)
        return report_error(AC_EINVAL, "ac_server_opts: negative limit");
    r.mode = o->mode;
    if (o->n_streams) r.n_streams = o->n_streams;
    if (r.mode == AC_SERVE_FIFO) r.n_streams = 1;
    if (o->hbm_budget_bytes) r.budget = o->hbm_budget_bytes;
    if (o->max_batch_bytes) r.max_batch_bytes = o->max_batch_bytes;
    if (o->max_batch_texts) r.max_batch_texts = o->max_batch_texts;
    if (o->matches_per_kib) r.matches_per_kib = o->matches_per_kib;
    return AC_OK;
}

// match slots reserved for a request of len bytes
int64_t reserve_matches(const Opts &o, int64_t len) {
    return std::max<int64_t>(256, (len + 1023) / 1024 * o.matches_per_kib);
}

int64_t charge_of(const Opts &o, int64_t len) { return len + 16 * reserve_matches(o, len); }

int32_t plan_batch(const Opts &o, int32_t n, const int32_t *aut, const int64_t *len, int64_t free_budget,
                   int32_t *picked) {
    if (n <= 0) return 0;
    int64_t used = charge_of(o, len[0]);
    if (used > free_budget) return 0;
    picked[0] = 0;
    int32_t k = 1;
    if (o.mode == AC_SERVE_FIFO) return k;
    int64_t bytes = len[0];
    for (int32_t i = 1; i < n && k < o.max_batch_texts; ++i) {
        if (aut[i] != aut[0]) continue;
        const int64_t c = charge_of(o, len[i]);
        if (bytes + len[i] > o.max_batch_bytes || used + c > free_budget) continue;
        picked[k++] = i;
        bytes += len[i];
        used += c;
    }
    return k;
}

struct Request {
    int64_t id = 0;
    int32_t aut = 0;
    const ac_automaton *a = nullptr;
    const uint8_t *text = nullptr;
    int64_t len = 0;
    int64_t charge = 0;
    int64_t submit_ns = 0, done_ns = 0;
    int32_t status = AC_OK;
    int32_t batch_n = 0;
    bool done = false;
    std::vector<int64_t> off;
    std::vector<int32_t> pid;
};
using ReqPtr = std::shared_ptr<Request>;

// One stream with the buffers of the batch it runs.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    uint8_t *d_text = nullptr;
    int64_t text_cap = 0;
    int64_t *d_offs = nullptr, *h_offs = nullptr;
    int64_t *d_per = nullptr, *h_per = nullptr;
    int64_t texts_cap = 0;
    int32_t *d_tid = nullptr, *h_tid = nullptr;
    int64_t *d_off = nullptr, *h_off = nullptr;
    int32_t *d_pid = nullptr, *h_pid = nullptr;
    int64_t match_cap = 0;
    int64_t *d_count = nullptr, *h_count = nullptr;
    int64_t scratch_bytes = 0;      // the scan's per-stream scratch
    // batch in flight
    int phase = 0;                  // 0 idle, 1 scan + counts, 2 matches coming back
    std::vector<ReqPtr> batch;
    const ac_automaton *aut = nullptr;
    int64_t total = 0, cap = 0, charged = 0;
};

template <typename T>
int dev_alloc(T **p, int64_t n) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), size_t(std::max<int64_t>(n, 1)) * sizeof(T));
    return e == hipSuccess ? AC_OK : report_error(AC_ENOMEM, std::string("server hipMalloc: ") + hipGetErrorString(e));
}

template <typename T>
int host_alloc(T **p, int64_t n) {
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(p), size_t(std::max<int64_t>(n, 1)) * sizeof(T),
                                 hipHostMallocDefault);
    return e == hipSuccess ? AC_OK
                           : report_error(AC_ENOMEM, std::string("server hipHostMalloc: ") + hipGetErrorString(e));
}

int grow(Slot &s, int64_t text_bytes, int64_t texts, int64_t matches) {
    int rc = AC_OK;
    if (text_bytes > s.text_cap) {
        if ((rc = dev_alloc(&s.d_text, text_bytes))) return rc;
        s.text_cap = text_bytes;
    }
    if (texts > s.texts_cap) {
        if ((rc = dev_alloc(&s.d_offs, texts + 1)) || (rc = host_alloc(&s.h_offs, texts + 1)) ||
            (rc = dev_alloc(&s.d_per, texts)) || (rc = host_alloc(&s.h_per, texts)))
            return rc;
        s.texts_cap = texts;
    }
    if (matches > s.match_cap) {
        if ((rc = dev_alloc(&s.d_tid, matches)) || (rc = host_alloc(&s.h_tid, matches)) ||
            (rc = dev_alloc(&s.d_off, matches)) || (rc = host_alloc(&s.h_off, matches)) ||
            (rc = dev_alloc(&s.d_pid, matches)) || (rc = host_alloc(&s.h_pid, matches)))
            return rc;
        s.match_cap = matches;
    }
    return AC_OK;
}

// Device memory a slot holds: its buffers and the scan's stream scratch.
int64_t slot_device_bytes(const Slot &s) {
    return s.text_cap + (s.texts_cap + 1) * 8 + s.texts_cap * 8 + s.match_cap * (4 + 8 + 4) + 8 + s.scratch_bytes;
}

void release_slot(Slot &s) {
    for (void *p : {static_cast<void *>(s.d_text), static_cast<void *>(s.d_offs), static_cast<void *>(s.d_per),
                    static_cast<void *>(s.d_tid), static_cast<void *>(s.d_off), static_cast<void *>(s.d_pid),
                    static_cast<void *>(s.d_count)})
        if (p) (void)hipFree(p);
    for (void *p : {static_cast<void *>(s.h_offs), static_cast<void *>(s.h_per), static_cast<void *>(s.h_tid),
                    static_cast<void *>(s.h_off), static_cast<void *>(s.h_pid), static_cast<void *>(s.h_count)})
        if (p) (void)hipHostFree(p);
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.stream) {
        (void)hipStreamSynchronize(s.stream);
        pfac::release_stream_scratch(s.stream);
        (void)hipStreamDestroy(s.stream);
    }
    s = Slot();
}

}  // namespace

struct ac_server {
    Opts o;
    int device = 0;
    std::vector<const ac_automaton *> auts;
    int64_t aut_bytes = 0;
    // device bytes of the server's own buffers (all slots), charged against
    // the budget like the automata; written by the engine thread under mu
    int64_t resident = 0;

    mutable std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ReqPtr> waiting;
    std::unordered_map<int64_t, ReqPtr> reqs;
    int64_t next_id = 0;
    int64_t inflight_charge = 0;
    bool stop = false;
    bool blocked = false;            // the oldest request is waiting for budget
    ac_server_stats stats{};

    std::vector<Slot> slots;         // touched by the engine thread only
    std::thread engine;

    void run();
    void note_resident();
    bool launch(Slot &s, std::vector<ReqPtr> batch);
    bool advance(Slot &s);
    void finish(Slot &s, int status);
    int enqueue_scan(Slot &s);
};

// Recomputes the resident bytes after a slot's buffers grew.
void ac_server::note_resident() {
    int64_t r = 0;
    for (const auto &sl : slots) r += slot_device_bytes(sl);
    std::lock_guard<std::mutex> lk(mu);
    resident = r;
    stats.resident_bytes = r;
}

int ac_server::enqueue_scan(Slot &s) {
    ac_batch_matches m{s.d_tid, s.d_off, s.d_pid, s.cap, s.d_per};
    const int rc = ac_match_batch_async(s.aut, s.d_text, s.d_offs, int32_t(s.batch.size()), s.total, &m, nullptr,
                                        s.d_count, s.stream);
    if (rc) return rc;
    const int64_t n = int64_t(s.batch.size());
    hipError_t e = hipMemcpyAsync(s.h_count, s.d_count, sizeof(int64_t), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_per, s.d_per, size_t(n) * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.ev, s.stream);
    return e == hipSuccess ? AC_OK : report_error(AC_EHIP, std::string("server copy: ") + hipGetErrorString(e));
}

// Copies the batch's texts in and enqueues its scan; false on failure (the
// batch is then finished with the error).
bool ac_server::launch(Slot &s, std::vector<ReqPtr> batch) {
    s.batch = std::move(batch);
    s.aut = s.batch[0]->a;
    s.total = 0;
    s.cap = 0;
    s.charged = 0;
    for (const auto &r : s.batch) {
        s.total += r->len;
        s.cap += reserve_matches(o, r->len);
        s.charged += r->charge;
    }
    const int64_t n = int64_t(s.batch.size());
    const int64_t before = slot_device_bytes(s);
    int rc = grow(s, s.total, n, s.cap);
    if (slot_device_bytes(s) != before) note_resident();
    hipError_t e = hipSuccess;
    if (!rc) {
        int64_t pos = 0;
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
            const Request &r = *s.batch[size_t(i)];
            s.h_offs[i] = pos;
            if (r.len) e = hipMemcpyAsync(s.d_text + pos, r.text, size_t(r.len), hipMemcpyHostToDevice, s.stream);
            pos += r.len;
        }
        s.h_offs[n] = pos;
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.d_offs, s.h_offs, size_t(n + 1) * 8, hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) rc = report_error(AC_EHIP, std::string("server copy: ") + hipGetErrorString(e));
    }
    if (!rc) rc = enqueue_scan(s);
    if (rc) {
        (void)hipStreamSynchronize(s.stream);
        finish(s, rc);
        return false;
    }
    s.phase = 1;
    std::lock_guard<std::mutex> lk(mu);
    stats.batches++;
    stats.max_batch_requests = std::max<int64_t>(stats.max_batch_requests, n);
    return true;
}

// Moves a slot whose event has completed to its next phase.
bool ac_server::advance(Slot &s) {
    if (s.phase == 1) {
        const int64_t count = *s.h_count;
        if (count > s.cap) {
            // more matches than reserved slots: scan the resident texts again
            const int64_t before = slot_device_bytes(s);
            int rc = grow(s, s.total, int64_t(s.batch.size()), count);
            if (slot_device_bytes(s) != before) note_resident();
            s.cap = count;
            if (!rc) rc = enqueue_scan(s);
            if (rc) { finish(s, rc); return true; }
            std::lock_guard<std::mutex> lk(mu);
            stats.rescans++;
            return true;
        }
        if (count > 0) {
            hipError_t e = hipMemcpyAsync(s.h_tid, s.d_tid, size_t(count) * 4, hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.h_off, s.d_off, size_t(count) * 8, hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.h_pid, s.d_pid, size_t(count) * 4, hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess) e = hipEventRecord(s.ev, s.stream);
            if (e != hipSuccess) {
                finish(s, report_error(AC_EHIP, std::string("server copy: ") + hipGetErrorString(e)));
                return true;
            }
            s.phase = 2;
            return true;
        }
    }
    finish(s, AC_OK);
    return true;
}

// Hands every request of the slot's batch its matches and frees its charge.
void ac_server::finish(Slot &s, int status) {
    const int64_t n = int64_t(s.batch.size());
    if (status == AC_OK) {
        const int64_t count = s.phase == 2 ? *s.h_count : 0;
        std::vector<int64_t> fill(size_t(n), 0);
        for (int64_t i = 0; i < n; ++i) {
            Request &r = *s.batch[size_t(i)];
            r.off.resize(size_t(s.h_per[i]));
            r.pid.resize(size_t(s.h_per[i]));
        }
        for (int64_t j = 0; j < count; ++j) {
            const int32_t t = s.h_tid[j];
            if (t < 0 || t >= n) continue;
            Request &r = *s.batch[size_t(t)];
            const int64_t k = fill[size_t(t)]++;
            if (k >= int64_t(r.off.size())) continue;
            r.off[size_t(k)] = s.h_off[j];
            r.pid[size_t(k)] = s.h_pid[j];
        }
    }
    const int64_t t_done = now_ns();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const auto &rp : s.batch) {
            rp->status = status;
            rp->batch_n = int32_t(n);
            rp->done_ns = t_done;
            rp->done = true;
            stats.requests++;
            stats.text_bytes += rp->len;
        }
        inflight_charge -= s.charged;
        blocked = false;
    }
    cv_done.notify_all();
    s.batch.clear();
    s.phase = 0;
}

void ac_server::run() {
    (void)hipSetDevice(device);
    std::vector<int32_t> aut_ids, picked;
    std::vector<int64_t> lens;
    while (true) {
        bool progressed = false;
        for (auto &s : slots) {
            if (s.phase == 0) continue;
            const hipError_t q = hipEventQuery(s.ev);
            if (q == hipSuccess) {
                progressed |= advance(s);
            } else if (q != hipErrorNotReady) {
                (void)hipStreamSynchronize(s.stream);
                finish(s, report_error(AC_EHIP, std::string("server scan: ") + hipGetErrorString(q)));
                progressed = true;
            }
        }
        for (auto &s : slots) {
            if (s.phase != 0) continue;
            std::vector<ReqPtr> batch;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (waiting.empty()) break;
                const int32_t n = int32_t(std::min<size_t>(waiting.size(), size_t(1) << 20));
                aut_ids.resize(size_t(n));
                lens.resize(size_t(n));
                picked.resize(size_t(n));
                for (int32_t i = 0; i < n; ++i) {
                    aut_ids[size_t(i)] = waiting[size_t(i)]->aut;
                    lens[size_t(i)] = waiting[size_t(i)]->len;
                }
                const int64_t free_budget = o.budget - aut_bytes - resident - inflight_charge;
                const int32_t k = plan_batch(o, n, aut_ids.data(), lens.data(), free_budget, picked.data());
                if (k == 0) {
                    if (!blocked) stats.admission_waits++;
                    blocked = true;
                    break;
                }
                for (int32_t j = k - 1; j >= 0; --j) {
                    const size_t i = size_t(picked[size_t(j)]);
                    batch.push_back(waiting[i]);
                    waiting.erase(waiting.begin() + std::ptrdiff_t(i));
                }
                std::reverse(batch.begin(), batch.end());
                int64_t c = 0;
                for (const auto &r : batch) c += r->charge;
                inflight_charge += c;
                stats.peak_charged = std::max(stats.peak_charged, inflight_charge + aut_bytes + resident);
            }
            launch(s, std::move(batch));
            progressed = true;
        }
        if (progressed) continue;
        bool busy = false;
        for (auto &s : slots) busy |= s.phase != 0;
        std::unique_lock<std::mutex> lk(mu);
        if (!busy) {
            if (stop && waiting.empty()) break;
            if (waiting.empty() || blocked) cv_work.wait(lk, [&] { return stop || (!waiting.empty() && !blocked); });
        } else {
            lk.unlock();
            std::this_thread::yield();   // batches in flight: poll their events
        }
    }
}

extern "C" {

int64_t ac_serve_charge(const ac_server_opts *opts, int64_t len) {
    Opts o;
    if (int rc = resolve_opts(opts, o)) return rc;
    if (len < 0) return report_error(AC_EINVAL, "ac_serve_charge: negative length");
    return charge_of(o, len);
}

int32_t ac_serve_plan(const ac_server_opts *opts, int32_t n_waiting, const int32_t *automaton, const int64_t *len,
                      int64_t free_budget, int32_t *picked) {
    Opts o;
    if (int rc = resolve_opts(opts, o)) return rc;
    if (n_waiting < 0 || (n_waiting > 0 && (!automaton || !len || !picked)))
        return report_error(AC_EINVAL, "ac_serve_plan: bad arguments");
    return plan_batch(o, n_waiting, automaton, len, free_budget, picked);
}

int ac_server_create(const ac_server_opts *opts, ac_server **out) {
    if (!out) return report_error(AC_EINVAL, "ac_server_create: NULL output");
    *out = nullptr;
    Opts o;
    if (int rc = resolve_opts(opts, o)) return rc;
    ac_server *s = new (std::nothrow) ac_server();
    if (!s) return report_error(AC_ENOMEM, "ac_server_create: out of host memory");
    s->o = o;
    hipError_t e = hipGetDevice(&s->device);
    int rc = e == hipSuccess ? AC_OK : report_error(AC_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    s->slots.resize(size_t(o.n_streams));
    for (auto &sl : s->slots) {
        if (rc) break;
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess) {
            rc = report_error(AC_EHIP, std::string("server stream: ") + hipGetErrorString(e));
            break;
        }
        if ((rc = dev_alloc(&sl.d_count, 1)) || (rc = host_alloc(&sl.h_count, 1))) break;
        // the scan's scratch: hit regions for the widest launch
        if ((rc = pfac::reserve_stream_scratch(sl.stream, &sl.scratch_bytes))) break;
        // sized for a full batch, so that serving never reallocates (a single
        // request longer than max_batch_bytes still grows its stream's buffers)
        const int64_t texts = std::min<int64_t>(o.max_batch_texts, 1 << 16);
        rc = grow(sl, o.max_batch_bytes, texts, reserve_matches(o, o.max_batch_bytes) + 256 * texts);
    }
    if (!rc) {
        s->note_resident();
        if (s->resident > o.budget)
            rc = report_error(AC_EINVAL, "ac_server_create: the server's own buffers (" + std::to_string(s->resident) +
                                             " bytes) exceed the HBM budget");
    }
    if (rc) {
        for (auto &sl : s->slots) release_slot(sl);
        delete s;
        return rc;
    }
    s->engine = std::thread([s] { s->run(); });
    *out = s;
    return AC_OK;
}

void ac_server_destroy(ac_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->engine.joinable()) s->engine.join();
    for (auto &sl : s->slots) release_slot(sl);
    delete s;
}

int ac_server_add_automaton(ac_server *s, const ac_automaton *a) {
    if (!s || !a) return report_error(AC_EINVAL, "ac_server_add_automaton: NULL argument");
    if (a->device != s->device) return report_error(AC_EINVAL, "ac_server_add_automaton: automaton on another device");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->aut_bytes + s->resident + a->dbytes > s->o.budget)
        return report_error(AC_EINVAL, "ac_server_add_automaton: automata exceed the HBM budget");
    s->auts.push_back(a);
    s->aut_bytes += a->dbytes;
    return int(s->auts.size()) - 1;
}

int64_t ac_server_submit(ac_server *s, int32_t automaton, const uint8_t *text, int64_t len) {
    if (!s) return report_error(AC_EINVAL, "ac_server_submit: NULL server");
    if (len < 0 || (len > 0 && !text)) return report_error(AC_EINVAL, "ac_server_submit: bad text");
    auto r = std::make_shared<Request>();
    r->aut = automaton;
    r->text = text;
    r->len = len;
    r->charge = charge_of(s->o, len);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (automaton < 0 || size_t(automaton) >= s->auts.size())
            return report_error(AC_EINVAL, "ac_server_submit: unknown automaton id");
        r->a = s->auts[size_t(automaton)];
        if (s->stop) return report_error(AC_EINVAL, "ac_server_submit: server is stopping");
        if (r->charge > s->o.budget - s->aut_bytes - s->resident)
            return report_error(AC_EINVAL, "ac_server_submit: request larger than the HBM budget");
        r->id = s->next_id++;
        r->submit_ns = now_ns();
        s->reqs[r->id] = r;
        s->waiting.push_back(r);
    }
    s->cv_work.notify_one();
    return r->id;
}

static void fill_result(const Request &r, ac_request_result *out) {
    out->status = r.status;
    out->batch_requests = r.batch_n;
    out->count = int64_t(r.off.size());
    out->offset = r.off.data();
    out->pattern_id = r.pid.data();
    out->submit_ns = r.submit_ns;
    out->done_ns = r.done_ns;
}

int ac_server_wait(ac_server *s, int64_t request, ac_request_result *out) {
    if (!s || !out) return report_error(AC_EINVAL, "ac_server_wait: NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request);
    if (it == s->reqs.end()) return report_error(AC_EINVAL, "ac_server_wait: unknown request");
    ReqPtr r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    fill_result(*r, out);
    return r->status;
}

int ac_server_poll(ac_server *s, int64_t request, ac_request_result *out) {
    if (!s || !out) return report_error(AC_EINVAL, "ac_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request);
    if (it == s->reqs.end()) return report_error(AC_EINVAL, "ac_server_poll: unknown request");
    if (!it->second->done) return 0;
    fill_result(*it->second, out);
    return it->second->status ? it->second->status : 1;
}

void ac_server_release(ac_server *s, int64_t request) {
    if (!s) return;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request);
    if (it != s->reqs.end() && it->second->done) s->reqs.erase(it);
}

int ac_server_replay(ac_server *s, int32_t n, const int32_t *automaton, const uint8_t *const *text,
                     const int64_t *len, const int64_t *arrival_ns, int64_t *latency_ns, int64_t *count) {
    if (!s || n < 0 || (n > 0 && (!automaton || !text || !len || !arrival_ns || !latency_ns || !count)))
        return report_error(AC_EINVAL, "ac_server_replay: bad arguments");
    std::vector<int64_t> ids(size_t(n), -1);
    const int64_t start = now_ns();
    int first_err = AC_OK;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t target = start + arrival_ns[i];
        int64_t t = now_ns();
        if (target - t > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(target - t - 150000));
        while (now_ns() < target) {
        }
        const int64_t id = ac_server_submit(s, automaton[i], text[i], len[i]);
        if (id < 0 && !first_err) first_err = int(id);
        ids[size_t(i)] = id;
    }
    for (int32_t i = 0; i < n; ++i) {
        latency_ns[i] = -1;
        count[i] = -1;
        if (ids[size_t(i)] < 0) continue;
        ac_request_result r{};
        const int rc = ac_server_wait(s, ids[size_t(i)], &r);
        if (rc && !first_err) first_err = rc;
        latency_ns[i] = r.done_ns - (start + arrival_ns[i]);
        count[i] = r.count;
        ac_server_release(s, ids[size_t(i)]);
    }
    return first_err;
}

int ac_server_get_stats(const ac_server *s, ac_server_stats *out) {
    if (!s || !out) return report_error(AC_EINVAL, "ac_server_get_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return AC_OK;
}

}  // extern "C"
