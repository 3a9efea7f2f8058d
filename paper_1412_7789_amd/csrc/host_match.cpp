// CPU matcher of the library: the same failure-less walk as the GPU kernels
// (paper, Section II, Fig. 5: every offset walks the Goto trie from the root
// and stops at the first missing transition), run on host threads over the
// tables the builder made for the GPU (dense rows for shallow states, sorted
// child lists below, Output lists).  It serves the CPU side of the CPU/GPU
// dispatch (Section IV and V: below a crossover size the CPU finishes first,
// so small inputs should go to it).
#include <algorithm>
#include <thread>
#include <vector>

#include "pfac_internal.hpp"

namespace pfac {

namespace {

// Every keyword starting at offset o of text[0, n): calls emit(state) for
// each final state the walk from o enters.
template <typename Emit>
inline void walk_from(const Plan &P, const uint8_t *t, int64_t n, int64_t o, Emit &&emit) {
    int32_t s = 0;
    for (int64_t j = o; j < n; ++j) {
        const uint8_t b = t[j];
        if (s < P.S_dense) {
            const int32_t e = P.dense[size_t(s) * size_t(P.C) + P.cls[b]];
            if (e == 0) return;
            s = e & 0x7fffffff;
            if (e < 0) emit(s);
        } else {
            // children of s: first_child[s] .. + n_child[s], edge bytes ascending
            const int32_t fc = P.first_child[size_t(s)];
            const uint8_t *lab = P.label.data() + fc;
            const uint8_t *end = lab + P.n_child[size_t(s)];
            const uint8_t *it = std::lower_bound(lab, end, b);
            if (it == end || *it != b) return;
            s = fc + int32_t(it - lab);
            if (P.out_off[size_t(s) + 1] > P.out_off[size_t(s)]) emit(s);
        }
    }
}

struct Found {
    std::vector<int64_t> off;
    std::vector<int32_t> pid;
};

void scan_range(const Plan &P, const uint8_t *t, int64_t n, int64_t o0, int64_t o1, Found &out) {
    for (int64_t o = o0; o < o1; ++o) {
        // most offsets end at the root: no keyword starts with this byte
        if (P.dense[P.cls[t[o]]] == 0) continue;
        walk_from(P, t, n, o, [&](int32_t s) {
            for (int32_t k = P.out_off[size_t(s)]; k < P.out_off[size_t(s) + 1]; ++k) {
                out.off.push_back(o);
                out.pid.push_back(P.out_pid[size_t(k)]);
            }
        });
    }
}

}  // namespace

int64_t host_match(const Plan &P, const uint8_t *text, int64_t n, int64_t *off, int32_t *pid, int64_t cap,
                   int32_t n_threads) {
    if (n <= 0) return 0;
    int64_t threads = n_threads;
    if (threads <= 0) {
        // one thread below 1 MiB (starting threads costs more than it saves),
        // else one per 256 KiB up to the machine's threads
        threads = n < (int64_t(1) << 20) ? 1
                                         : std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()),
                                                             n / (int64_t(256) << 10));
    }
    threads = std::max<int64_t>(1, std::min<int64_t>({threads, n, 256}));
    std::vector<Found> found(static_cast<size_t>(threads));
    const int64_t per = (n + threads - 1) / threads;
    if (threads == 1) {
        scan_range(P, text, n, 0, n, found[0]);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(size_t(threads));
        for (int64_t i = 0; i < threads; ++i) {
            const int64_t o0 = std::min(n, i * per), o1 = std::min(n, o0 + per);
            pool.emplace_back([&, i, o0, o1] { scan_range(P, text, n, o0, o1, found[size_t(i)]); });
        }
        for (auto &th : pool) th.join();
    }
    int64_t total = 0;
    for (const Found &f : found) {
        const int64_t k = int64_t(f.off.size());
        const int64_t put = std::max<int64_t>(0, std::min<int64_t>(k, cap - total));
        if (put > 0) {
            std::copy(f.off.begin(), f.off.begin() + put, off + total);
            std::copy(f.pid.begin(), f.pid.begin() + put, pid + total);
        }
        total += k;
    }
    return total;
}

}  // namespace pfac
