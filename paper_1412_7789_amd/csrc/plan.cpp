// Host-side automaton builder for the failure-less Aho-Corasick matcher.
//
// Builds the Goto trie of the keyword set (paper, Section II and Fig. 5: the
// failure-less machine is the Goto function alone plus the Output lists),
// numbers its states breadth first, compresses the byte alphabet into classes
// and lays the transitions out for the GPU:
//
//   * dense rows  int32[C] for every state of depth <= D, where D is the
//     largest depth whose rows fit the dense budget.  Entry = next state with
//     bit 31 set when that state ends a keyword; 0 = no transition (the root
//     is never a target, so 0 is free to mean "dead");
//   * compact nodes for deeper states: (first child, child count | final bit)
//     with the children's edge bytes in `label`, contiguous and sorted by the
//     breadth-first numbering;
//   * Output lists as CSR (keyword ids ending at each state, ascending);
//   * candidate filters: each keyword's first K = min(3, shortest keyword)
//     bytes hashed into byte maps and bit maps sized for LDS.
//
// The trie is built from the keywords in lexicographic order, which creates
// each state's children in increasing byte order without any hashing.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>

#include "pfac_internal.hpp"

namespace pfac {

uint32_t prefix_hash(uint32_t x, uint32_t mul) {
    // Same arithmetic as the kernel's 24 x 24-bit multiply (low 32 bits).
    return uint32_t(uint64_t(x & 0xFFFFFFu) * uint64_t(mul & 0xFFFFFFu));
}

void prefix_buckets(uint32_t x, uint32_t mul, int bits, uint32_t &b1, uint32_t &b2) {
    const int nb = bits - 2;                      // buckets of 4 slots
    b1 = prefix_hash(x, mul) >> (32 - nb);
    b2 = prefix_hash(x, kPrefixMul2) >> (32 - nb);
    if (b2 == b1) b2 = b1 ^ 1u;
}

namespace {

// Places every (key, value) in one of its two buckets by cuckoo insertion
// (a deterministic walk of evictions); false when some key found no place.
bool build_cuckoo(const std::vector<std::pair<uint32_t, uint32_t>> &items, int bits, uint32_t mul,
                  std::vector<uint32_t> &table) {
    table.assign(size_t(2) << bits, 0u);
    uint32_t rng = 0x2545F491u;
    for (auto item : items) {
        uint32_t key = item.first, val = item.second;
        uint32_t b1, b2;
        prefix_buckets(key & 0xFFFFFFu, mul, bits, b1, b2);
        uint32_t next = b1;
        bool placed = false;
        for (int kick = 0; kick < 1000 && !placed; ++kick) {
            // a free slot in either bucket ends the walk
            for (uint32_t b : {b1, b2}) {
                for (uint32_t j = 0; j < 4 && !placed; ++j) {
                    const size_t at = (size_t(b) * 4 + j) * 2;
                    if (table[at + 1] == 0u) {
                        table[at] = key;
                        table[at + 1] = val;
                        placed = true;
                    }
                }
                if (placed) break;
            }
            if (placed) break;
            // evict a slot of `next` and carry its entry to its other bucket
            rng ^= rng << 13; rng ^= rng >> 17; rng ^= rng << 5;
            const size_t at = (size_t(next) * 4 + (rng & 3u)) * 2;
            std::swap(key, table[at]);
            std::swap(val, table[at + 1]);
            uint32_t e1, e2;
            prefix_buckets(key & 0xFFFFFFu, mul, bits, e1, e2);
            b1 = e1;
            b2 = e2;
            next = (e1 == next) ? e2 : e1;
        }
        if (!placed) return false;
    }
    return true;
}

}  // namespace

int compile_plan(const uint8_t *bytes, const int64_t *offsets, int32_t n,
                 const ac_build_opts *opts, Plan &P, std::string &err) {
    auto t0 = std::chrono::steady_clock::now();
    if (n <= 0) { err = "ac_build: need at least one keyword"; return AC_EINVAL; }
    if (!bytes || !offsets) { err = "ac_build: NULL keyword buffer"; return AC_EINVAL; }
    int64_t dense_budget = (opts && opts->dense_budget_bytes > 0) ? opts->dense_budget_bytes
                                                                   : kDefaultDenseBudget;
    uint32_t mul = (opts && opts->hash_multiplier) ? (opts->hash_multiplier & 0xFFFFFFu) | 1u
                                                   : kDefaultHashMul;
    P = Plan();
    P.n_patterns = n;
    P.hash_mul = mul;
    P.kw_len.resize(n);
    int64_t total = 0;
    P.min_len = INT32_MAX;
    for (int32_t p = 0; p < n; ++p) {
        int64_t L = offsets[p + 1] - offsets[p];
        if (L <= 0) { err = "ac_build: keyword " + std::to_string(p) + " is empty"; return AC_EINVAL; }
        if (L > (1 << 30)) { err = "ac_build: keyword longer than 2^30 bytes"; return AC_EINVAL; }
        P.kw_len[p] = L;
        total += L;
        P.min_len = std::min<int64_t>(P.min_len, L);
        P.max_len = std::max<int64_t>(P.max_len, L);
    }
    if (total >= (int64_t(1) << 30) - 1) { err = "ac_build: more than 2^30 trie states"; return AC_EINVAL; }
    P.K = std::min(kMaxPrefix, P.min_len);

    // ---- Goto trie, built in lexicographic keyword order -------------------
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto kw = [&](int32_t p) { return bytes + offsets[p]; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        int64_t la = P.kw_len[a], lb = P.kw_len[b];
        int c = std::memcmp(kw(a), kw(b), size_t(std::min(la, lb)));
        if (c) return c < 0;
        return la < lb;
    });
    // creation-order trie: parent, edge byte, depth; terminal state per keyword
    std::vector<int32_t> parent(1, -1), cdepth(1, 0);
    std::vector<uint8_t> clabel(1, 0);
    std::vector<int32_t> terminal(n, 0);
    std::vector<int32_t> path(1, 0);
    parent.reserve(size_t(total) + 1);
    cdepth.reserve(size_t(total) + 1);
    clabel.reserve(size_t(total) + 1);
    int32_t prev = -1;
    for (int32_t idx = 0; idx < n; ++idx) {
        int32_t p = order[idx];
        int64_t L = P.kw_len[p], lcp = 0;
        if (prev >= 0) {
            int64_t m = std::min(L, P.kw_len[prev]);
            const uint8_t *a = kw(p), *b = kw(prev);
            while (lcp < m && a[lcp] == b[lcp]) ++lcp;
        }
        path.resize(size_t(lcp) + 1);
        for (int64_t d = lcp; d < L; ++d) {
            int32_t t = int32_t(parent.size());
            parent.push_back(path[size_t(d)]);
            clabel.push_back(kw(p)[d]);
            cdepth.push_back(int32_t(d + 1));
            path.push_back(t);
        }
        terminal[p] = path[size_t(L)];
        prev = p;
    }
    const int32_t S = int32_t(parent.size());
    P.S = S;

    // children lists in creation order (already sorted by byte)
    std::vector<int32_t> ch_off(size_t(S) + 1, 0), ch(size_t(S > 0 ? S - 1 : 0));
    for (int32_t t = 1; t < S; ++t) ch_off[size_t(parent[t]) + 1]++;
    for (int32_t s = 0; s < S; ++s) ch_off[size_t(s) + 1] += ch_off[size_t(s)];
    {
        std::vector<int32_t> fill(ch_off.begin(), ch_off.end() - 1);
        for (int32_t t = 1; t < S; ++t) ch[size_t(fill[size_t(parent[t])]++)] = t;
    }

    // ---- breadth-first numbering ------------------------------------------
    std::vector<int32_t> bfs(static_cast<size_t>(S)), newid(static_cast<size_t>(S));
    bfs[0] = 0;
    newid[0] = 0;
    int64_t head = 0, tail = 1;
    while (head < tail) {
        int32_t s = bfs[size_t(head++)];
        for (int32_t e = ch_off[size_t(s)]; e < ch_off[size_t(s) + 1]; ++e) {
            int32_t t = ch[size_t(e)];
            newid[size_t(t)] = int32_t(tail);
            bfs[size_t(tail++)] = t;
        }
    }
    P.depth.resize(size_t(S));
    P.first_child.assign(size_t(S), 0);
    P.n_child.assign(size_t(S), 0);
    P.label.assign(size_t(S), 0);
    for (int32_t i = 0; i < S; ++i) {
        int32_t s = bfs[size_t(i)];
        P.depth[size_t(i)] = cdepth[size_t(s)];
        P.label[size_t(i)] = clabel[size_t(s)];
        int32_t nc = ch_off[size_t(s) + 1] - ch_off[size_t(s)];
        P.n_child[size_t(i)] = nc;
        P.first_child[size_t(i)] = nc ? newid[size_t(ch[size_t(ch_off[size_t(s)])])] : 0;
    }

    // ---- Output lists: keyword ids per state, ascending -------------------
    P.out_off.assign(size_t(S) + 1, 0);
    for (int32_t p = 0; p < n; ++p) P.out_off[size_t(newid[size_t(terminal[p])]) + 1]++;
    for (int32_t s = 0; s < S; ++s) P.out_off[size_t(s) + 1] += P.out_off[size_t(s)];
    P.out_pid.resize(size_t(n));
    {
        std::vector<int32_t> fill(P.out_off.begin(), P.out_off.end() - 1);
        for (int32_t p = 0; p < n; ++p) P.out_pid[size_t(fill[size_t(newid[size_t(terminal[p])])]++)] = p;
    }
    auto is_final = [&](int32_t s) { return P.out_off[size_t(s) + 1] > P.out_off[size_t(s)]; };

    // ---- alphabet compression ---------------------------------------------
    bool used[256] = {};
    for (int32_t p = 0; p < n; ++p)
        for (int64_t j = 0; j < P.kw_len[p]; ++j) used[kw(p)[j]] = true;
    int n_used = 0;
    for (int b = 0; b < 256; ++b) n_used += used[b];
    if (n_used == 256) {
        P.C = 256;
        for (int b = 0; b < 256; ++b) P.cls[b] = uint8_t(b);
    } else {
        P.C = n_used + 1;                       // class 0 = bytes in no keyword
        int c = 1;
        for (int b = 0; b < 256; ++b) P.cls[b] = used[b] ? uint8_t(c++) : 0;
    }

    // ---- dense rows for the shallow states, compact nodes below ------------
    const int64_t row_bytes = int64_t(P.C) * 4;
    int32_t D = 0, S_dense = 1;
    {
        // states are depth-sorted: count states per depth
        int32_t maxd = P.depth[size_t(S - 1)];
        std::vector<int64_t> upto(size_t(maxd) + 1, 0);
        for (int32_t i = 0; i < S; ++i) upto[size_t(P.depth[size_t(i)])]++;
        int64_t acc = 0;
        for (int32_t d = 0; d <= maxd; ++d) {
            acc += upto[size_t(d)];
            if (d == 0 || acc * row_bytes <= dense_budget) {
                D = d;
                S_dense = int32_t(acc);
            } else {
                break;
            }
        }
    }
    P.dense_depth = D;
    P.S_dense = S_dense;
    P.dense.assign(size_t(S_dense) * size_t(P.C), 0);
    for (int32_t s = 0; s < S_dense; ++s) {
        for (int32_t k = 0; k < P.n_child[size_t(s)]; ++k) {
            int32_t t = P.first_child[size_t(s)] + k;
            int32_t e = t | (is_final(t) ? kFinalBit : 0);
            P.dense[size_t(s) * size_t(P.C) + P.cls[P.label[size_t(t)]]] = e;
        }
    }
    P.node.assign(size_t(S - S_dense) * 2, 0);
    for (int32_t s = S_dense; s < S; ++s) {
        size_t i = size_t(s - S_dense) * 2;
        P.node[i] = P.first_child[size_t(s)];
        P.node[i + 1] = P.n_child[size_t(s)] | (is_final(s) ? kFinalBit : 0);
    }

    // ---- candidate filters over the first K bytes of every keyword --------
    std::vector<uint32_t> prefixes(static_cast<size_t>(n));
    for (int32_t p = 0; p < n; ++p) {
        uint32_t x = 0;
        for (int j = 0; j < P.K; ++j) x |= uint32_t(kw(p)[j]) << (8 * j);
        prefixes[size_t(p)] = x;
    }
    std::sort(prefixes.begin(), prefixes.end());
    prefixes.erase(std::unique(prefixes.begin(), prefixes.end()), prefixes.end());
    P.n_prefixes = int32_t(prefixes.size());
    // windows for the sampled filters: bytes [j, j + 3) of each keyword for
    // j = 1, 2 (stride 2, keywords of 5 bytes or more) and j = 1 .. 4 (stride
    // 4, 7 bytes or more)
    auto windows_of = [&](int count) {
        std::vector<uint32_t> w;
        w.reserve(size_t(n) * size_t(count));
        for (int32_t p = 0; p < n; ++p) {
            const uint8_t *k = kw(p);
            for (int j = 1; j <= count; ++j)
                w.push_back(uint32_t(k[j]) | uint32_t(k[j + 1]) << 8 | uint32_t(k[j + 2]) << 16);
        }
        std::sort(w.begin(), w.end());
        w.erase(std::unique(w.begin(), w.end()), w.end());
        return w;
    };
    P.sampled = P.K == 3 && P.min_len >= 5;
    P.sampled4 = P.K == 3 && P.min_len >= 7;
    const std::vector<uint32_t> windows = P.sampled ? windows_of(2) : std::vector<uint32_t>();
    const std::vector<uint32_t> windows4 = P.sampled4 ? windows_of(4) : std::vector<uint32_t>();
    P.n_windows2 = int32_t(windows.size());
    P.n_windows4 = int32_t(windows4.size());
    // 4-byte windows at positions 1 .. count (keywords of count + 4 bytes or more)
    auto quads_of = [&](int count) {
        std::vector<uint32_t> w;
        w.reserve(size_t(n) * size_t(count));
        for (int32_t p = 0; p < n; ++p) {
            const uint8_t *k = kw(p);
            for (int j = 1; j <= count; ++j)
                w.push_back(uint32_t(k[j]) | uint32_t(k[j + 1]) << 8 | uint32_t(k[j + 2]) << 16 |
                            uint32_t(k[j + 3]) << 24);
        }
        std::sort(w.begin(), w.end());
        w.erase(std::unique(w.begin(), w.end()), w.end());
        return w;
    };
    P.pair2 = P.K == 3 && P.min_len >= 6;
    P.pair4 = P.K == 3 && P.min_len >= 8;
    const std::vector<uint32_t> quads2 = P.pair2 ? quads_of(2) : std::vector<uint32_t>();
    const std::vector<uint32_t> quads4 = P.pair4 ? quads_of(4) : std::vector<uint32_t>();
    P.n_quads2 = int32_t(quads2.size());
    P.n_quads4 = int32_t(quads4.size());
    // A key x with hash h = x * mul (mod 2^32) owns bit h mod 32 of word (or
    // byte) h >> shift.  The sampled kernels hash x * mul + c with 0 <= c <
    // 32, which may carry into the index: those maps also set the key's bit
    // at index (h + 31) >> shift, so every c finds it.
    for (int set = 0; set < 3; ++set) {
        const std::vector<uint32_t> &keys = set == 0 ? prefixes : set == 1 ? windows : windows4;
        const uint32_t carry = set == 0 ? 0u : 31u;
        for (int kind = 1; kind <= kNumFilterKinds; ++kind) {
            FilterGeom g = filter_geom(kind);
            std::vector<uint8_t> &f = P.filter[set * kNumFilterKinds + kind - 1];
            if ((set == 1 && !P.sampled) || (set == 2 && !P.sampled4)) { f.clear(); continue; }
            if (g.pair) {
                // 4-byte window x: bits h mod 32 and (x >> 24) mod 32 of word h >> shift,
                // h the hash of its first three bytes (the kernel adds nothing to h);
                // the stride-2 map also sets bit (x >> 16) mod 32
                const bool have = (set == 1 && P.pair2) || (set == 2 && P.pair4);
                if (!have) { f.clear(); continue; }
                f.assign(size_t(g.bytes), 0);
                for (uint32_t x : set == 1 ? quads2 : quads4) {
                    const uint32_t h = prefix_hash(x & 0xFFFFFFu, mul);
                    const size_t w = size_t(h >> g.shift) * 4;
                    const uint32_t third = set == 1 ? (x >> 16) & 31u : h & 31u;
                    for (uint32_t bit : {h & 31u, (x >> 24) & 31u, third}) f[w + bit / 8] |= uint8_t(1u << (bit % 8));
                }
                continue;
            }
            f.assign(size_t(g.bytes), 0);
            // one bit map of `words` 32-bit words starting at byte `at`
            auto set_bit = [&](size_t at, uint32_t h, int shift) {
                const uint32_t bit = h & 31u;
                for (uint32_t hh : {h, h + carry}) {
                    const uint32_t w = hh >> shift;
                    f[at + size_t(w) * 4 + bit / 8] |= uint8_t(1u << (bit % 8));
                }
            };
            for (uint32_t x : keys) {
                const uint32_t h = prefix_hash(x, mul);
                if (g.dual) {   // map A, then map B with its own hash: both halves of the bytes
                    set_bit(0, h, g.shift);
                    set_bit(size_t(g.bytes / 2), prefix_hash(x, kFilterMul2), g.shift);
                } else if (g.bitmap) {
                    set_bit(0, h, g.shift);
                } else {
                    f[size_t(h >> g.shift)] = 1;
                    f[size_t((h + carry) >> g.shift)] = 1;
                }
            }
        }
    }

    // ---- exact prefix table: K-byte prefix -> state at depth K ------------
    // Two-choice cuckoo table of 2^bits slots in buckets of 4, at most half
    // full: every prefix lies in one of its two buckets, so a lookup reads
    // two buckets and never probes further.  Slot = {key, value}:
    //   key   = prefix (24 bits) | next byte << 24
    //   value = state | has-next << 30 | final << 31, 0 for an empty slot.
    // When the state has exactly one child, "next byte" is that child's edge
    // byte and has-next is set: an offset whose following byte differs
    // cannot match deeper than the prefix.
    {
        std::vector<std::pair<uint32_t, uint32_t>> items;   // (key, value), one per prefix
        items.reserve(size_t(P.n_prefixes));
        std::vector<uint32_t> seen;
        for (int32_t p = 0; p < n; ++p) {
            uint32_t x = 0;
            for (int j = 0; j < P.K; ++j) x |= uint32_t(kw(p)[j]) << (8 * j);
            seen.push_back(x);
        }
        std::sort(seen.begin(), seen.end());
        seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
        for (uint32_t x : seen) {
            int32_t s = 0;   // follow the trie for K bytes
            for (int j = 0; j < P.K; ++j) {
                const uint8_t b = uint8_t(x >> (8 * j));
                int32_t lo = P.first_child[size_t(s)], hi = lo + P.n_child[size_t(s)];
                while (lo < hi && P.label[size_t(lo)] != b) ++lo;
                s = lo;
            }
            uint32_t key = x, val = uint32_t(s) | (is_final(s) ? 0x80000000u : 0u);
            if (P.n_child[size_t(s)] == 1) {
                key |= uint32_t(P.label[size_t(P.first_child[size_t(s)])]) << 24;
                val |= 0x40000000u;
            }
            items.emplace_back(key, val);
        }
        int bits = 6;
        while ((int64_t(1) << bits) < 2 * int64_t(P.n_prefixes)) ++bits;
        while (!build_cuckoo(items, bits, mul, P.ptab)) ++bits;
        P.ptab_bits = bits;
    }

    // ---- unary tails: state -> leaf when the rest of the path is forced -----
    // tail[s] = leaf l when every state from s down to l has one child and no
    // state strictly between s and l ends a keyword; the remaining bytes can
    // then be compared with the leaf's keyword in one pass.  -1 otherwise.
    P.tail.assign(size_t(S), -1);
    for (int32_t s = S - 1; s >= 0; --s) {
        const int32_t nc = P.n_child[size_t(s)];
        if (nc == 0) {
            P.tail[size_t(s)] = s;
        } else if (nc == 1) {
            const int32_t c = P.first_child[size_t(s)];
            if (P.n_child[size_t(c)] == 0) P.tail[size_t(s)] = c;
            else if (!is_final(c)) P.tail[size_t(s)] = P.tail[size_t(c)];
        }
    }
    // Unary chains that do not end at a leaf: chain[s] = the first state
    // below s that ends a keyword or has other than one child, when s has
    // one child (else -1); rep[s] = a keyword whose path passes through s
    // down to a leaf (so it spells every chain below s).
    std::vector<int32_t> chain(size_t(S), -1), rep(size_t(S), -1);
    for (int32_t s = S - 1; s >= 0; --s) {
        const int32_t nc = P.n_child[size_t(s)];
        rep[size_t(s)] = nc > 0 ? rep[size_t(P.first_child[size_t(s)])] : P.out_pid[size_t(P.out_off[size_t(s)])];
        if (nc == 1) {
            const int32_t c = P.first_child[size_t(s)];
            chain[size_t(s)] = (is_final(c) || P.n_child[size_t(c)] != 1) ? c : chain[size_t(c)];
        }
    }
    // per state, everything one step of a walk needs in one 16-byte record:
    // {leaf, position in kw_bytes of the first byte below s, bytes from s
    // down to the leaf, leaf's only keyword id + 1 or 0} when tail[s] is a
    // deeper leaf; {-3, position in kw_bytes of the first byte below s,
    // bytes from s down to c, c} when s starts a unary chain of two or more
    // bytes to a state c that ends a keyword or branches (no state strictly
    // between ends one); {-2, 0, 0, 0} when s is itself a leaf; {-1, first
    // child, child count, 0} otherwise.  Bit 31 of the last field is set
    // when a keyword ends at s.
    P.tailinfo.assign(size_t(S) * 4, 0);
    for (int32_t s = 0; s < S; ++s) {
        const int32_t t = P.tail[size_t(s)];
        int32_t *ti = &P.tailinfo[size_t(s) * 4];
        const int32_t c = chain[size_t(s)];
        if (t < 0 && c >= 0 && P.depth[size_t(c)] - P.depth[size_t(s)] >= 2) {
            const int32_t p = rep[size_t(s)];
            ti[0] = -3;
            ti[1] = int32_t(offsets[p] - offsets[0]) + P.depth[size_t(s)];
            ti[2] = P.depth[size_t(c)] - P.depth[size_t(s)];
            ti[3] = c;
        } else if (t < 0) {
            ti[0] = -1;
            ti[1] = P.first_child[size_t(s)];
            ti[2] = P.n_child[size_t(s)];
        } else if (t == s) {
            ti[0] = -2;
        } else {
            const int32_t p = P.out_pid[size_t(P.out_off[size_t(t)])];
            ti[0] = t;
            ti[1] = int32_t(offsets[p] - offsets[0]) + P.depth[size_t(s)];
            ti[2] = P.depth[size_t(t)] - P.depth[size_t(s)];
            // the leaf's keyword id + 1 when exactly one keyword ends there
            ti[3] = P.out_off[size_t(t) + 1] - P.out_off[size_t(t)] == 1 ? p + 1 : 0;
        }
        if (is_final(s)) ti[3] = int32_t(uint32_t(ti[3]) | kFinalBit);
    }
    // keyword bytes (for tail comparisons) with int32 offsets
    P.kw_bytes.assign(bytes + offsets[0], bytes + offsets[0] + total);
    P.kw_off.resize(size_t(n) + 1);
    for (int32_t p = 0; p <= n; ++p) P.kw_off[size_t(p)] = int32_t(offsets[p] - offsets[0]);

    P.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return AC_OK;
}

}  // namespace pfac
