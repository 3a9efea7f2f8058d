"""Host-side checks of the GPU library's automaton builder (no GPU needed).

``ac_compile`` runs every host step of ``ac_build``; its tables are exported
and walked here by a small test-side walker to check the invariants the
kernels rely on.  The CPU oracle is not involved: these are properties of the
built tables themselves (trie size, keyword paths, layouts, prefix table,
forced-path tails, filters), plus the C-ABI surface.
"""

import ctypes
import dataclasses
import os
import re

import numpy as np
import pytest

import paper_1412_7789_amd as pf
from paper_1412_7789_amd import _lib as L
from workloads import SPECS, make_keywords

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not os.path.exists(pf.LIB_PATH):
        from paper_1412_7789_amd.build import build
        build()
    return pf.load()


def declared_functions(header="pfac.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ac_[a-z_0-9]+)\s*\(", src)))


@pytest.mark.parametrize("header,exports", [("pfac.h", L.EXPORTS), ("pfac_serve.h", L.SERVE_EXPORTS)])
def test_every_declared_symbol_is_exported(lib, header, exports):
    names = declared_functions(header)
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(exports) == names


class Tables:
    def __init__(self, kws, budget=0):
        self.plan = pf.Plan(kws, dense_budget_bytes=budget)
        self.info = self.plan.info()
        e = self.plan.export
        self.cls = e(L.AC_TABLE_CLASS_MAP, np.uint8)
        self.dense = e(L.AC_TABLE_DENSE, np.int32)
        self.node = e(L.AC_TABLE_NODE, np.int32)
        self.label = e(L.AC_TABLE_LABEL, np.uint8)
        self.out_off = e(L.AC_TABLE_OUT_OFF, np.int32)
        self.out_pid = e(L.AC_TABLE_OUT_PID, np.int32)
        self.depth = e(L.AC_TABLE_DEPTH, np.int32)
        self.ptab = e(L.AC_TABLE_PREFIX, np.uint32)
        self.tail = e(L.AC_TABLE_TAIL, np.int32)
        self.tailinfo = e(L.AC_TABLE_TAIL_INFO, np.int32).reshape(-1, 4)
        self.C = self.info["n_classes"]
        self.S = self.info["n_states"]
        self.Sd = self.info["n_dense_states"]

    def step(self, s, b):
        """(next state, final) or None, read from the built layout."""
        if s < self.Sd:
            e = int(self.dense[s * self.C + int(self.cls[b])])
            if e == 0:
                return None
            return e & 0x7FFFFFFF, e < 0
        r = s - self.Sd
        fc, nc = int(self.node[2 * r]), int(self.node[2 * r + 1]) & 0x7FFFFFFF
        for t in range(fc, fc + nc):
            if self.label[t] == b:
                return t, int(self.node[2 * (t - self.Sd) + 1]) < 0
        return None

    def children(self, s):
        return [t for b in range(256) for t in [self.step(s, b)] if t is not None]

    def outputs(self, s):
        return self.out_pid[self.out_off[s]:self.out_off[s + 1]].tolist()


def kw_sets():
    rng = np.random.default_rng(2)
    yield "fig4", [b"AB", b"ABG", b"BEDE", b"ED"]
    yield "nested", [b"a", b"ab", b"abc", b"bc", b"c", b"abc"]
    yield "chains", [b"abcdefghij", b"abcdefghXY", b"abcde", b"abcdefghijklmnop", b"zz1", b"zzzzzzzzzzzz2"]
    yield "tiny", make_keywords(SPECS["tiny"], np.random.default_rng(0), np.random.default_rng(1))
    yield "bytes", [bytes(rng.integers(0, 256, size=int(L), dtype=np.uint8)) for L in rng.integers(1, 9, size=300)]
    yield "shared", make_keywords(dataclasses.replace(SPECS["large"], n=500),
                                  np.random.default_rng(3), np.random.default_rng(4))


@pytest.mark.parametrize("name,kws", list(kw_sets()))
@pytest.mark.parametrize("budget", [0, 1])
def test_trie_paths_outputs_and_layouts(name, kws, budget):
    T = Tables(kws, budget)
    prefixes = {k[:i] for k in kws for i in range(len(k) + 1)}
    assert T.S == len(prefixes)
    if budget == 1:
        assert T.Sd == 1          # only the root row is dense; every other state is compact
    # each keyword's path ends at a state whose outputs contain its id
    for p, k in enumerate(kws):
        s = 0
        for j, b in enumerate(k):
            nxt = T.step(s, b)
            assert nxt is not None, (name, p, j)
            s, fin = nxt
            assert fin == (k[:j + 1] in set(kws))
        assert p in T.outputs(s)
        assert T.depth[s] == len(k)
    # outputs partition the ids, ascending per state
    allp = sorted(T.out_pid.tolist())
    assert allp == list(range(len(kws)))
    for s in range(T.S):
        o = T.outputs(s)
        assert o == sorted(o)
    # breadth-first numbering: depths non-decreasing
    assert (np.diff(T.depth) >= 0).all()


def test_dense_and_compact_layouts_agree():
    rng = np.random.default_rng(9)
    kws = [bytes(rng.integers(97, 101, size=int(L), dtype=np.uint8)) for L in rng.integers(1, 10, size=200)]
    full, compact = Tables(kws, 0), Tables(kws, 1)
    assert full.Sd == full.S and compact.Sd == 1
    for s in range(full.S):
        for b in list(range(96, 102)) + [0, 255]:
            assert full.step(s, b) == compact.step(s, b), (s, b)


def test_class_map():
    T = Tables([b"abc", b"zz"])
    used = {ord(c) for c in "abcz"}
    assert T.C == len(used) + 1
    assert sorted(int(T.cls[b]) for b in used) == list(range(1, len(used) + 1))
    assert all(T.cls[b] == 0 for b in range(256) if b not in used)
    T = Tables([bytes([b]) for b in range(256)])
    assert T.C == 256 and (T.cls == np.arange(256)).all()


@pytest.mark.parametrize("name,kws", list(kw_sets()))
def test_prefix_table_and_tails(name, kws):
    T = Tables(kws)
    K = T.info["prefix_len"]
    assert K == min(3, min(len(k) for k in kws))

    def walk(prefix):
        s = 0
        for b in prefix:
            nxt = T.step(s, b)
            if nxt is None:
                return None
            s = nxt[0]
        return s

    slots = len(T.ptab) // 2
    assert slots & (slots - 1) == 0 and 2 * T.info["n_prefixes"] <= slots
    occupied = [(int(T.ptab[2 * i]), int(T.ptab[2 * i + 1])) for i in range(slots) if T.ptab[2 * i + 1]]
    assert len(occupied) == T.info["n_prefixes"]          # each prefix stored once

    def lookup(x):
        """(key, value) of x's slot in its two buckets; value 0 when absent."""
        b1, b2 = T.plan.prefix_buckets(x)
        assert b1 != b2 and max(b1, b2) < slots // 4
        for b in (b1, b2):
            for j in range(4):
                k, v = int(T.ptab[2 * (4 * b + j)]), int(T.ptab[2 * (4 * b + j) + 1])
                if v and (k & 0xFFFFFF) == x:
                    return k, v
        return 0, 0

    keyset = set(kws)
    pref = {k[:K] for k in kws}
    assert T.info["n_prefixes"] == len(pref)
    for pr in pref:
        x = int.from_bytes(pr, "little")
        k, v = lookup(x)
        s = walk(pr)
        assert v & 0x3FFFFFFF == s
        assert bool(v >> 31) == (pr in keyset)
        ch = T.children(s)
        # has-next flag and the single child's byte
        assert bool(v & 0x40000000) == (len(ch) == 1)
        if len(ch) == 1:
            assert k >> 24 == [b for b in range(256) if T.step(s, b) is not None][0]
    # values that start no keyword are absent
    rng = np.random.default_rng(1)
    for x in rng.integers(0, 1 << (8 * K), size=2000):
        pr = int(x).to_bytes(K, "little")
        if pr not in pref:
            assert lookup(int(x))[1] == 0
    # tails: tail[s] = leaf reached by a forced path with no keyword ending strictly between
    for s in range(T.S):
        path, t = [s], s
        while True:
            ch = T.children(t)
            if len(ch) != 1:
                break
            t, fin = ch[0]
            path.append(t)
            if fin and T.children(t):
                t = None
                break
        leaf = t if (t is not None and not T.children(t)) else None
        assert T.tail[s] == (leaf if leaf is not None else -1), s
        ti = T.tailinfo[s]
        # bit 31 of the last field: a keyword ends at s
        assert (int(ti[3]) < 0) == bool(T.outputs(s)), s
        only = int(ti[3]) & 0x7FFFFFFF
        if leaf is None:
            # not forced: a unary chain of two or more bytes to a state that
            # ends a keyword or branches, else the children
            chain, c = b"", s
            while len(T.children(c)) == 1:
                c, fin = T.children(c)[0]
                chain += bytes([int(T.label[c])])
                if fin or len(T.children(c)) != 1:
                    break
            if len(chain) >= 2:
                flat = b"".join(kws)
                assert ti[0] == -3 and only == int(c) and ti[2] == len(chain), s
                assert flat[ti[1]:ti[1] + ti[2]] == chain, s
            else:
                ch = sorted(t for t, _ in T.children(s))
                assert ti[0] == -1 and ch == list(range(int(ti[1]), int(ti[1]) + int(ti[2]))), s
                assert only == 0
        elif leaf == s:
            assert ti[0] == -2 and ti[1] == 0 and ti[2] == 0 and only == 0
        else:
            assert ti[0] == leaf and ti[2] == len(path) - 1
            ids = T.out_pid[T.out_off[leaf]:T.out_off[leaf + 1]]
            assert only == (ids[0] + 1 if len(ids) == 1 else 0)
            # the keyword bytes at ti[1] spell the path below s
            kw = kws[ids[0]]
            d = int(T.depth[s])
            flat = b"".join(kws)
            assert flat[ti[1]:ti[1] + ti[2]] == kw[d:d + ti[2]]


def test_filters_have_no_false_negatives():
    """Every key of each filter set is present in every map of that set:
    K-byte prefixes (stride 1), windows [1,4) and [2,5) (stride 2) and
    windows [1,4) .. [4,7) (stride 4).  A key with hash h owns bit h mod 32
    of word h >> shift; the sampled maps set it at index (h + 31) >> shift
    too, since their kernels add up to 31 to the hash before indexing."""
    kws = make_keywords(SPECS["sweep"], np.random.default_rng(0), np.random.default_rng(1))
    T = Tables(kws)
    K = T.info["prefix_len"]
    assert K == 3
    geoms = {1: (False, 17), 2: (True, 17), 3: (False, 16), 4: (True, 16)}
    key_sets = {0: {k[:K] for k in kws},
                1: {k[j:j + 3] for k in kws for j in (1, 2)},
                2: {k[j:j + 3] for k in kws for j in (1, 2, 3, 4)}}
    assert T.info["n_windows2"] == len(key_sets[1])
    assert T.info["n_windows4"] == len(key_sets[2])
    M32 = 0xFFFFFFFF
    for set_, keys in key_sets.items():
        carries = (0,) if set_ == 0 else (0, 31)
        for kind, (bitmap, flog2) in geoms.items():
            f = T.plan.export(L.AC_TABLE_FILTER_BASE + 6 * set_ + kind, np.uint8)
            assert len(f) == 1 << flog2
            for key in keys:
                h = T.plan.hash(int.from_bytes(key, "little"))
                for c in carries:
                    hc = (h + c) & M32
                    if bitmap:
                        w = f.view(np.uint32)[hc >> (32 - (flog2 - 2))]
                        assert (int(w) >> (h & 31)) & 1
                    else:
                        assert f[hc >> (32 - flog2)] == 1
        # dual map: 2^19 bits hashed as `hash`, then 2^19 bits hashed as `hash2`
        f = T.plan.export(L.AC_TABLE_FILTER_BASE + 6 * set_ + L.AC_FILTER_DUAL19, np.uint8).view(np.uint32)
        assert len(f) == 2 << 14
        for key in keys:
            x = int.from_bytes(key, "little")
            h1, h2 = T.plan.hash(x), T.plan.hash2(x)
            assert h1 != h2 or x == 0
            for c in carries:
                assert (int(f[((h1 + c) & M32) >> 18]) >> (h1 & 31)) & 1
                assert (int(f[(1 << 14) + (((h2 + c) & M32) >> 18)]) >> (h2 & 31)) & 1


def test_rotated_bit_test_finds_every_key():
    """The sampled kernels test key x for destination bit b by hashing p =
    x * mul + c with c = -b mod 32, reading word p >> shift and rotating it
    right by p mod 32: the key's bit must land on bit b, for every b they
    use (0 .. 14 at stride 2, 0, 4, 8, 12 at stride 4)."""
    kws = make_keywords(SPECS["sweep"], np.random.default_rng(0), np.random.default_rng(1))
    T = Tables(kws)
    words = T.plan.export(L.AC_TABLE_FILTER_BASE + 6 * 1 + L.AC_FILTER_BITS20, np.uint8).view(np.uint32)
    M32 = 0xFFFFFFFF
    rot = lambda v, r: ((v >> r) | (v << (32 - r))) & M32 if r else v
    for key in sorted({k[j:j + 3] for k in kws for j in (1, 2)})[:500]:
        h = T.plan.hash(int.from_bytes(key, "little"))
        for b in range(0, 16, 2):
            p = (h + ((32 - b) & 31)) & M32
            assert (rot(int(words[p >> 17]), p & 31) >> b) & 1


def test_pair_map_holds_both_bits_of_every_4_byte_window():
    """AC_FILTER_PAIR20 (strides 2 and 4): every 4-byte window x at keyword
    positions 1 .. stride owns bits h mod 32 and (x >> 24) mod 32 of word
    h >> 17, h the hash of its first three bytes, and at stride 2 also bit
    (x >> 16) mod 32; no such map at stride 1."""
    kws = make_keywords(SPECS["sweep"], np.random.default_rng(0), np.random.default_rng(1))
    T = Tables(kws)
    quads = {k[j:j + 4] for k in kws for j in (1, 2, 3, 4)}
    assert T.info["n_quads4"] == len(quads)
    words = T.plan.export(L.AC_TABLE_FILTER_BASE + 12 + L.AC_FILTER_PAIR20, np.uint8).view(np.uint32)
    assert len(words) == 1 << 15
    for q in quads:
        x = int.from_bytes(q, "little")
        h = T.plan.hash(x & 0xFFFFFF)
        w = int(words[h >> 17])
        assert (w >> (h & 31)) & 1 and (w >> ((x >> 24) & 31)) & 1
    # bits set: at most two per window
    assert sum(bin(int(v)).count("1") for v in words) <= 2 * len(quads)
    # stride 2: the 4-byte windows at positions 1 and 2, the same layout
    quads2 = {k[j:j + 4] for k in kws for j in (1, 2)}
    assert T.info["n_quads2"] == len(quads2)
    words2 = T.plan.export(L.AC_TABLE_FILTER_BASE + 6 + L.AC_FILTER_PAIR20, np.uint8).view(np.uint32)
    assert len(words2) == 1 << 15
    for q in quads2:
        x = int.from_bytes(q, "little")
        h = T.plan.hash(x & 0xFFFFFF)
        w = int(words2[h >> 17])
        assert (w >> (h & 31)) & 1 and (w >> ((x >> 24) & 31)) & 1 and (w >> ((x >> 16) & 31)) & 1
    assert sum(bin(int(v)).count("1") for v in words2) <= 3 * len(quads2)
    # and no bit a window does not own: rebuilt from the windows, the map is the same
    rebuilt = np.zeros(1 << 15, dtype=np.uint32)
    for q in quads2:
        x = int.from_bytes(q, "little")
        h = T.plan.hash(x & 0xFFFFFF)
        rebuilt[h >> 17] |= np.uint32((1 << (h & 31)) | (1 << ((x >> 24) & 31)) | (1 << ((x >> 16) & 31)))
    assert np.array_equal(rebuilt, words2)
    assert len(T.plan.export(L.AC_TABLE_FILTER_BASE + L.AC_FILTER_PAIR20, np.uint8)) == 0
    # keywords shorter than 8 bytes: no stride-4 map; shorter than 6: no stride-2 map
    T7 = Tables([b"abcdefg", b"bcdefghij"])
    assert T7.info["n_quads4"] == 0 and T7.info["n_windows4"] > 0 and T7.info["n_quads2"] > 0
    T5 = Tables([b"abcde", b"bcdefghij"])
    assert T5.info["n_quads2"] == 0 and T5.info["n_windows2"] > 0
    assert len(T5.plan.export(L.AC_TABLE_FILTER_BASE + 6 + L.AC_FILTER_PAIR20, np.uint8)) == 0


def test_sampled_filters_need_long_enough_keywords():
    T = Tables([b"abcdef", b"bcdefg"])         # shortest 6: stride 2 only
    assert T.info["n_windows2"] > 0 and T.info["n_windows4"] == 0
    assert len(T.plan.export(L.AC_TABLE_FILTER_BASE + 12 + L.AC_FILTER_BITS19, np.uint8)) == 0
    T = Tables([b"abcdefg", b"bcdefgh"])       # shortest 7: both
    assert T.info["n_windows2"] > 0 and T.info["n_windows4"] > 0
    T = Tables([b"abcd", b"abcdef"])           # shortest 4: neither
    assert T.info["n_windows2"] == 0 and T.info["n_windows4"] == 0


def test_build_errors(lib):
    with pytest.raises(pf.PfacError):
        pf.Plan([b"a", b""])
    h = ctypes.c_void_p()
    assert lib.ac_compile(None, None, 0, None, ctypes.byref(h)) == L.AC_EINVAL
    assert b"keyword" in lib.ac_last_error()
    # a NULL automaton is rejected before any GPU call
    assert lib.ac_match(None, None, 0, None, None) == L.AC_EINVAL
