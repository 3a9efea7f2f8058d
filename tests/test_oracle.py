"""Pins for the CPU oracle (serial Aho-Corasick, paper Section II).

The oracle is checked against things other than itself:

* the brute-force definition of the result on many random tiny inputs,
* the hand-derived Fig. 4 machine and a worked scan (tests/golden),
* closed forms (runs of one byte, self-overlap, whole-text keywords, every
  single-byte keyword, the paper's own permutation workload of Section III),
* invariants on a full 1 MiB workload (soundness, planted completeness and
  per-keyword counts from the library substring search).
"""

import os
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import Oracle, brute_match, find_all, oracle_match
from workloads import config_tiny, paper_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pairs(res):
    off, pid = res
    return list(zip(off.tolist(), pid.tolist()))


def load_fig4():
    kws, fails, outs, matches, text, n_states = {}, {}, {}, [], None, None
    with open(os.path.join(GOLDEN, "fig4_machine.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "keyword":
                kws[int(tok[1])] = tok[2].encode()
            elif tok[0] == "states":
                n_states = int(tok[1])
            elif tok[0] == "fail":
                fails[tok[1]] = "" if tok[2] == "-" else tok[2]
            elif tok[0] == "out":
                outs[tok[1]] = [int(t) for t in tok[2:]]
            elif tok[0] == "text":
                text = tok[1].encode()
            elif tok[0] == "match":
                matches.append((int(tok[1]), int(tok[2])))
    return [kws[i] for i in range(len(kws))], n_states, fails, outs, text, matches


def test_fig4_machine_goto_failure_output(oracle_lib):
    kws, n_states, fails, outs, _, _ = load_fig4()
    o = Oracle(kws)
    assert o.n_states == n_states
    for s_str, f_str in fails.items():
        s = o.state_of(s_str.encode())
        f = 0 if f_str == "" else o.state_of(f_str.encode())
        assert s > 0 and f >= 0
        assert o.fail(s) == f, s_str
    for s_str in fails:
        s = o.state_of(s_str.encode())
        assert sorted(o.output(s)) == sorted(outs.get(s_str, [])), s_str
    # g(0, a) is total: bytes without a root edge loop to the root
    assert o.goto(0, ord("Z")) == 0
    # g(s, a) undefined away from the root
    assert o.goto(o.state_of(b"AB"), ord("Z")) == -1


def test_fig4_worked_scan(oracle_lib):
    kws, _, _, _, text, matches = load_fig4()
    assert pairs(oracle_match(kws, text)) == matches
    assert pairs(brute_match(kws, text)) == matches


def test_closed_forms(oracle_lib):
    # c^L in c^N: N - L + 1 overlapping occurrences
    for L, N in [(1, 1), (1, 7), (3, 10), (5, 5), (6, 5)]:
        off, pid = oracle_match([b"c" * L], b"c" * N)
        assert off.tolist() == list(range(max(0, N - L + 1)))
    # self-overlap
    assert pairs(oracle_match([b"abab"], b"ababab")) == [(0, 0), (2, 0)]
    # keyword equal to the whole text, and longer than the text
    assert pairs(oracle_match([b"xyz", b"hello"], b"hello")) == [(0, 1)]
    assert pairs(oracle_match([b"hello!"], b"hello")) == []
    # empty text
    assert pairs(oracle_match([b"a"], b"")) == []
    # nested prefixes and suffixes all reported at every offset
    kws = [b"a", b"ab", b"abc", b"bc", b"c"]
    assert pairs(oracle_match(kws, b"abc")) == [(0, 0), (0, 1), (0, 2), (1, 3), (2, 4)]
    # duplicates: every id is reported
    assert pairs(oracle_match([b"ab", b"ab"], b"abab")) == [(0, 0), (0, 1), (2, 0), (2, 1)]


def test_every_single_byte_keyword(oracle_lib):
    rng = np.random.default_rng(7)
    text = rng.integers(0, 256, size=5000, dtype=np.uint8)
    text[:2] = [0x00, 0xFF]
    kws = [bytes([b]) for b in range(256)]
    off, pid = oracle_match(kws, text)
    assert off.tolist() == list(range(len(text)))
    assert pid.tolist() == text.astype(np.int32).tolist()


def test_empty_keyword_rejected(oracle_lib):
    with pytest.raises(ValueError):
        Oracle([b"a", b""])


def test_paper_permutation_workload_closed_form(oracle_lib):
    """Section III: permutations of a..z as keywords, the alphabet written
    repeatedly as text.  With 131-byte lines (alphabet x5 + newline) the
    identity occurs at 131 j + 26 t (t = 0..4), a rotation by r at
    131 j + 26 t + r (t = 0..3), any other permutation nowhere."""
    m = 125                                  # 16,375 bytes: the paper's first size
    w = paper_workload(5, m)
    assert len(w.text) == 16375
    rot = bytes(b"abcdefghijklmnopqrstuvwxyz"[3:] + b"abc")
    kws = list(w.keywords) + [rot]
    off, pid = oracle_match(kws, w.text)
    got = {p: sorted(off[pid == p].tolist()) for p in range(len(kws))}
    assert got[0] == sorted(131 * j + 26 * t for j in range(m) for t in range(5))
    assert got[len(kws) - 1] == sorted(131 * j + 26 * t + 3 for j in range(m) for t in range(4))
    for p in range(1, len(kws) - 1):
        k = kws[p]
        is_rotation = k in (b"abcdefghijklmnopqrstuvwxyz" * 2)
        assert len(got[p]) == (4 * m if is_rotation else 0)
    assert len(off) == 5 * m + 4 * m


def _check_random_case(rng, alphabet, n_kw, max_len, n_text):
    kws = []
    for _ in range(n_kw):
        L = rng.randint(1, max_len)
        kws.append(bytes(rng.choice(alphabet) for _ in range(L)))
    text = bytes(rng.choice(alphabet) for _ in range(n_text))
    # plant a few keyword copies so that matches are not all accidental
    text = bytearray(text)
    for _ in range(rng.randint(0, 4)):
        k = rng.choice(kws)
        if len(k) <= len(text):
            o = rng.randint(0, len(text) - len(k))
            text[o:o + len(k)] = k
    text = bytes(text)
    assert pairs(oracle_match(kws, text)) == pairs(brute_match(kws, text)), (kws, text)


@pytest.mark.parametrize("alphabet_size", [2, 4, 26, 256])
def test_random_vs_brute_force(oracle_lib, alphabet_size):
    rng = random.Random(1000 + alphabet_size)
    alphabet = list(range(256)) if alphabet_size == 256 else list(range(97, 97 + alphabet_size))
    for _ in range(150):
        _check_random_case(rng, alphabet, rng.randint(1, 12), rng.randint(1, 8),
                           rng.randint(0, 200))


@settings(max_examples=200, deadline=None)
@given(kws=st.lists(st.binary(min_size=1, max_size=6), min_size=1, max_size=10),
       text=st.binary(max_size=120))
def test_hypothesis_vs_brute_force(oracle_lib, kws, text):
    assert pairs(oracle_match(kws, text)) == pairs(brute_match(kws, text))


@settings(max_examples=100, deadline=None)
@given(kws=st.lists(st.text(alphabet="ab", min_size=1, max_size=5).map(str.encode),
                    min_size=1, max_size=8),
       text=st.text(alphabet="ab", max_size=100).map(str.encode))
def test_hypothesis_binary_alphabet(oracle_lib, kws, text):
    # a two-letter alphabet exercises long failure chains and nested outputs
    assert pairs(oracle_match(kws, text)) == pairs(brute_match(kws, text))


def test_invariants_full_tiny_workload(oracle_lib):
    """Tiny workload (64 keywords, 1 MiB): the result is checked in full
    against a per-keyword library substring search."""
    w = config_tiny()
    off, pid = oracle_match(w.keywords, w.text)
    tb = w.text.tobytes()
    # soundness
    for o, p in zip(off.tolist(), pid.tolist()):
        k = w.keywords[p]
        assert tb[o:o + len(k)] == k
    # completeness, keyword by keyword
    for p, k in enumerate(w.keywords):
        assert off[pid == p].tolist() == find_all(k, tb).tolist()
    # every surviving plant is present
    got = set(zip(off.tolist(), pid.tolist()))
    for o, p in w.plants:
        if tb[o:o + len(w.keywords[p])] == w.keywords[p]:
            assert (o, p) in got
    # sorted by (offset, id)
    order = np.lexsort((pid, off))
    assert (order == np.arange(len(off))).all()
    assert len(off) > 1900   # 2000 plants, a few overwritten by later ones


def test_pid_permutation_equivariance_and_monotonicity(oracle_lib):
    rng = np.random.default_rng(3)
    w = config_tiny()
    text = w.text[:200_000]
    kws = w.keywords
    base = set(pairs(oracle_match(kws, text)))
    perm = rng.permutation(len(kws))
    permuted = [kws[i] for i in perm]
    got = {(o, int(perm[p])) for o, p in pairs(oracle_match(permuted, text))}
    assert got == base
    sub = kws[:32]
    assert set(pairs(oracle_match(sub, text))) <= base


def test_stored_digests_still_match(oracle_lib):
    """The stored digests (written by tests/golden/make_golden.py from the
    oracle) guard against unreviewed drift of the oracle or the generators."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    stored = {}
    with open(mg.OUT) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, count, dig = line.split()
            stored[name] = (int(count), dig)
    for w in mg.workloads():
        off, pid = oracle_match(w.keywords, w.text)
        assert stored[w.name] == (len(off), mg.digest(off, pid)), w.name


@pytest.mark.parametrize("slice_bytes", [4096, 65536, 1 << 20])
def test_sliced_oracle_equals_whole(oracle_lib, slice_bytes):
    """The GPU tests compare their largest texts with the oracle run over
    overlapping slices on host threads (tests/helpers.py).  Pinned here
    against the oracle run once over the whole text: sweep keywords on 4 MiB
    of text with every keyword planted across slice boundaries (starting up
    to max_len bytes before a boundary and just after it), and the tiny
    workload."""
    from tests.helpers import oracle_sliced
    from workloads import config_sweep
    w = config_sweep(4 << 20)
    text = w.text.copy()
    rng = np.random.default_rng(9)
    L = max(len(k) for k in w.keywords)
    for b in range(slice_bytes, len(text) - 64, slice_bytes):
        for d in (-L, -L + 1, -3, -1, 0, 1):
            k = w.keywords[int(rng.integers(len(w.keywords)))]
            o = b + d
            if 0 <= o <= len(text) - len(k):
                text[o:o + len(k)] = np.frombuffer(k, dtype=np.uint8)
    o = Oracle(w.keywords)
    whole = o.match(text)
    (got,) = oracle_sliced(o, L, [text], slice_bytes=slice_bytes, workers=4)
    assert np.array_equal(got[0], whole[0]) and np.array_equal(got[1], whole[1])
    o.close()
    t = config_tiny()
    o = Oracle(t.keywords)
    whole = o.match(t.text)
    (got,) = oracle_sliced(o, max(len(k) for k in t.keywords), [t.text], slice_bytes=slice_bytes, workers=4)
    assert np.array_equal(got[0], whole[0]) and np.array_equal(got[1], whole[1])
    o.close()


def test_sliced_oracle_handles_empty_and_short_texts(oracle_lib):
    from tests.helpers import oracle_sliced
    kws = [b"ab", b"abc"]
    o = Oracle(kws)
    texts = [np.zeros(0, np.uint8), np.frombuffer(b"a", np.uint8), np.frombuffer(b"abcab", np.uint8)]
    res = oracle_sliced(o, 3, texts, slice_bytes=2, workers=2)
    assert len(res[0][0]) == 0 and len(res[1][0]) == 0
    assert res[2][0].tolist() == [0, 0, 3] and res[2][1].tolist() == [0, 1, 0]
    o.close()
