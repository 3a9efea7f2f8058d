"""The library's CPU matcher (the CPU side of the CPU/GPU dispatch) against
the oracle, on the CPU: no GPU is needed, the tables come from ac_compile.
It is product code, independent of the oracle: it walks the library's own
dense rows and child lists from every offset."""

import numpy as np
import pytest

import paper_1412_7789_amd as pf
from oracle import Oracle, brute_match
from tests.helpers import as_pairs, assert_same
from workloads import SPECS, config_large_automaton, config_sweep, config_tiny, make_keywords


@pytest.fixture(scope="module", autouse=True)
def lib():
    import os
    if not os.path.exists(pf.LIB_PATH):
        from paper_1412_7789_amd.build import build
        build()
    return pf.load()


def host(kws, text, budget=0, n_threads=0, capacity=None):
    return pf.Plan(kws, dense_budget_bytes=budget).match_host(text, n_threads=n_threads, capacity=capacity)


@pytest.mark.parametrize("budget", [0, 4096])
def test_tiny_workload(budget):
    w = config_tiny()
    assert_same(host(w.keywords, w.text, budget), Oracle(w.keywords).match(w.text), f"tiny budget {budget}")


@pytest.mark.parametrize("n_threads", [1, 3, 8])
def test_sweep_workload_threads(n_threads):
    w = config_sweep(4 << 20)
    assert_same(host(w.keywords, w.text, n_threads=n_threads), Oracle(w.keywords).match(w.text),
                f"sweep {n_threads} threads")


def test_large_automaton_compact_layout():
    """20000 byte keywords sharing prefixes: most states below the dense
    rows, so the walk runs through the sorted child lists."""
    w = config_large_automaton(8 << 20)
    p = pf.Plan(w.keywords)
    info = p.info()
    assert info["n_dense_states"] < info["n_states"]
    assert_same(p.match_host(w.text, n_threads=4), Oracle(w.keywords).match(w.text), "large 8 MiB")


def test_random_small_against_brute_force():
    rng = np.random.default_rng(11)
    for case in range(60):
        sigma = int(rng.integers(1, 5))
        kws = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 7)), dtype=np.uint8)) for _ in range(int(rng.integers(1, 9)))]
        text = rng.integers(0, sigma, size=int(rng.integers(0, 300)), dtype=np.uint8)
        assert_same(host(kws, text, budget=64 if case % 2 else 0), brute_match(kws, text.tobytes()), f"case {case}")


def test_nested_duplicate_and_zero_byte_keywords():
    kws = [b"a", b"aa", b"aaa", b"\x00\x00", b"aa", b"ba\x00"]
    text = np.frombuffer(b"aaaa\x00\x00\x00ba\x00a", dtype=np.uint8)
    assert_same(host(kws, text), brute_match(kws, text.tobytes()), "nested")
    assert len(host(kws, np.zeros(0, np.uint8))[0]) == 0


def test_capacity_returns_true_count_and_a_subset():
    w = config_tiny()
    exp = Oracle(w.keywords).match(w.text)
    n = len(exp[0])
    p = pf.Plan(w.keywords)
    lib = pf.load()
    expset = set(zip(exp[0].tolist(), exp[1].tolist()))
    for cap in (0, 1, n - 3, n):
        off = np.empty(max(cap, 1), np.int64)
        pid = np.empty(max(cap, 1), np.int32)
        got = lib.ac_plan_match_host(p._h, w.text.ctypes.data, len(w.text), off.ctypes.data, pid.ctypes.data, cap, 3)
        assert got == n
        sub = set(zip(off[:cap].tolist(), pid[:cap].tolist()))
        assert len(sub) == cap and sub <= expset


def test_errors():
    lib = pf.load()
    from paper_1412_7789_amd import _lib as L
    assert lib.ac_plan_match_host(None, None, 0, None, None, 0, 0) == L.AC_EINVAL
    p = pf.Plan([b"abc"])
    assert lib.ac_plan_match_host(p._h, None, 5, None, None, 0, 0) == L.AC_EINVAL
    assert lib.ac_plan_match_host(p._h, None, 0, None, None, 4, 0) == L.AC_EINVAL
