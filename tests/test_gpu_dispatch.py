"""CPU/GPU dispatch (ac_match_dispatch): texts below the automaton's
threshold run on the library's CPU matcher, the others on the GPU, host text
in and host matches out either way; every result against the oracle, on both
sides of a set threshold and of a measured one."""

import sys

import numpy as np
import pytest

from oracle import Oracle
from tests.helpers import assert_same
from workloads import config_large_automaton, config_sweep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

pf = None


def setup_module(module):
    global pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_7789_amd as _pf
    _pf.load()
    pf = _pf


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_both_sides_of_a_set_threshold():
    w = config_sweep(8 << 20)
    a = pf.Automaton(w.keywords)
    o = Oracle(w.keywords)
    a.dispatch_threshold = 64 << 10
    assert a.dispatch_threshold == 64 << 10
    for n, where in ((1, pf.AC_RAN_CPU), (1000, pf.AC_RAN_CPU), ((64 << 10) - 1, pf.AC_RAN_CPU),
                     (64 << 10, pf.AC_RAN_GPU), ((4 << 20) + 3, pf.AC_RAN_GPU), (8 << 20, pf.AC_RAN_GPU)):
        text = w.text[:n]
        off, pid, ran = a.match_dispatch(text)
        say("dispatch", n, ran)
        assert ran == where, (n, ran)
        assert_same((off, pid), o.match(text), f"{n} bytes on unit {ran}")
    # the whole text on each unit by moving the threshold
    exp = o.match(w.text)
    for thr, where in ((0, pf.AC_RAN_GPU), (1 << 30, pf.AC_RAN_CPU)):
        a.dispatch_threshold = thr
        off, pid, ran = a.match_dispatch(w.text)
        assert ran == where
        assert_same((off, pid), exp, f"threshold {thr}")
    a.dispatch_threshold = -1
    assert a.dispatch_threshold == 8 << 10


def test_calibrated_threshold_and_large_automaton():
    w = config_large_automaton(4 << 20)
    a = pf.Automaton(w.keywords)
    o = Oracle(w.keywords)
    thr = a.calibrate_dispatch(w.text)
    say("calibrated threshold", thr)
    assert thr >= 512 and (thr & (thr - 1)) == 0 and a.dispatch_threshold == thr
    for n in sorted({max(1, thr // 2), thr - 1, thr, min(len(w.text), 2 * thr), len(w.text)}):
        n = min(n, len(w.text))
        off, pid, ran = a.match_dispatch(w.text[:n])
        assert ran == (pf.AC_RAN_CPU if n < thr else pf.AC_RAN_GPU)
        assert_same((off, pid), o.match(w.text[:n]), f"{n} bytes")


def test_host_matcher_on_a_built_automaton_and_capacity():
    w = config_sweep(1 << 20)
    a = pf.Automaton(w.keywords)
    exp = Oracle(w.keywords).match(w.text)
    assert_same(a.match_host(w.text, n_threads=5), exp, "ac_match_host")
    # a capacity below the count: the call grows its arrays once
    off, pid, ran = a.match_dispatch(w.text, capacity=3)
    assert_same((off, pid), exp, "dispatch, small capacity")
