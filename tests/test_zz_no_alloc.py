"""The allocation-free scan (ac_match_async_noalloc) against the allocating
asynchronous scan (ac_match_async) it mirrors, through the C ABI: two calls
in a row on one stream, the second on a shorter text, each compared element
by element with ac_match_async's matches on the same input (and with the
oracle), for the default launch and two explicit ones."""

import sys

import numpy as np
import pytest

from oracle import oracle_match
from tests.helpers import assert_same
from workloads import config_sweep

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


def run(fn, t, cap, launch, stream):
    off = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    pid = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(stream):
        fn(t, off, pid, cnt, launch=launch, stream=stream)
    stream.synchronize()
    n = int(cnt.item())
    return n, (off[:n].cpu().numpy(), pid[:n].cpu().numpy())


@pytest.mark.parametrize("cfg", [None, dict(policy=1, filter=2, stride=2, segs=4), dict(policy=1, segs=1, stride=1)])
def test_noalloc_equals_async_twice(cfg):
    w = config_sweep(48 << 20)
    a = pf.Automaton(w.keywords)
    launch = pf.launch_config(**cfg) if cfg else None
    s = torch.cuda.Stream()
    for n in (48 << 20, (3 << 20) + 7):               # the second call on a shorter text
        text = w.text[:n]
        t = torch.from_numpy(text).cuda()
        exp = oracle_match(w.keywords, text)
        cap = len(exp[0]) + 16
        say("noalloc", cfg, n)
        n_ref, ref = run(a.match_async, t, cap, launch, s)
        n_got, got = run(a.match_async_noalloc, t, cap, launch, s)
        assert n_got == n_ref == len(exp[0])
        assert_same(got, ref, f"noalloc vs async, {n} bytes")
        assert_same(got, exp, f"noalloc vs oracle, {n} bytes")


def test_noalloc_dense_text_uses_slow_mode():
    """Every offset a match: every wave fills its (smaller) static region at
    once and finishes in the slow mode; same matches as ac_match_async."""
    kws = [b"a" * 8, b"a" * 9]
    text = np.full((8 << 20) + 3, ord("a"), dtype=np.uint8)
    a = pf.Automaton(kws)
    t = torch.from_numpy(text).cuda()
    s = torch.cuda.Stream()
    cap = 2 * len(text)
    n_ref, ref = run(a.match_async, t, cap, None, s)
    n_got, got = run(a.match_async_noalloc, t, cap, None, s)
    assert n_got == n_ref == 2 * len(text) - 15
    assert_same(got, ref, "dense noalloc vs async")


def test_noalloc_rejects_bad_arguments():
    a = pf.Automaton([b"abcdefgh"])
    t = torch.zeros(100, dtype=torch.uint8, device="cuda")
    off = torch.empty(4, dtype=torch.int64, device="cuda")
    pid = torch.empty(4, dtype=torch.int32, device="cuda")
    import ctypes
    from paper_1412_7789_amd import _lib as L
    lib = L.load()
    m = L.Matches(ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(pid.data_ptr()), 4)
    rc = lib.ac_match_async_noalloc(a._h, ctypes.c_void_p(t.data_ptr()), 100, ctypes.byref(m), None, None, None)
    assert rc == L.AC_EINVAL and b"count" in lib.ac_last_error()
