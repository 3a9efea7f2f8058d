"""GPU parity: the HIP matcher against the CPU oracle, bit-exact.

Every case compares the sorted (offset, keyword id) set of the GPU with the
serial Aho-Corasick oracle on the same seeded input.  Kernels are reached only
through the C ABI (via the ctypes binding).
"""

import sys

import numpy as np
import pytest

from oracle import oracle_match
from tests.helpers import assert_same
from workloads import config_tiny

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

pf = None


def setup_module(module):
    global pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_7789_amd as _pf
    _pf.load()          # fails loudly when the HIP library is missing
    pf = _pf


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_match(keywords, text, launch=None, offset=0, automaton=None):
    """Run through the C ABI; `offset` shifts the text inside its buffer to test alignment."""
    a = automaton or pf.Automaton(keywords)
    buf = np.zeros(len(text) + offset + 16, dtype=np.uint8)
    buf[offset:offset + len(text)] = np.frombuffer(bytes(text), dtype=np.uint8) if not isinstance(text, np.ndarray) else text
    d = torch.from_numpy(buf).cuda()
    t = d[offset:offset + len(text)]
    off, pid = a.match(t, launch=launch)
    return off.cpu().numpy(), pid.cpu().numpy()


POLICIES = [
    ("filtered-bytes17-s4", dict(policy=1, filter=1, segs=4)),
    ("filtered-bits20-s2", dict(policy=1, filter=2, segs=2)),
    ("filtered-bytes16-s1", dict(policy=1, filter=3, segs=1)),
    ("filtered-bits19-s4-b256", dict(policy=1, filter=4, segs=4, block=256)),
    ("filtered-bytes17-s2-b512", dict(policy=1, filter=1, segs=2, block=512)),
    ("stride1-bytes17-s4", dict(policy=1, filter=1, segs=4, stride=1)),
    ("stride2-bits20-s4", dict(policy=1, filter=2, segs=4, stride=2)),
    ("stride2-bytes16-s1-b256", dict(policy=1, filter=3, segs=1, stride=2, block=256)),
    ("stride4-falls-back", dict(policy=1, filter=2, segs=4, stride=4)),
    ("dual19-s4", dict(policy=1, filter=5, segs=4)),
    ("dual19-stride1-s2-b512", dict(policy=1, filter=5, segs=2, stride=1, block=512)),
    ("pair20-falls-back", dict(policy=1, filter=6, segs=4, stride=4)),
    ("pair20-stride2-s2", dict(policy=1, filter=6, segs=2, stride=2)),
    ("pair20-stride2-s1-b256", dict(policy=1, filter=6, segs=1, stride=2, block=256)),
    ("direct-lds", dict(policy=2, table_in_lds=1)),
    ("direct-global", dict(policy=2, table_in_lds=2)),
]


def test_fig4_keywords():
    kws = [b"AB", b"ABG", b"BEDE", b"ED"]
    for text in [b"ABGBEDED", b"ABGBEDED" * 1000, b"xBEDEDABG" * 777]:
        say("fig4", len(text))
        assert_same(gpu_match(kws, text), oracle_match(kws, text), "fig4")


@pytest.mark.parametrize("name,cfg", POLICIES)
def test_tiny_config_all_policies(name, cfg):
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    exp = oracle_match(w.keywords, w.text)
    say("tiny", name)
    got = gpu_match(w.keywords, w.text, launch=pf.launch_config(**cfg), automaton=a)
    assert_same(got, exp, f"tiny {name}")


@pytest.mark.parametrize("offset", [0, 1, 3, 7, 15])
def test_unaligned_text_and_ragged_lengths(offset):
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    for n in [0, 1, 2, 3, 11, 15, 16, 17, 1023, 1024, 1025, 4095, 4096, 4097, 4111, 4112, 4113,
              65535, 65536 + 7, 200_003]:
        text = w.text[:n]
        say("unaligned", offset, n)
        assert_same(gpu_match(w.keywords, text, offset=offset, automaton=a),
                    oracle_match(w.keywords, text), f"offset {offset} n {n}")


def test_hand_built_edge_cases():
    cases = [
        ([b"abab"], b"ababab"),
        ([b"a", b"ab", b"abc", b"bc", b"c"], b"abc" * 500),
        ([b"ab", b"ab"], b"abab" * 300),                  # duplicate keywords
        ([b"hello"], b"hello"),                           # keyword = text
        ([b"hello!"], b"hello"),                          # keyword longer than text
        ([b"x" * 64], b"x" * 5000),                       # long self-overlapping keyword
        ([b"\x00", b"\xff", b"\x00\xff"], bytes([0, 255] * 3000)),
        ([b"aa"], b"a" * 10_000),
        ([b"q"], b""),
    ]
    for kws, text in cases:
        say("edge", kws[:3], len(text))
        assert_same(gpu_match(kws, text), oracle_match(kws, text), repr(kws[:3]))


def test_every_single_byte_keyword():
    rng = np.random.default_rng(11)
    kws = [bytes([b]) for b in range(256)]
    text = rng.integers(0, 256, size=50_000, dtype=np.uint8)
    for name, cfg in POLICIES:
        say("single-byte", name)
        assert_same(gpu_match(kws, text, launch=pf.launch_config(**cfg)),
                    oracle_match(kws, text), f"single bytes {name}")


@pytest.mark.parametrize("lens,strides", [((4, 7, 12, 31, 64), (1, 2)), ((6, 7, 12, 31, 64), (4,))])
def test_plants_straddling_chunk_boundaries(lens, strides):
    """Keywords planted across every position near 1 KiB / 2 KiB / 4 KiB
    boundaries, for each chunk geometry and sampling stride."""
    rng = np.random.default_rng(5)
    kws = [bytes(rng.integers(97, 123, size=L, dtype=np.uint8)) for L in lens]
    text = rng.integers(97, 123, size=3 * 4096 + 100, dtype=np.uint8)
    texts = []
    for boundary in (1024, 2048, 4096, 8192):
        for k in kws:
            for d in range(-len(k) - 1, 2):
                t = text.copy()
                o = boundary + d
                if 0 <= o and o + len(k) <= len(t):
                    t[o:o + len(k)] = np.frombuffer(k, dtype=np.uint8)
                    texts.append(t)
    a = pf.Automaton(kws)
    for segs, stride in [(sg, st) for sg in (1, 2, 4) for st in strides]:
        cfg = pf.launch_config(policy=1, segs=segs, stride=stride)
        for i, t in enumerate(texts):
            if i % 16 == 0:
                say("straddle", segs, i)
            assert_same(gpu_match(kws, t, launch=cfg, automaton=a), oracle_match(kws, t), f"segs {segs} #{i}")


def test_capacity_overflow_returns_true_count():
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    t = torch.from_numpy(w.text).cuda()
    exp_off, exp_pid = oracle_match(w.keywords, w.text)
    n = len(exp_off)
    assert a.count(t) == n
    for cap in (0, 1, n - 1, n):
        off = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
        pid = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        got = a.match_into(t, off[:cap], pid[:cap])
        assert got == n
        exp = set(zip(exp_off.tolist(), exp_pid.tolist()))
        sub = set(zip(off[:cap].cpu().tolist(), pid[:cap].cpu().tolist()))
        assert len(sub) == cap and sub <= exp


def test_errors_are_reported():
    with pytest.raises(pf.PfacError):
        pf.Automaton([b"ok", b""])
    a = pf.Automaton([b"abc"])
    t = torch.zeros(10, dtype=torch.uint8, device="cuda")
    with pytest.raises(pf.PfacError):
        a.count(t, launch=pf.launch_config(block=100))


@pytest.mark.parametrize("stride,filt", [(1, 0), (2, 0), (4, 0), (4, 6)])
def test_hit_region_overflow(stride, filt):
    """A periodic text where a third of all offsets match fills every wave's
    hit region at once, so every wave leaves the streaming loop for the slow
    mode that walks each hit as the prefix table confirms it."""
    kws = [b"abcab", b"cabca", b"zzzz"] if stride < 4 else [b"abcabcab", b"cabcabca", b"zzzzzzzz"]
    text = np.frombuffer(b"abc" * (16 << 20 // 3), dtype=np.uint8)
    text = np.ascontiguousarray(text[: 16 << 20])
    say("overflow", stride, filt, len(text))
    cfg = pf.launch_config(policy=1, stride=stride, segs=4, filter=filt)
    assert_same(gpu_match(kws, text, launch=cfg), oracle_match(kws, text), f"overflow stride {stride}")


@pytest.mark.parametrize("cfg", [None, dict(policy=1, stride=2, filter=2, segs=4),
                                 dict(policy=1, stride=4, filter=6, segs=2), dict(policy=1, stride=2, filter=6, segs=2),
                                 dict(policy=1, stride=1, segs=1)])
def test_dense_stretch_sends_some_waves_to_slow_mode(cfg):
    """32 MiB of the 1000-keyword workload with 2 MiB of one repeated byte
    in the middle and two keywords made of that byte: the waves that draw the
    dense chunks overflow their hit regions and finish in the slow mode, the
    others stay in the streaming loop; the whole match set against the
    oracle, single text and as a batch of 7 uneven texts."""
    from workloads import config_sweep
    w = config_sweep(32 << 20)
    text = w.text.copy()
    text[15 << 20:17 << 20] = ord("a")
    kws = list(w.keywords) + [b"a" * 8, b"a" * 12]
    a = pf.Automaton(kws)
    exp = oracle_match(kws, text)
    launch = pf.launch_config(**cfg) if cfg else None
    say("dense stretch", cfg, a.default_launch(len(text)))
    assert_same(gpu_match(kws, text, launch=launch, automaton=a), exp, f"dense stretch {cfg}")
    cuts = np.array([0, 1 << 20, 15 << 20, (15 << 20) + 12345, 16 << 20, 17 << 20, 30 << 20, 32 << 20], dtype=np.int64)
    tid, off, pid, per = (x.cpu().numpy() for x in a.match_batch(torch.from_numpy(text).cuda(),
                                                                  torch.from_numpy(cuts).cuda(), launch=launch))
    for t in range(len(cuts) - 1):
        seg = text[cuts[t]:cuts[t + 1]]
        sel = tid == t
        assert_same((off[sel], pid[sel]), oracle_match(kws, seg), f"batch text {t} {cfg}")


def test_graph_stays_valid_after_larger_calls_on_its_stream():
    """A scan captured in a HIP graph keeps its stream's scratch: larger
    synchronous and asynchronous calls on the same stream in between (the
    scratch is sized for the widest launch when the stream is first used)
    leave every replay equal to the oracle."""
    from workloads import config_sweep
    w = config_sweep(1 << 20)
    a = pf.Automaton(w.keywords)
    exp = oracle_match(w.keywords, w.text)
    n = len(exp[0])
    t = torch.from_numpy(w.text).cuda()
    off = torch.empty(n + 8, dtype=torch.int64, device="cuda")
    pid = torch.empty(n + 8, dtype=torch.int32, device="cuda")
    d_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    big = config_sweep(64 << 20)
    tb = torch.from_numpy(big.text).cuda()
    nb = len(oracle_match(big.keywords, big.text)[0])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.match_async(t, off, pid, d_count, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.match_async(t, off, pid, d_count, stream=s)
    for r in range(3):
        with torch.cuda.stream(s):
            assert a.count(tb, stream=s) == nb                  # 64x longer text, same stream
            bo = torch.empty(nb + 8, dtype=torch.int64, device="cuda")
            bp = torch.empty(nb + 8, dtype=torch.int32, device="cuda")
            bc = torch.zeros(1, dtype=torch.int64, device="cuda")
            a.match_async(tb, bo, bp, bc, stream=s)
        torch.cuda.synchronize()
        assert int(bc.item()) == nb
        off.fill_(-1)
        d_count.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        say("replay after larger calls", r)
        assert int(d_count.item()) == n
        assert_same((off[:n].cpu().numpy(), pid[:n].cpu().numpy()), exp, f"replay {r}")


def test_interleaved_call_kinds_share_a_stream():
    """Synchronous single-text calls number their matches from the stream's
    running count; batch and asynchronous calls in between must not disturb
    that numbering."""
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    t = torch.from_numpy(w.text).cuda()
    exp = oracle_match(w.keywords, w.text)
    n = len(exp[0])
    flat = torch.from_numpy(np.concatenate([w.text[:5000], w.text[:3000]])).cuda()
    offs = torch.tensor([0, 5000, 8000], dtype=torch.int64, device="cuda")
    d_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    for round_ in range(3):
        say("interleave", round_)
        off1, pid1 = a.match(t)
        assert_same((off1.cpu().numpy(), pid1.cpu().numpy()), exp, f"single #{round_}")
        tid, off, pid, per = a.match_batch(flat, offs)
        assert int(per.sum()) == len(tid)
        off2 = torch.empty(n, dtype=torch.int64, device="cuda")
        pid2 = torch.empty(n, dtype=torch.int32, device="cuda")
        a.match_async(t, off2, pid2, d_count)
        torch.cuda.synchronize()
        assert int(d_count.item()) == n
        assert_same((off2.cpu().numpy(), pid2.cpu().numpy()), exp, f"async #{round_}")
        assert a.count(t[:0]) == 0
        assert a.count(t) == n


@pytest.mark.parametrize("offset", [0, 1, 2, 3, 5])
def test_stride4_unaligned_and_ragged(offset):
    """Stride-4 sampling (keywords of 8..32 bytes) on every alignment and on
    lengths around chunk and segment sizes."""
    from workloads import config_sweep
    w = config_sweep(300_000)
    a = pf.Automaton(w.keywords)
    for n in [0, 5, 6, 7, 8, 15, 16, 17, 1023, 1024, 1031, 4096, 4099, 16384 + 9, 65536 + 3, 300_000]:
        text = w.text[:n]
        for segs in (1, 4):
            cfg = pf.launch_config(policy=1, segs=segs, stride=4)
            say("stride4", offset, n, segs)
            assert_same(gpu_match(w.keywords, text, launch=cfg, offset=offset, automaton=a),
                        oracle_match(w.keywords, text), f"offset {offset} n {n} segs {segs}")


def test_long_keywords_and_long_shared_prefixes():
    """Keywords of 1000 and 4097 bytes (forced-path compares over many
    16-byte rounds, a direct-policy halo of 4 KiB), keywords that share a
    900-byte prefix and differ only at the end, and nested long keywords."""
    rng = np.random.default_rng(21)
    base = bytes(rng.integers(0, 256, size=4097, dtype=np.uint8))
    kws = [base, base[:1000], base[:900] + b"\x00", base[:900] + b"\xff", base[100:1100], base[:7]]
    text = bytearray(rng.integers(0, 256, size=300_000, dtype=np.uint8).tobytes())
    for at in (0, 5000, 77_777, 150_001, 300_000 - 4097):
        text[at:at + 4097] = base
    text[200_000:200_901] = base[:900] + b"\x00"
    text[250_000:250_901] = base[:900] + b"\xfe"          # differs in its last byte: no match
    text = bytes(text)
    exp = oracle_match(kws, text)
    assert len(exp[0]) >= 15
    for name, cfg in POLICIES:
        say("long", name)
        assert_same(gpu_match(kws, text, launch=pf.launch_config(**cfg)), exp, f"long {name}")


def test_unary_chains_to_final_and_branching_states():
    """Walk steps that skip a unary chain with one compare: chains that end
    at a state where a keyword ends, at a branch, or at a forced path;
    every single-byte change inside each planted keyword; and a text that
    ends inside a chain."""
    kws = [b"abcdefghij", b"abcdefghXY", b"abcde", b"abcdefghijklmnop", b"zzzzzzzzzzzz1",
           b"zzzzzzzzzzzz2", b"qrstuvwxyz0123456789"]
    text = bytearray()
    for piece in kws:
        text += piece + b"."
        for i in range(len(piece)):
            changed = bytearray(piece)
            changed[i] ^= 0x20
            text += changed + b"."
    text += b"abcdefghijklm"            # the text ends inside a chain
    text = bytes(text)
    exp = oracle_match(kws, text)
    assert len(exp[0]) >= len(kws)
    for name, cfg in POLICIES:
        say("chains", name)
        assert_same(gpu_match(kws, text, launch=pf.launch_config(**cfg)), exp, f"chains {name}")


def test_binary_keywords_with_zero_bytes():
    rng = np.random.default_rng(22)
    kws = [b"\x00\x00\x00\x00", b"\x00\x01\x00", b"\x00" * 9, bytes(range(256)), b"\xff\x00\xff\x00"]
    text = np.zeros(70_000, dtype=np.uint8)
    text[10_000:10_256] = np.arange(256, dtype=np.uint8)
    text[20_000:30_000] = rng.integers(0, 2, size=10_000, dtype=np.uint8)
    text[40_000:40_008] = np.frombuffer(b"\xff\x00\xff\x00\xff\x00\xff\x00", dtype=np.uint8)
    exp = oracle_match(kws, text)
    for name, cfg in POLICIES:
        say("binary", name)
        assert_same(gpu_match(kws, text, launch=pf.launch_config(**cfg)), exp, f"binary {name}")


def test_concurrent_host_threads_on_their_own_streams():
    """Synchronous calls from four host threads at once, each on its own
    stream (its own count word and hit regions) and text, with one shared
    automaton: every call gives the oracle's result for its text."""
    import threading
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    slices = [w.text[s:s + (1 << 18) + 7 * s] for s in (0, 3, 100_001, 500_000)]
    exp = [oracle_match(w.keywords, s) for s in slices]
    errors = []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                d = torch.from_numpy(slices[t]).cuda()
                for r in range(12):
                    off, pid = a.match(d, stream=s)
                    assert_same((off.cpu().numpy(), pid.cpu().numpy()), exp[t], f"thread {t} call {r}")
                    assert a.count(d, stream=s) == len(exp[t][0])
        except Exception as e:          # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads), "a worker did not finish"
    assert not errors, errors[0]


def test_released_stream_scratch_is_rebuilt():
    """ac_release_stream frees a stream's scratch; the next call on the stream
    allocates it again and gives the same result.  Releasing a stream the
    library never used, or twice, is harmless."""
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    text = w.text[:(1 << 19) + 13]
    exp = oracle_match(w.keywords, text)
    s = torch.cuda.Stream()
    pf.release_stream(s)
    with torch.cuda.stream(s):
        d = torch.from_numpy(text).cuda()
        for r in range(3):
            off, pid = a.match(d, stream=s)
            assert_same((off.cpu().numpy(), pid.cpu().numpy()), exp, f"call {r}")
            s.synchronize()
            pf.release_stream(s)
            pf.release_stream(s)
        assert a.count(d, stream=s) == len(exp[0])
        off, pid, ran = a.match_dispatch(text, stream=s)
        assert ran == pf.AC_RAN_GPU
        assert_same((off, pid), exp, "dispatch after release")
    s.synchronize()
    pf.release_stream(s)


def test_every_offset_matches_closed_form():
    """A text of one repeated byte with keywords c^L: every offset is a
    candidate and a hit, walks run 32 states deep past keywords ending on the
    way, and every wave's hit region overflows.  The full match set against
    the oracle at 1 MiB; the count against the closed form sum(N - L + 1) at
    64 MiB, for the default launch and each segment count."""
    kws = [b"a" * L for L in (1, 2, 4, 9, 32)] + [b"ab"]
    a = pf.Automaton(kws)
    small = np.full(1 << 20, ord("a"), dtype=np.uint8)
    say("every offset, 1 MiB")
    assert_same(gpu_match(kws, small, automaton=a), oracle_match(kws, small), "1 MiB of a")
    n = 64 << 20
    t = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda")
    exp = sum(n - len(k) + 1 for k in kws[:-1])
    for cfg in (None, dict(policy=1, segs=1), dict(policy=1, segs=2), dict(policy=1, segs=4)):
        say("every offset, 64 MiB", cfg)
        assert a.count(t, launch=pf.launch_config(**cfg) if cfg else None) == exp, str(cfg)


def test_single_text_graph_replays_match_eager():
    """The asynchronous single-text call (clearing kernel + scan) captured in
    a HIP graph: each replay, with eager synchronous calls on the default
    stream in between, writes the oracle's match set and count again."""
    w = config_tiny()
    a = pf.Automaton(w.keywords)
    text = w.text[: (1 << 19) + 5]
    exp = oracle_match(w.keywords, text)
    n = len(exp[0])
    t = torch.from_numpy(text).cuda()
    off = torch.empty(n + 8, dtype=torch.int64, device="cuda")
    pid = torch.empty(n + 8, dtype=torch.int32, device="cuda")
    d_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.match_async(t, off, pid, d_count, stream=s)     # sizes the stream's scratch before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.match_async(t, off, pid, d_count, stream=s)
    for r in range(4):
        say("single graph replay", r)
        off.fill_(-1)
        pid.fill_(-1)
        d_count.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert int(d_count.item()) == n
        assert_same((off[:n].cpu().numpy(), pid[:n].cpu().numpy()), exp, f"replay {r}")
        assert a.count(t) == n                              # eager work between replays
