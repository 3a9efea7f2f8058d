"""GPU parity on the benchmark workloads, at their real sizes.

* sweep (1000 printable keywords): every size of the x16 sweep up to 1 GiB
  compared in full with the oracle (1 GiB in the benchmark's launch
  configuration, the oracle run over slices on host threads), plus soundness
  of every match, completeness of every surviving plant and sampled
  per-keyword counts at 1 GiB.
* large automaton (20000 byte keywords, ~734k states, compact layout): 64 MiB
  and 1 GiB in full.
* batched (2000 keywords, 4096 log-normal texts): every text against the
  oracle, and the batch against per-text calls.
"""

import sys

import numpy as np
import pytest

from oracle import Oracle
from tests.helpers import as_pairs, assert_same, oracle_sliced
from workloads import GIB, MIB, config_batched, config_large_automaton, config_sweep

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


def run_gpu(a, text_np, launch=None):
    t = torch.from_numpy(text_np).cuda()
    off, pid = a.match(t, launch=launch)
    res = (off.cpu().numpy(), pid.cpu().numpy())
    del t
    return res


def check_sound(keywords, text, off, pid):
    """Every reported (o, p) really is an occurrence (vectorised per keyword)."""
    for p in np.unique(pid):
        k = np.frombuffer(keywords[p], dtype=np.uint8)
        o = off[pid == p]
        assert (o >= 0).all() and (o + len(k) <= len(text)).all()
        win = text[o[:, None] + np.arange(len(k))[None, :]]
        assert (win == k[None, :]).all(), f"unsound match for keyword {p}"


def count_overlapping(text_bytes, k):
    """Occurrences of k in the text, overlapping ones included (bytes.find)."""
    n, i = 0, text_bytes.find(k)
    while i >= 0:
        n += 1
        i = text_bytes.find(k, i + 1)
    return n


def check_sampled_counts(keywords, text, pid, n_keywords=20, seed=0):
    """Per-keyword match counts over the whole text equal a plain substring
    count for a sample of keywords."""
    tb = text.tobytes()
    got = np.bincount(pid, minlength=len(keywords))
    for p in np.random.default_rng(seed).choice(len(keywords), size=n_keywords, replace=False):
        assert got[p] == count_overlapping(tb, keywords[p]), f"keyword {p}"


def check_plants(keywords, text, off, pid, plants):
    got = set(zip(off.tolist(), pid.tolist()))
    for o, p in plants:
        k = keywords[p]
        if bytes(text[o:o + len(k)]) == k:
            assert (o, p) in got


@pytest.mark.parametrize("size", [1 << 10, 1 << 14, 1 << 18, 1 << 22, 1 << 26])
def test_sweep_sizes_full(size):
    w = config_sweep(size)
    a = pf.Automaton(w.keywords)
    say("sweep", size)
    assert_same(run_gpu(a, w.text), Oracle(w.keywords).match(w.text), f"sweep {size}")


def test_sweep_policies_agree():
    w = config_sweep(1 << 22)
    a = pf.Automaton(w.keywords)
    exp = Oracle(w.keywords).match(w.text)
    for cfg in [dict(policy=1, filter=f, segs=s, block=b, stride=st) for f in (1, 2, 3, 4, 5) for s in (1, 2, 4)
                for b in (256, 1024) for st in (1, 2, 4)] + \
               [dict(policy=1, filter=6, segs=s, block=b, stride=st) for s in (1, 2, 4) for b in (256, 512, 1024)
                for st in (2, 4)] + \
               [dict(policy=2)]:
        say("sweep policy", cfg)
        assert_same(run_gpu(a, w.text, pf.launch_config(**cfg)), exp, str(cfg))


def full_oracle(keywords, text):
    o = Oracle(keywords)
    (res,) = oracle_sliced(o, max(len(k) for k in keywords), [text])
    o.close()
    return res


def test_sweep_1gib_launch():
    w = config_sweep(GIB)
    a = pf.Automaton(w.keywords)
    launch = a.default_launch(GIB)
    say("sweep 1 GiB", launch)
    # the measured default for 1000 printable keywords: 4-byte windows at stride 4, two segments
    assert (launch["stride"], launch["filter"], launch["segs"]) == (4, 6, 2)
    off, pid = run_gpu(a, w.text)
    off, pid = as_pairs(off, pid)
    assert len(off) > 250_000
    say("sweep 1 GiB: oracle")
    assert_same((off, pid), full_oracle(w.keywords, w.text), "sweep 1 GiB")
    check_sound(w.keywords, w.text, off, pid)
    check_plants(w.keywords, w.text, off, pid, w.plants)
    check_sampled_counts(w.keywords, w.text, pid)


def test_large_automaton_64mib_full():
    w = config_large_automaton(64 * MIB)
    a = pf.Automaton(w.keywords)
    info = a.info()
    say("large 64 MiB", info["n_states"], info["n_dense_states"])
    assert info["n_dense_states"] < info["n_states"]      # compact layout in use
    exp = Oracle(w.keywords).match(w.text)
    assert_same(run_gpu(a, w.text), exp, "large 64 MiB")
    for cfg in [dict(policy=1, filter=1, stride=1), dict(policy=1, filter=4, segs=1, stride=2),
                dict(policy=1, filter=2, stride=2), dict(policy=1, filter=5, stride=1),
                dict(policy=1, filter=6, stride=4), dict(policy=1, filter=6, stride=2, segs=2),
                dict(policy=1, filter=6, stride=2, segs=4), dict(policy=2)]:
        say("large policy", cfg)
        assert_same(run_gpu(a, w.text, pf.launch_config(**cfg)), exp, str(cfg))


def test_large_automaton_1gib_launch():
    w = config_large_automaton(GIB)
    a = pf.Automaton(w.keywords)
    launch = a.default_launch(GIB)
    say("large 1 GiB", launch)
    # the measured default for 20000 byte keywords: 4-byte windows (three bits) at stride 2, four segments
    assert (launch["stride"], launch["filter"], launch["segs"]) == (2, 6, 4)
    assert a.default_launch(128 * MIB)["segs"] == 2
    off, pid = run_gpu(a, w.text)
    off, pid = as_pairs(off, pid)
    say("large 1 GiB: oracle")
    assert_same((off, pid), full_oracle(w.keywords, w.text), "large 1 GiB")
    check_sound(w.keywords, w.text, off, pid)
    check_plants(w.keywords, w.text, off, pid, w.plants)


def test_pid_permutation_and_keyword_subsets():
    """Renumbering the keywords renumbers the matches and nothing else, and an
    automaton of a subset of the keywords finds exactly the full set's
    matches of those keywords (the subsets get their own filter choices)."""
    w = config_sweep(64 * MIB)
    n = len(w.keywords)
    full = run_gpu(pf.Automaton(w.keywords), w.text)
    rng = np.random.default_rng(3)
    perm = rng.permutation(n)
    off, pid = run_gpu(pf.Automaton([w.keywords[i] for i in perm]), w.text)
    assert_same((off, perm[pid]), full, "permuted keyword ids")
    for size in (10, 300, 999):
        sub = np.sort(rng.choice(n, size=size, replace=False))
        say("subset", size)
        off, pid = run_gpu(pf.Automaton([w.keywords[i] for i in sub]), w.text)
        sel = np.isin(full[1], sub)
        assert_same((off, sub[pid]), (full[0][sel], full[1][sel]), f"subset of {size}")


def batch_expected(keywords, texts, offsets):
    o = Oracle(keywords)
    tids, offs, pids = [], [], []
    for t in range(len(offsets) - 1):
        eo, ep = o.match(texts[offsets[t]:offsets[t + 1]])
        tids.append(np.full(len(eo), t, dtype=np.int64))
        offs.append(eo)
        pids.append(ep)
    o.close()
    return np.concatenate(tids), np.concatenate(offs), np.concatenate(pids)


def batch_key(tid, off, pid):
    # one int64 per match for set comparison: (text id, offset, keyword id)
    return np.sort((np.asarray(tid, np.int64) << 44) | (np.asarray(off, np.int64) << 16) | np.asarray(pid, np.int64))


def test_batched_config_every_text():
    w = config_batched()
    a = pf.Automaton(w.keywords)
    say("batched", len(w.offsets) - 1, int(w.offsets[-1]))
    d_texts = torch.from_numpy(w.texts).cuda()
    d_offs = torch.from_numpy(w.offsets).cuda()
    tid, off, pid, per = a.match_batch(d_texts, d_offs)
    tid, off, pid, per = (x.cpu().numpy() for x in (tid, off, pid, per))
    et, eo, ep = batch_expected(w.keywords, w.texts, w.offsets)
    assert len(tid) == len(et)
    assert (batch_key(tid, off, pid) == batch_key(et, eo, ep)).all()
    assert (per == np.bincount(et, minlength=len(w.offsets) - 1)).all()
    # the same texts scanned alone give the same matches
    rng = np.random.default_rng(0)
    for t in rng.choice(len(w.offsets) - 1, size=40, replace=False):
        s, e = int(w.offsets[t]), int(w.offsets[t + 1])
        alone = run_gpu(a, w.texts[s:e])
        sel = tid == t
        assert_same(alone, (off[sel], pid[sel]), f"text {t} alone vs batch")


def test_batch_edge_cases():
    kws = [b"abc", b"abcd", b"bcd", b"zz", b"a"]
    texts = [b"", b"a", b"ab", b"abcd", b"", b"zzz", b"xabcdx" * 50, b"a" * 3, b"", b"bcd"]
    flat = np.frombuffer(b"".join(texts), dtype=np.uint8).copy()
    offs = np.zeros(len(texts) + 1, dtype=np.int64)
    np.cumsum([len(t) for t in texts], out=offs[1:])
    a = pf.Automaton(kws)
    for shift in (0, 1, 5):          # unaligned packed buffers
        buf = np.zeros(len(flat) + shift, dtype=np.uint8)
        buf[shift:] = flat
        d = torch.from_numpy(buf).cuda()[shift:]
        tid, off, pid, per = (x.cpu().numpy() for x in a.match_batch(d, torch.from_numpy(offs).cuda()))
        et, eo, ep = batch_expected(kws, flat, offs)
        assert (batch_key(tid, off, pid) == batch_key(et, eo, ep)).all(), shift
        assert (per == np.bincount(et, minlength=len(texts))).all()


def test_batches_without_per_text_counts_interleave_with_single_calls():
    """A batch call without per-text counts launches the scan kernel alone
    and numbers its matches on from the stream's count word, as single-text
    calls do; one with per-text counts clears the word first.  Interleaved on
    one stream, every call gives its own exact result."""
    w = config_batched()
    n = 500
    end = int(w.offsets[n])
    texts, offsets = w.texts[:end], w.offsets[:n + 1]
    a = pf.Automaton(w.keywords)
    et, eo, ep = batch_expected(w.keywords, texts, offsets)
    want = batch_key(et, eo, ep)
    single = w.texts[end:end + 3 * MIB]
    exp_single = Oracle(w.keywords).match(single)
    d_texts = torch.from_numpy(texts).cuda()
    d_offs = torch.from_numpy(offsets).cuda()
    cap = len(et) + 64
    tid = torch.empty(cap, dtype=torch.int32, device="cuda")
    off = torch.empty(cap, dtype=torch.int64, device="cuda")
    pid = torch.empty(cap, dtype=torch.int32, device="cuda")
    per = torch.empty(n, dtype=torch.int64, device="cuda")
    for step, kind in enumerate(["plain", "single", "plain", "per", "plain", "single", "single", "plain", "per"]):
        say("interleave", step, kind)
        if kind == "single":
            assert_same(run_gpu(a, single), exp_single, f"single text, step {step}")
            continue
        got = a.match_batch_into(d_texts, d_offs, tid, off, pid, per if kind == "per" else None)
        assert got == len(et), (step, kind, got)
        t, o, p = (x[:got].cpu().numpy() for x in (tid, off, pid))
        assert (batch_key(t, o, p) == want).all(), (step, kind)
        if kind == "per":
            assert (per.cpu().numpy() == np.bincount(et, minlength=n)).all(), step


@pytest.mark.parametrize("n_texts", [12000, 16383, 16384, 24000])
def test_batch_text_lookup_in_lds_and_global(n_texts):
    """Walks find their text by a binary search over the text starts, in LDS
    when the batch's starts fit beside the match stage (fewer than 16384
    texts with the 64 KiB maps, about 20400 with the 128 KiB maps), else in
    global memory: both sides of each limit against the oracle."""
    w = config_batched()
    rng = np.random.default_rng(n_texts)
    lens = rng.integers(0, 700, size=n_texts)
    offsets = np.zeros(n_texts + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    texts = w.texts[: int(offsets[-1])].copy()
    a = pf.Automaton(w.keywords)
    et, eo, ep = batch_expected(w.keywords, texts, offsets)
    d_texts = torch.from_numpy(texts).cuda()
    d_offs = torch.from_numpy(offsets).cuda()
    for cfg in (None, dict(policy=1, filter=2), dict(policy=1, filter=4, stride=1)):
        say("batch lookup", n_texts, cfg)
        launch = pf.launch_config(**cfg) if cfg else None
        tid, off, pid, per = (x.cpu().numpy() for x in a.match_batch(d_texts, d_offs, launch=launch))
        assert len(tid) == len(et)
        assert (batch_key(tid, off, pid) == batch_key(et, eo, ep)).all(), str(cfg)
        assert (per == np.bincount(et, minlength=n_texts)).all(), str(cfg)


def test_batch_graph_replays_match_eager():
    """The asynchronous batch call captured in a HIP graph: every replay, with
    eager calls on other streams in between, gives the eager result."""
    w = config_batched()
    n = 300
    end = int(w.offsets[n])
    texts, offsets = w.texts[:end], w.offsets[:n + 1]
    a = pf.Automaton(w.keywords)
    d_texts = torch.from_numpy(texts).cuda()
    d_offs = torch.from_numpy(offsets).cuda()
    et, eo, ep, eper = (x.cpu().numpy() for x in a.match_batch(d_texts, d_offs))
    exp_key = batch_key(et, eo, ep)
    bt, bo, bp = batch_expected(w.keywords, texts, offsets)
    assert (batch_key(bt, bo, bp) == exp_key).all()
    cap = len(et) + 16
    tid = torch.empty(cap, dtype=torch.int32, device="cuda")
    off = torch.empty(cap, dtype=torch.int64, device="cuda")
    pid = torch.empty(cap, dtype=torch.int32, device="cuda")
    per = torch.empty(n, dtype=torch.int64, device="cuda")
    d_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.match_batch_async(d_texts, d_offs, tid, off, pid, d_count, per, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.match_batch_async(d_texts, d_offs, tid, off, pid, d_count, per, stream=s)
    for r in range(4):
        say("graph replay", r)
        tid.fill_(-1)
        per.fill_(-7)
        d_count.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        k = int(d_count.item())
        assert k == len(et)
        got = batch_key(tid[:k].cpu().numpy(), off[:k].cpu().numpy(), pid[:k].cpu().numpy())
        assert (got == exp_key).all()
        assert (per.cpu().numpy() == eper).all()
        # eager work on the default stream between replays
        assert a.count(d_texts[: int(offsets[1])]) == int(eper[0])


def test_tune_records_a_choice_and_keeps_results():
    """ac_tune times every filtered choice on a sample; later default calls of
    a similar length use the choice, and every choice gives the same matches."""
    w = config_sweep(8 * MIB)
    a = pf.Automaton(w.keywords)
    t = torch.from_numpy(w.text).cuda()
    exp = Oracle(w.keywords).match(w.text)
    before = a.default_launch(t.numel())
    cfg = a.tune(t)
    say("tuned", cfg, "default was", before)
    assert cfg["policy"] == 1 and cfg["stride"] in (1, 2, 4) and cfg["segs"] in (1, 2, 4)
    assert a.default_launch(t.numel()) == cfg
    assert a.default_launch(t.numel() + 12345) == cfg              # same length bucket
    assert a.default_launch(t.numel() * 64) == a.default_launch(t.numel() * 64)
    assert_same(run_gpu(a, w.text), exp, "after tuning")
    half = w.text[: t.numel() // 2 + 3]
    assert_same(run_gpu(a, half), Oracle(w.keywords).match(half), "other length")


def test_tune_batch_records_a_choice_and_keeps_results():
    """ac_tune_batch times every filtered choice on a batch; later default
    batch calls of a similar total length use it, with the same matches."""
    w = config_batched()
    n = 1500
    end = int(w.offsets[n])
    texts, offsets = w.texts[:end], w.offsets[:n + 1]
    a = pf.Automaton(w.keywords)
    d_texts = torch.from_numpy(texts).cuda()
    d_offs = torch.from_numpy(offsets).cuda()
    cfg = a.tune_batch(d_texts, d_offs)
    say("batch tuned", cfg)
    assert cfg["policy"] == 1 and cfg["stride"] in (1, 2, 4) and cfg["segs"] in (1, 2, 4)
    tid, off, pid, per = (x.cpu().numpy() for x in a.match_batch(d_texts, d_offs))
    et, eo, ep = batch_expected(w.keywords, texts, offsets)
    assert (batch_key(tid, off, pid) == batch_key(et, eo, ep)).all()
    assert (per == np.bincount(et, minlength=n)).all()


@pytest.mark.parametrize("n_texts", [5000, 20000])
def test_batch_of_one_byte_texts_closed_form(n_texts):
    """Texts of one repeated byte with keywords c^1, c^3, c^7: text i of
    length L holds max(0, L - k + 1) matches of c^k and no match may run into
    the next text.  Per-text counts against that closed form, and every
    reported match inside its own text; on both sides of the LDS limit of the
    walks' text lookup."""
    kws = [b"a", b"aaa", b"a" * 7]
    klen = np.array([len(k) for k in kws])
    rng = np.random.default_rng(n_texts + 1)
    lens = rng.integers(0, 200, size=n_texts)
    offsets = np.zeros(n_texts + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    texts = np.full(int(offsets[-1]), ord("a"), dtype=np.uint8)
    a = pf.Automaton(kws)
    tid, off, pid, per = (x.cpu().numpy() for x in a.match_batch(torch.from_numpy(texts).cuda(),
                                                                  torch.from_numpy(offsets).cuda()))
    exp = sum(np.maximum(0, lens - L + 1) for L in klen)
    assert (per == exp).all()
    assert len(tid) == int(exp.sum())
    assert (off >= 0).all() and (off + klen[pid] <= lens[tid]).all()
    # no (text, offset, keyword) reported twice
    key = (tid.astype(np.int64) << 40) | (off.astype(np.int64) << 8) | pid
    assert len(np.unique(key)) == len(key)
