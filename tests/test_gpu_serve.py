"""GPU tests of the request server: every served request's match set equals
the CPU oracle's for its text, whatever the batching, mode, budget or
match-slot reservation, and equals the same text scanned alone.  One test
serves the full-size mix: the four resident automata of 500, 5000, 20000
and 50000 byte keywords and requests of up to 64 MiB."""

import sys

import numpy as np
import pytest

from oracle import Oracle
from tests.helpers import assert_same, oracle_sliced
from workloads import KIB, MIB, config_served

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


def texts_of(w):
    return [w.pool[int(s):int(s) + int(n)] for s, n in zip(w.start, w.length)]


def oracle_results(w, texts, which):
    """The oracle's match set of every request (per automaton, over slices
    on host threads)."""
    exp = [None] * len(texts)
    for k, kws in enumerate(w.automata):
        ids = [i for i in range(len(texts)) if int(which[i]) == k]
        if not ids:
            continue
        o = Oracle(kws)
        for i, r in zip(ids, oracle_sliced(o, max(len(x) for x in kws), [texts[i] for i in ids])):
            exp[i] = r
        o.close()
    return exp


@pytest.fixture(scope="module")
def served():
    w = config_served(n_requests=160, pool_bytes=32 * MIB, size_hi=2 * MIB, sizes=(500, 5000, 20000, 500))
    automata = [pf.Automaton(k) for k in w.automata]
    texts = texts_of(w)
    exp = oracle_results(w, texts, w.automaton)
    pool_dev = torch.from_numpy(w.pool).cuda()
    alone = []
    for i in range(len(w.length)):
        s, n = int(w.start[i]), int(w.length[i])
        off, pid = automata[int(w.automaton[i])].match(pool_dev[s:s + n])
        alone.append((off.cpu().numpy(), pid.cpu().numpy()))
    return w, automata, alone, exp


def resident_of(**opts):
    """Device bytes of a server's own buffers (charged against its budget)."""
    with pf.Server(pf.server_opts(**opts)) as probe:
        return probe.stats()["resident_bytes"]


def run_burst(w, automata, opts, texts=None, which=None):
    texts = texts_of(w) if texts is None else texts
    which = w.automaton if which is None else which
    with pf.Server(opts) as srv:
        ids = [srv.add_automaton(a) for a in automata]
        assert ids == list(range(len(automata)))
        reqs = [srv.submit(int(which[i]), texts[i]) for i in range(len(texts))]
        res = [srv.wait(r) for r in reqs]
        return res, srv.stats()


def test_alone_equals_oracle(served):
    w, automata, alone, exp = served
    for i in range(len(alone)):
        assert_same(alone[i], exp[i], f"request {i} alone vs oracle")


def test_batched_mix_equals_oracle_and_alone(served):
    w, automata, alone, exp = served
    res, st = run_burst(w, automata, pf.server_opts())
    say("batched stats", st)
    assert st["requests"] == len(alone)
    assert st["batches"] < len(alone)            # requests really were batched together
    assert max(r[2]["batch_requests"] for r in res) > 1
    for i, (off, pid, meta) in enumerate(res):
        assert_same((off, pid), exp[i], f"request {i} served vs oracle")
        assert_same((off, pid), alone[i], f"request {i} served vs alone")


def test_fifo_mode_equals_oracle(served):
    w, automata, alone, exp = served
    res, st = run_burst(w, automata, pf.server_opts(mode=pf.AC_SERVE_FIFO))
    assert st["batches"] == len(alone)
    for i, (off, pid, meta) in enumerate(res):
        assert meta["batch_requests"] == 1
        assert_same((off, pid), exp[i], f"request {i} fifo vs oracle")


def test_small_budget_forces_admission_waits(served):
    w, automata, alone, exp = served
    aut_bytes = sum(a.info()["device_bytes"] for a in automata)
    resident = resident_of(n_streams=4)
    # per stream at least the scan's scratch and a full batch's text buffer
    assert resident >= 4 * (256 << 20)
    with pytest.raises(pf.PfacError):
        pf.Server(pf.server_opts(hbm_budget_bytes=resident - 1, n_streams=4))
    with pf.Server(pf.server_opts(hbm_budget_bytes=resident + 1024, n_streams=4)) as srv:
        with pytest.raises(pf.PfacError):
            srv.add_automaton(automata[0])
    opts = pf.server_opts(hbm_budget_bytes=aut_bytes + resident + 3 * pf.serve_charge(2 * MIB), n_streams=4)
    res, st = run_burst(w, automata, opts)
    say("small budget stats", st)
    assert st["admission_waits"] > 0
    assert st["resident_bytes"] == resident
    assert aut_bytes + resident < st["peak_charged"] <= opts.hbm_budget_bytes
    for i, (off, pid, meta) in enumerate(res):
        assert_same((off, pid), exp[i], f"request {i} vs oracle")


def test_full_size_mix_equals_oracle():
    """The served workload at full size: the four automata of 500, 5000,
    20000 and 50000 byte keywords (the last one about 1.7M states), the
    first 48 requests of the Poisson trace (up to 42 MiB) and two 64 MiB
    requests, batched and FIFO; every request against the oracle."""
    w = config_served(n_requests=48)
    texts = texts_of(w)
    which = list(int(x) for x in w.automaton)
    for k, start in ((3, 0), (2, 128 * MIB)):          # the largest size the mix draws
        texts.append(w.pool[start:start + 64 * MIB])
        which.append(k)
    assert 3 in which[:48] and max(len(t) for t in texts) == 64 * MIB
    automata = [pf.Automaton(k) for k in w.automata]
    say("full mix: states", [a.info()["n_states"] for a in automata])
    exp = oracle_results(w, texts, which)
    for mode in (pf.AC_SERVE_BATCHED, pf.AC_SERVE_FIFO):
        res, st = run_burst(w, automata, pf.server_opts(mode=mode), texts, which)
        say("full mix mode", mode, st)
        assert st["requests"] == len(texts)
        for i, (off, pid, meta) in enumerate(res):
            assert_same((off, pid), exp[i], f"mode {mode} request {i} (automaton {which[i]}, {len(texts[i])} B)")


def test_too_few_match_slots_rescans():
    kws = [b"ab", b"abc", b"bca", b"zz"]
    text = np.frombuffer(b"abc" * 200_000, dtype=np.uint8).copy()
    a = pf.Automaton(kws)
    exp = Oracle(kws).match(text)
    with pf.Server(pf.server_opts(matches_per_kib=1)) as srv:
        srv.add_automaton(a)
        reqs = [srv.submit(0, text[: 600_000 - 7 * k]) for k in range(5)]
        res = [srv.wait(r) for r in reqs]
        st = srv.stats()
    assert st["rescans"] >= 1
    assert_same(res[0][:2], exp, "rescanned request")
    for k, (off, pid, _) in enumerate(res):
        n = 600_000 - 7 * k
        e = Oracle(kws).match(text[:n])
        assert_same((off, pid), e, f"prefix {n}")


def test_empty_and_tiny_requests():
    a = pf.Automaton([b"a", b"ab"])
    with pf.Server() as srv:
        srv.add_automaton(a)
        texts = [np.zeros(0, np.uint8), np.frombuffer(b"a", np.uint8), np.frombuffer(b"ab" * 3, np.uint8)]
        res = [srv.wait(srv.submit(0, t)) for t in texts]
    assert len(res[0][0]) == 0
    assert sorted(res[1][0].tolist()) == [0]
    assert len(res[2][0]) == 6


def test_replay_reports_latencies(served):
    w, automata, alone, exp = served
    n = 60
    texts = texts_of(w)[:n]
    arrivals = np.rint(w.arrivals[:n] * 1e9).astype(np.int64)
    with pf.Server() as srv:
        for a in automata:
            srv.add_automaton(a)
        lat, cnt = srv.replay(w.automaton[:n].astype(np.int32), texts, arrivals)
    assert (lat > 0).all()
    assert cnt.tolist() == [len(alone[i][0]) for i in range(n)]


def test_submit_errors():
    a = pf.Automaton([b"abc"])
    budget = resident_of() + a.info()["device_bytes"] + pf.serve_charge(4096)
    with pf.Server(pf.server_opts(hbm_budget_bytes=budget)) as srv:
        assert srv.add_automaton(a) == 0
        with pytest.raises(pf.PfacError):
            srv.submit(1, np.zeros(10, np.uint8))            # unknown automaton
        with pytest.raises(pf.PfacError):
            srv.submit(0, np.zeros(1 << 20, np.uint8))       # larger than the whole budget
        off, pid, _ = srv.wait(srv.submit(0, np.frombuffer(b"xabcx", np.uint8)))
        assert off.tolist() == [1]
