"""GPU tests of the request server: every served request's match set equals
the same text scanned alone (and, for a sample, the CPU oracle), whatever the
batching, mode, budget or match-slot reservation."""

import sys

import numpy as np
import pytest

from oracle import Oracle
from tests.helpers import assert_same
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


@pytest.fixture(scope="module")
def served():
    w = config_served(n_requests=160, pool_bytes=32 * MIB, size_hi=2 * MIB, sizes=(500, 5000, 20000, 500))
    automata = [pf.Automaton(k) for k in w.automata]
    pool_dev = torch.from_numpy(w.pool).cuda()
    alone = []
    for i in range(len(w.length)):
        s, n = int(w.start[i]), int(w.length[i])
        off, pid = automata[int(w.automaton[i])].match(pool_dev[s:s + n])
        alone.append((off.cpu().numpy(), pid.cpu().numpy()))
    return w, automata, alone


def texts_of(w):
    return [w.pool[int(s):int(s) + int(n)] for s, n in zip(w.start, w.length)]


def run_burst(w, automata, opts):
    with pf.Server(opts) as srv:
        ids = [srv.add_automaton(a) for a in automata]
        assert ids == list(range(len(automata)))
        texts = texts_of(w)
        reqs = [srv.submit(int(w.automaton[i]), texts[i]) for i in range(len(texts))]
        res = [srv.wait(r) for r in reqs]
        return res, srv.stats()


def test_batched_mix_equals_alone(served):
    w, automata, alone = served
    res, st = run_burst(w, automata, pf.server_opts())
    say("batched stats", st)
    assert st["requests"] == len(alone)
    assert st["batches"] < len(alone)            # requests really were batched together
    assert max(r[2]["batch_requests"] for r in res) > 1
    for i, (off, pid, meta) in enumerate(res):
        assert_same((off, pid), alone[i], f"request {i}")


def test_fifo_mode_equals_alone(served):
    w, automata, alone = served
    res, st = run_burst(w, automata, pf.server_opts(mode=pf.AC_SERVE_FIFO))
    assert st["batches"] == len(alone)
    for i, (off, pid, meta) in enumerate(res):
        assert meta["batch_requests"] == 1
        assert_same((off, pid), alone[i], f"request {i}")


def test_sample_against_oracle(served):
    w, automata, alone = served
    texts = texts_of(w)
    for i in range(0, len(texts), 23):
        o = Oracle(w.automata[int(w.automaton[i])])
        assert_same(alone[i], o.match(texts[i]), f"request {i} vs oracle")
        o.close()


def test_small_budget_forces_admission_waits(served):
    w, automata, alone = served
    aut_bytes = sum(a.info()["device_bytes"] for a in automata)
    opts = pf.server_opts(hbm_budget_bytes=aut_bytes + 3 * pf.serve_charge(2 * MIB), n_streams=4)
    res, st = run_burst(w, automata, opts)
    say("small budget stats", st)
    assert st["admission_waits"] > 0
    assert st["peak_charged"] <= opts.hbm_budget_bytes
    for i, (off, pid, meta) in enumerate(res):
        assert_same((off, pid), alone[i], f"request {i}")


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
    w, automata, alone = served
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
    with pf.Server(pf.server_opts(hbm_budget_bytes=a.info()["device_bytes"] + pf.serve_charge(4096))) as srv:
        assert srv.add_automaton(a) == 0
        with pytest.raises(pf.PfacError):
            srv.submit(1, np.zeros(10, np.uint8))            # unknown automaton
        with pytest.raises(pf.PfacError):
            srv.submit(0, np.zeros(1 << 20, np.uint8))       # larger than the whole budget
        off, pid, _ = srv.wait(srv.submit(0, np.frombuffer(b"xabcx", np.uint8)))
        assert off.tolist() == [1]
