"""Shared helpers of the GPU parity tests (no matching arithmetic)."""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def as_pairs(off, pid):
    off = np.asarray(off, dtype=np.int64)
    pid = np.asarray(pid, dtype=np.int32)
    order = np.lexsort((pid, off))
    return off[order], pid[order]


def assert_same(got, exp, what=""):
    go, gp = as_pairs(*got)
    eo, ep = as_pairs(*exp)
    if len(go) != len(eo) or not (np.array_equal(go, eo) and np.array_equal(gp, ep)):
        gs = set(zip(go.tolist(), gp.tolist()))
        es = set(zip(eo.tolist(), ep.tolist()))
        missing = sorted(es - gs)[:10]
        extra = sorted(gs - es)[:10]
        raise AssertionError(f"{what}: GPU {len(go)} vs oracle {len(eo)} matches; "
                             f"missing {missing} extra {extra}")


def host_workers():
    """Threads for the oracle: the cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_sliced(oracle, max_len, texts, slice_bytes=16 << 20, workers=None):
    """The oracle's result for each text of `texts`, computed over slices on
    host threads (the oracle's C match call releases the GIL and reads its
    machine only).

    Slice [a, b) of a text is matched as text[a : b + max_len - 1] (clipped
    to the text), and only the occurrences starting before b are kept: an
    occurrence that starts in [a, b) ends before b + max_len - 1, so it lies
    wholly inside that window, and every start belongs to exactly one slice.
    The union is the whole text's result, which
    tests/test_oracle.py::test_sliced_oracle_equals_whole checks.
    """
    jobs = []
    for t, text in enumerate(texts):
        n = len(text)
        for a in range(0, max(n, 1), slice_bytes):
            b = min(a + slice_bytes, n)
            jobs.append((t, a, b, text[a:min(b + max_len - 1, n)]))

    def run(job):
        t, a, b, window = job
        off, pid = oracle.match(window)
        keep = off < (b - a)
        return t, off[keep] + a, pid[keep]

    parts = [[] for _ in texts]
    with ThreadPoolExecutor(max_workers=workers or host_workers()) as ex:
        for t, off, pid in ex.map(run, jobs):
            parts[t].append((off, pid))
    out = []
    for p in parts:
        if not p:
            out.append((np.zeros(0, np.int64), np.zeros(0, np.int32)))
            continue
        off = np.concatenate([x[0] for x in p])
        pid = np.concatenate([x[1] for x in p])
        out.append(as_pairs(off, pid))
    return out
