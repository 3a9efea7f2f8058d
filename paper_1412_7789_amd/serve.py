"""ctypes binding of the request server (include/pfac_serve.h).

Argument marshalling only: admission, batching, copies and scans all run in
libpfac.so's engine thread.
"""

from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L


def server_opts(mode: int = L.AC_SERVE_BATCHED, n_streams: int = 0, hbm_budget_bytes: int = 0,
                max_batch_bytes: int = 0, max_batch_texts: int = 0, matches_per_kib: int = 0) -> L.ServerOpts:
    o = L.ServerOpts()
    o.mode, o.n_streams, o.hbm_budget_bytes = mode, n_streams, hbm_budget_bytes
    o.max_batch_bytes, o.max_batch_texts, o.matches_per_kib = max_batch_bytes, max_batch_texts, matches_per_kib
    return o


def serve_charge(length: int, opts: Optional[L.ServerOpts] = None) -> int:
    """Budget bytes a request of `length` bytes is charged."""
    return L.check(L.load().ac_serve_charge(ctypes.byref(opts) if opts is not None else None, length),
                   "ac_serve_charge")


def serve_plan(automata: Sequence[int], lengths: Sequence[int], free_budget: int,
               opts: Optional[L.ServerOpts] = None) -> list:
    """Indices of the next batch the server would form from waiting requests."""
    a = np.ascontiguousarray(automata, dtype=np.int32)
    n = np.ascontiguousarray(lengths, dtype=np.int64)
    picked = np.zeros(max(len(a), 1), dtype=np.int32)
    k = L.check(L.load().ac_serve_plan(ctypes.byref(opts) if opts is not None else None, len(a),
                                       a.ctypes.data, n.ctypes.data, free_budget, picked.ctypes.data),
                "ac_serve_plan")
    return picked[:k].tolist()


class Server:
    """A request server on the current device.  Automata are registered, not
    owned: keep the Automaton objects alive while the server runs."""

    def __init__(self, opts: Optional[L.ServerOpts] = None):
        lib = L.load()
        h = ctypes.c_void_p()
        L.check(lib.ac_server_create(ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)),
                "ac_server_create")
        self._h = h
        self._keep = []

    def add_automaton(self, automaton) -> int:
        self._keep.append(automaton)
        return L.check(L.load().ac_server_add_automaton(self._h, automaton._h), "ac_server_add_automaton")

    def submit(self, automaton_id: int, text: np.ndarray) -> int:
        """Queue host `text` (uint8 array; pinned memory copies asynchronously).
        The array must stay alive until the request completes."""
        buf = np.ascontiguousarray(text, dtype=np.uint8)
        return L.check(L.load().ac_server_submit(self._h, automaton_id, buf.ctypes.data if buf.size else None,
                                                 buf.size), "ac_server_submit")

    def _result(self, r: L.RequestResult) -> Tuple[np.ndarray, np.ndarray, Dict[str, int]]:
        n = r.count
        off = np.ctypeslib.as_array(r.offset, shape=(n,)).copy() if n else np.zeros(0, np.int64)
        pid = np.ctypeslib.as_array(r.pattern_id, shape=(n,)).copy() if n else np.zeros(0, np.int32)
        return off, pid, {"batch_requests": r.batch_requests, "submit_ns": r.submit_ns, "done_ns": r.done_ns}

    def wait(self, request: int, release: bool = True):
        """(offsets, pattern_ids, meta) of a request, blocking until done."""
        r = L.RequestResult()
        L.check(L.load().ac_server_wait(self._h, request, ctypes.byref(r)), "ac_server_wait")
        out = self._result(r)
        if release:
            self.release(request)
        return out

    def poll(self, request: int):
        """None while pending, else what wait() returns (result kept)."""
        r = L.RequestResult()
        rc = L.check(L.load().ac_server_poll(self._h, request, ctypes.byref(r)), "ac_server_poll")
        return self._result(r) if rc == 1 else None

    def release(self, request: int) -> None:
        L.load().ac_server_release(self._h, request)

    def replay(self, automata: Sequence[int], texts: Sequence[np.ndarray], arrival_ns: Sequence[int]):
        """Open-loop replay; returns (latency_ns, counts) int64 arrays."""
        n = len(texts)
        bufs = [np.ascontiguousarray(t, dtype=np.uint8) for t in texts]
        ptrs = (ctypes.c_void_p * max(n, 1))(*[b.ctypes.data if b.size else None for b in bufs])
        lens = np.array([b.size for b in bufs], dtype=np.int64)
        aut = np.ascontiguousarray(automata, dtype=np.int32)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        lat = np.zeros(max(n, 1), dtype=np.int64)
        cnt = np.zeros(max(n, 1), dtype=np.int64)
        L.check(L.load().ac_server_replay(self._h, n, aut.ctypes.data, ptrs, lens.ctypes.data, arr.ctypes.data,
                                          lat.ctypes.data, cnt.ctypes.data), "ac_server_replay")
        return lat[:n], cnt[:n]

    def stats(self) -> Dict[str, int]:
        st = L.ServerStats()
        L.check(L.load().ac_server_get_stats(self._h, ctypes.byref(st)), "ac_server_get_stats")
        return st.as_dict()

    def close(self) -> None:
        if self._h:
            L.load().ac_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
