"""ctypes wrapper over the serial Aho-Corasick oracle in ``ac_oracle.c``.

TEST INFRASTRUCTURE.  See the package docstring for who may use it.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

from .build import LIB, build

_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB) -> ctypes.CDLL:
    """Load (building first if absent) the oracle library."""
    global _lib
    if _lib is not None and path == LIB:
        return _lib
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.oracle_build.restype = vp
    lib.oracle_build.argtypes = [vp, vp, i32]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [vp]
    for name in ("oracle_num_states",):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [vp]
    lib.oracle_goto.restype = i32
    lib.oracle_goto.argtypes = [vp, i32, i32]
    lib.oracle_fail.restype = i32
    lib.oracle_fail.argtypes = [vp, i32]
    lib.oracle_out_count.restype = i32
    lib.oracle_out_count.argtypes = [vp, i32]
    lib.oracle_out_at.restype = i32
    lib.oracle_out_at.argtypes = [vp, i32, i32]
    lib.oracle_match.restype = vp
    lib.oracle_match.argtypes = [vp, vp, i64]
    lib.oracle_result_count.restype = i64
    lib.oracle_result_count.argtypes = [vp]
    lib.oracle_result_copy.restype = None
    lib.oracle_result_copy.argtypes = [vp, vp, vp]
    lib.oracle_result_free.restype = None
    lib.oracle_result_free.argtypes = [vp]
    if path == LIB:
        _lib = lib
    return lib


def _csr(keywords: Sequence[bytes]) -> Tuple[np.ndarray, np.ndarray]:
    lens = np.array([len(k) for k in keywords], dtype=np.int64)
    offs = np.zeros(len(keywords) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    flat = np.frombuffer(b"".join(keywords) or b"\0", dtype=np.uint8).copy()
    return flat, offs


class Oracle:
    """A built Aho-Corasick machine (Goto, Failure, Output) for ``keywords``."""

    def __init__(self, keywords: Sequence[bytes], lib_path: str = LIB):
        self._lib = load_library(lib_path)
        flat, offs = _csr(keywords)
        self._h = self._lib.oracle_build(flat.ctypes.data, offs.ctypes.data, len(keywords))
        if not self._h:
            raise ValueError("oracle: empty keyword or out of memory")
        self.n_keywords = len(keywords)

    def close(self) -> None:
        if self._h:
            self._lib.oracle_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the machine's three functions, for tests of the construction --------
    @property
    def n_states(self) -> int:
        return self._lib.oracle_num_states(self._h)

    def goto(self, s: int, a: int) -> int:
        """g(s, a); -1 when undefined (never at the root)."""
        return self._lib.oracle_goto(self._h, s, a)

    def fail(self, s: int) -> int:
        return self._lib.oracle_fail(self._h, s)

    def output(self, s: int) -> list:
        return [self._lib.oracle_out_at(self._h, s, k)
                for k in range(self._lib.oracle_out_count(self._h, s))]

    def state_of(self, prefix: bytes) -> int:
        """State reached from the root along ``prefix`` by Goto edges only."""
        s = 0
        for a in prefix:
            t = self.goto(s, a)
            if t <= 0:          # undefined, or the root's self-loop
                return -1
            s = t
        return s

    # -- matching --------------------------------------------------------------
    def match(self, text) -> Tuple[np.ndarray, np.ndarray]:
        """All (start offset, keyword id) occurrences, sorted by (offset, id)."""
        buf = np.ascontiguousarray(np.frombuffer(text, dtype=np.uint8)
                                   if isinstance(text, (bytes, bytearray)) else text,
                                   dtype=np.uint8)
        ptr = buf.ctypes.data if buf.size else None
        r = self._lib.oracle_match(self._h, ptr, buf.size)
        if not r:
            raise MemoryError("oracle_match: out of memory")
        try:
            n = self._lib.oracle_result_count(r)
            off = np.empty(n, dtype=np.int64)
            pid = np.empty(n, dtype=np.int32)
            self._lib.oracle_result_copy(r, off.ctypes.data, pid.ctypes.data)
        finally:
            self._lib.oracle_result_free(r)
        return off, pid


def oracle_match(keywords: Sequence[bytes], text) -> Tuple[np.ndarray, np.ndarray]:
    o = Oracle(keywords)
    try:
        return o.match(text)
    finally:
        o.close()
