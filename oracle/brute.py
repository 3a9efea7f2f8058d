"""The result's plain definition, written out.  TEST INFRASTRUCTURE.

For keywords k_0 .. k_{n-1} and a text T of N bytes the matcher must return

    R = { (o, p) : 0 <= o <= N - |k_p|,  T[o : o + |k_p|] == k_p }

sorted by (o, p) -- "all occurrences of any of a finite number of keywords"
(paper, Section II), each reported at the offset where it begins.
"""

from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def brute_match(keywords: Sequence[bytes], text: bytes) -> Tuple[np.ndarray, np.ndarray]:
    """Every offset against every keyword: O(N * sum|k|).  Tiny inputs only."""
    text = bytes(text)
    out = []
    for o in range(len(text)):
        for p, k in enumerate(keywords):
            if len(k) and text[o:o + len(k)] == k:
                out.append((o, p))
    out.sort()
    off = np.array([o for o, _ in out], dtype=np.int64)
    pid = np.array([p for _, p in out], dtype=np.int32)
    return off, pid


def find_all(keyword: bytes, text: bytes) -> np.ndarray:
    """Every start of ``keyword`` in ``text`` (overlaps included), via the
    library substring search; used for per-keyword completeness checks on
    texts too large for ``brute_match``."""
    res = []
    start = text.find(keyword)
    while start >= 0:
        res.append(start)
        start = text.find(keyword, start + 1)
    return np.array(res, dtype=np.int64)
