"""Seeded generators for the five matcher workloads and the paper's own one.

Every draw comes from ``numpy.random.SeedSequence(seed).spawn(7)``; the child
streams are used in a fixed order so that a test, the bench and the script that
writes stored expected values all regenerate byte-identical inputs:

    [0] keyword bytes      [1] keyword lengths     [2] text bytes
    [3] plant counts       [4] plant pids/offsets  [5] request trace
    [6] batch text lengths

Recipes (all lengths and bytes uniform over closed integer ranges):

* tiny      - 64 keywords, |k| in 4..12 over a..z; 1 MiB of a..z; exactly 2000
              planted keyword copies.
* sweep     - 1000 keywords, |k| in 8..32 over printable ASCII 0x20..0x7E;
              text of any size over the same bytes; Poisson(N/4096) plants.
* large     - 20000 keywords, |k| in 16..64 over bytes 0..255, 30 % of them
              (the last 6000) start with a copy of a 4..12 byte prefix of one of
              the first 14000; uniform random bytes; Poisson(N/65536) plants.
* batched   - 2000 printable keywords, |k| in 8..32; 4096 texts with
              log-normal lengths (median 8 KiB, sigma 2.1) clipped to
              [64 B, 4 MiB]; Poisson(len/4096) plants per text.
* served    - four byte-alphabet automata of 500, 5000, 20000 and 50000
              keywords, |k| in 8..64; a 256 MiB pool of random bytes carrying
              Poisson(pool/65536) plants of each automaton; Poisson arrivals at
              2000/s, each picking an automaton uniformly and a slice of the
              pool of log-uniform size in [1 KiB, 64 MiB].

Plants are written in draw order, so a later plant may overwrite an earlier
one: the plant log is a hint, never the ground truth.  Duplicate keywords are
redrawn so that every workload here has distinct keywords (the matcher itself
accepts duplicates).
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

KIB = 1 << 10
MIB = 1 << 20
GIB = 1 << 30

# Text sizes of the crossover sweep: 1 KiB, 16 KiB, ..., 1 GiB (x16 steps).
SWEEP_SIZES = [KIB * (16 ** i) for i in range(6)]


def _streams(seed: int) -> List[np.random.Generator]:
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(7)]


@dataclasses.dataclass(frozen=True)
class KeywordSpec:
    n: int
    len_lo: int
    len_hi: int
    byte_lo: int
    byte_hi: int
    shared_frac: float = 0.0   # fraction of keywords that copy another's prefix
    shared_lo: int = 0         # copied prefix length range
    shared_hi: int = 0


SPECS = {
    "tiny": KeywordSpec(64, 4, 12, 0x61, 0x7A),
    "sweep": KeywordSpec(1000, 8, 32, 0x20, 0x7E),
    "large": KeywordSpec(20000, 16, 64, 0x00, 0xFF, 0.30, 4, 12),
    "batched": KeywordSpec(2000, 8, 32, 0x20, 0x7E),
    "served_500": KeywordSpec(500, 8, 64, 0x00, 0xFF),
    "served_5000": KeywordSpec(5000, 8, 64, 0x00, 0xFF),
    "served_20000": KeywordSpec(20000, 8, 64, 0x00, 0xFF),
    "served_50000": KeywordSpec(50000, 8, 64, 0x00, 0xFF),
}


def make_keywords(spec: KeywordSpec, rng_bytes: np.random.Generator,
                  rng_len: np.random.Generator) -> List[bytes]:
    """Draw ``spec.n`` distinct keywords."""
    n = spec.n
    lengths = rng_len.integers(spec.len_lo, spec.len_hi + 1, size=n)
    n_shared = int(round(spec.shared_frac * n))
    n_free = n - n_shared
    kws: List[bytes] = []
    seen = set()

    def fresh(length: int) -> bytes:
        return rng_bytes.integers(spec.byte_lo, spec.byte_hi + 1, size=int(length),
                                  dtype=np.uint8).tobytes()

    for i in range(n):
        length = int(lengths[i])
        while True:
            if i < n_free:
                kw = fresh(length)
            else:
                donor = kws[int(rng_bytes.integers(0, n_free))]
                plen = int(rng_bytes.integers(spec.shared_lo, spec.shared_hi + 1))
                plen = min(plen, length, len(donor))
                kw = donor[:plen] + fresh(length - plen)
            if kw not in seen:
                break
        seen.add(kw)
        kws.append(kw)
    return kws


def make_text(n_bytes: int, byte_lo: int, byte_hi: int,
              rng: np.random.Generator) -> np.ndarray:
    """Uniform random text over the closed byte range."""
    return rng.integers(byte_lo, byte_hi + 1, size=int(n_bytes), dtype=np.uint8)


def plant(text: np.ndarray, keywords: Sequence[bytes], count: int,
          rng: np.random.Generator, lo: int = 0, hi: Optional[int] = None
          ) -> List[Tuple[int, int]]:
    """Write ``count`` keyword copies into ``text[lo:hi]`` in draw order.

    Returns the plant log [(offset, pid)] (offsets relative to ``text``).
    Plants whose keyword is longer than the window are skipped.
    """
    hi = len(text) if hi is None else hi
    n = len(keywords)
    log: List[Tuple[int, int]] = []
    if count <= 0 or n == 0:
        return log
    pids = rng.integers(0, n, size=count)
    u = rng.random(size=count)
    width = hi - lo
    for pid, uu in zip(pids.tolist(), u.tolist()):
        kw = keywords[pid]
        room = width - len(kw)
        if room < 0:
            continue
        off = lo + min(int(uu * (room + 1)), room)
        text[off:off + len(kw)] = np.frombuffer(kw, dtype=np.uint8)
        log.append((off, pid))
    return log


def keywords_to_csr(keywords: Sequence[bytes]) -> Tuple[np.ndarray, np.ndarray]:
    """Pack keywords as (bytes uint8[sum|k|], offsets int64[n+1])."""
    lens = np.fromiter((len(k) for k in keywords), dtype=np.int64, count=len(keywords))
    offs = np.zeros(len(keywords) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    flat = np.frombuffer(b"".join(keywords), dtype=np.uint8).copy()
    return flat, offs


@dataclasses.dataclass
class Workload:
    name: str
    keywords: List[bytes]
    text: np.ndarray
    plants: List[Tuple[int, int]]


@dataclasses.dataclass
class BatchWorkload:
    name: str
    keywords: List[bytes]
    texts: np.ndarray          # concatenated texts
    offsets: np.ndarray        # int64[n_texts + 1]
    plants: List[Tuple[int, int, int]]  # (text_id, offset, pid)


@dataclasses.dataclass
class ServedWorkload:
    name: str
    automata: List[List[bytes]]
    pool: np.ndarray
    # per request: arrival time (s), automaton index, pool start, length
    arrivals: np.ndarray
    automaton: np.ndarray
    start: np.ndarray
    length: np.ndarray


def config_tiny(seed: int = 0) -> Workload:
    """64 keywords over a..z, 1 MiB of a..z text, exactly 2000 plants."""
    r = _streams(seed)
    spec = SPECS["tiny"]
    kws = make_keywords(spec, r[0], r[1])
    text = make_text(MIB, spec.byte_lo, spec.byte_hi, r[2])
    log = plant(text, kws, 2000, r[4])
    return Workload("tiny", kws, text, log)


def config_sweep(n_bytes: int, seed: int = 0) -> Workload:
    """1000 printable keywords; printable text of ``n_bytes``; 1 plant / 4 KiB."""
    r = _streams(seed)
    spec = SPECS["sweep"]
    kws = make_keywords(spec, r[0], r[1])
    text = make_text(n_bytes, spec.byte_lo, spec.byte_hi, r[2])
    count = int(r[3].poisson(n_bytes / 4096.0))
    log = plant(text, kws, count, r[4])
    return Workload(f"sweep_{n_bytes}", kws, text, log)


def config_large_automaton(n_bytes: int = GIB, seed: int = 0) -> Workload:
    """20000 byte keywords (30 % prefix-shared); random bytes; 1 plant / 64 KiB."""
    r = _streams(seed)
    spec = SPECS["large"]
    kws = make_keywords(spec, r[0], r[1])
    text = make_text(n_bytes, 0, 255, r[2])
    count = int(r[3].poisson(n_bytes / 65536.0))
    log = plant(text, kws, count, r[4])
    return Workload(f"large_{n_bytes}", kws, text, log)


def config_batched(seed: int = 0, n_texts: int = 4096, median: float = 8 * KIB,
                   sigma: float = 2.1, lo: int = 64, hi: int = 4 * MIB) -> BatchWorkload:
    """2000 printable keywords; 4096 log-normal-length texts; 1 plant / 4 KiB."""
    r = _streams(seed)
    spec = SPECS["batched"]
    kws = make_keywords(spec, r[0], r[1])
    lens = np.exp(r[6].normal(np.log(median), sigma, size=n_texts))
    lens = np.clip(np.rint(lens), lo, hi).astype(np.int64)
    offsets = np.zeros(n_texts + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    texts = make_text(int(offsets[-1]), spec.byte_lo, spec.byte_hi, r[2])
    counts = r[3].poisson(lens / 4096.0)
    plants: List[Tuple[int, int, int]] = []
    for t in range(n_texts):
        a, b = int(offsets[t]), int(offsets[t + 1])
        for off, pid in plant(texts, kws, int(counts[t]), r[4], a, b):
            plants.append((t, off - a, pid))
    return BatchWorkload("batched", kws, texts, offsets, plants)


def config_served(seed: int = 0, n_requests: int = 2000, rate: float = 2000.0,
                  pool_bytes: int = 256 * MIB, size_lo: int = KIB,
                  size_hi: int = 64 * MIB,
                  sizes: Sequence[int] = (500, 5000, 20000, 50000)) -> ServedWorkload:
    """Four resident byte automata and an open-loop Poisson request trace."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(len(sizes) + 1)
    automata = []
    for n, kid in zip(sizes, kids[:len(sizes)]):
        rr = [np.random.default_rng(s) for s in kid.spawn(2)]
        automata.append(make_keywords(SPECS[f"served_{n}"], rr[0], rr[1]))
    r = [np.random.default_rng(s) for s in kids[-1].spawn(7)]
    pool = make_text(pool_bytes, 0, 255, r[2])
    for kws in automata:
        plant(pool, kws, int(r[3].poisson(pool_bytes / 65536.0)), r[4])
    gaps = r[5].exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = r[5].integers(0, len(sizes), size=n_requests)
    lengths = np.exp(r[5].uniform(np.log(size_lo), np.log(size_hi), size=n_requests))
    lengths = np.clip(np.rint(lengths), size_lo, size_hi).astype(np.int64)
    starts = (r[5].random(size=n_requests) * (pool_bytes - lengths + 1)).astype(np.int64)
    return ServedWorkload("served", automata, pool, arrivals, which, starts, lengths)


PAPER_LINE = (b"abcdefghijklmnopqrstuvwxyz" * 5) + b"\n"   # 131 bytes


def paper_workload(n_patterns: int, n_lines: int, seed: int = 0) -> Workload:
    """The paper's experiment (Section III): permutations of a..z as keywords,
    the alphabet written repeatedly as text.

    Only one permutation (the identity) is printed in the paper; the others are
    seeded random permutations.  The text is ``n_lines`` copies of a 131-byte
    line (the alphabet five times and a newline): every text size the paper
    quotes in Section IV is a multiple of 131.
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    alpha = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz", dtype=np.uint8)
    kws = [alpha.tobytes()]
    seen = set(kws)
    while len(kws) < n_patterns:
        p = rng.permutation(alpha).tobytes()
        if p not in seen:
            seen.add(p)
            kws.append(p)
    text = np.frombuffer(PAPER_LINE * n_lines, dtype=np.uint8).copy()
    return Workload(f"paper_{n_patterns}x{n_lines}", kws, text, [])
