"""Python face of the C ABI: argument marshalling only.

Every step of matching runs in the HIP library; PyTorch supplies device
memory (tensors) and streams.  Functions raise ``PfacError`` on a negative
return code and ``ImportError`` when the library has not been built.
"""

from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L


def _stream_ptr(stream) -> int:
    """Raw HIP stream handle: `stream`, else the current device's current
    stream."""
    import torch
    if stream is not None:
        return stream.cuda_stream
    return torch._C._cuda_getCurrentRawStream(torch.cuda.current_device())


def _csr(keywords: Sequence[bytes]) -> Tuple[np.ndarray, np.ndarray]:
    lens = np.fromiter((len(k) for k in keywords), dtype=np.int64, count=len(keywords))
    offs = np.zeros(len(keywords) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    flat = np.frombuffer(b"".join(keywords) or b"\0", dtype=np.uint8).copy()
    return flat, offs


def launch_config(policy: int = 0, filter: int = 0, block: int = 0, segs: int = 0,
                  grid_per_cu: int = 0, table_in_lds: int = 0, flags: int = 0, stride: int = 0) -> L.Launch:
    cfg = L.Launch()
    cfg.policy, cfg.filter, cfg.block, cfg.segs = policy, filter, block, segs
    cfg.grid_per_cu, cfg.table_in_lds, cfg.flags, cfg.stride = grid_per_cu, table_in_lds, flags, stride
    return cfg


def last_scan_ms() -> float:
    """Scan-kernel time of this thread's last synchronous call made with
    ``flags=AC_LAUNCH_TIME_SCAN`` (HIP events on the call's stream)."""
    return float(L.load().ac_last_scan_ms())


def last_scan_split() -> Tuple[float, float]:
    """(streaming kernel ms, walk kernel ms) of the same last timed call."""
    a, b = ctypes.c_float(), ctypes.c_float()
    L.load().ac_last_scan_split(ctypes.byref(a), ctypes.byref(b))
    return float(a.value), float(b.value)


def probe_read(buf, out, stream=None) -> None:
    """Enqueue the read-bandwidth probe over a uint8 CUDA tensor (16-byte
    aligned, length a multiple of 16); ``out`` is a 1-element int32 tensor."""
    L.check(L.load().ac_probe_read(ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "ac_probe_read")


def release_stream(stream=None) -> None:
    """Free the library's scratch for ``stream`` (idle) before it is destroyed."""
    L.check(L.load().ac_release_stream(_stream_ptr(stream)), "ac_release_stream")


def _opts(dense_budget_bytes: int, hash_multiplier: int) -> L.BuildOpts:
    o = L.BuildOpts()
    o.dense_budget_bytes = dense_budget_bytes
    o.hash_multiplier = hash_multiplier
    return o


def _host_bytes(text) -> np.ndarray:
    buf = np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else np.asarray(text)
    if buf.dtype != np.uint8 or buf.ndim != 1:
        raise TypeError("host text must be a 1-D uint8 array or bytes")
    return np.ascontiguousarray(buf)


def _host_call(fn, h, text, capacity, *tail):
    """Runs a host-output matcher call, growing the output arrays once if the
    first capacity was too small; returns (offsets, pattern_ids, count)."""
    buf = _host_bytes(text)
    cap = capacity if capacity is not None else max(256, buf.size // 8)
    while True:
        off = np.empty(max(cap, 1), dtype=np.int64)
        pid = np.empty(max(cap, 1), dtype=np.int32)
        n = L.check(fn(h, buf.ctypes.data if buf.size else None, buf.size, off.ctypes.data, pid.ctypes.data,
                       cap, *tail), fn.__name__)
        if n <= cap:
            return off[:n], pid[:n], n
        cap = n


class Plan:
    """Host-side build result (``ac_compile``): tables for inspection, no GPU."""

    def __init__(self, keywords: Sequence[bytes], dense_budget_bytes: int = 0, hash_multiplier: int = 0):
        lib = L.load()
        flat, offs = _csr(keywords)
        h = ctypes.c_void_p()
        opts = _opts(dense_budget_bytes, hash_multiplier)
        L.check(lib.ac_compile(flat.ctypes.data, offs.ctypes.data, len(keywords), ctypes.byref(opts),
                               ctypes.byref(h)), "ac_compile")
        self._h = h

    def info(self) -> Dict[str, float]:
        inf = L.Info()
        L.check(L.load().ac_plan_info(self._h, ctypes.byref(inf)), "ac_plan_info")
        return inf.as_dict()

    def export(self, table: int, dtype) -> np.ndarray:
        lib = L.load()
        nbytes = L.check(lib.ac_plan_export(self._h, table, None, 0), "ac_plan_export")
        out = np.empty(max(nbytes, 1), dtype=np.uint8)
        L.check(lib.ac_plan_export(self._h, table, out.ctypes.data, out.size), "ac_plan_export")
        return out[:nbytes].view(dtype)

    def hash(self, x: int) -> int:
        return int(L.load().ac_plan_hash(self._h, x & 0xFFFFFFFF))

    def hash2(self, x: int) -> int:
        return int(L.load().ac_plan_hash2(self._h, x & 0xFFFFFFFF))

    def prefix_buckets(self, x: int) -> Tuple[int, int]:
        b1, b2 = ctypes.c_uint32(), ctypes.c_uint32()
        L.load().ac_plan_prefix_buckets(self._h, x & 0xFFFFFFFF, ctypes.byref(b1), ctypes.byref(b2))
        return b1.value, b2.value

    def match_host(self, text, n_threads: int = 0, capacity: Optional[int] = None):
        """The library's CPU matcher (no GPU): host (offsets, pattern_ids)."""
        off, pid, _ = _host_call(L.load().ac_plan_match_host, self._h, text, capacity, n_threads)
        return off, pid

    def close(self) -> None:
        if self._h:
            L.load().ac_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Automaton:
    """A keyword set built into a device automaton on the current GPU."""

    def __init__(self, keywords: Sequence[bytes], dense_budget_bytes: int = 0, hash_multiplier: int = 0):
        lib = L.load()
        flat, offs = _csr(keywords)
        h = ctypes.c_void_p()
        opts = _opts(dense_budget_bytes, hash_multiplier)
        L.check(lib.ac_build_csr(flat.ctypes.data, offs.ctypes.data, len(keywords), ctypes.byref(opts),
                                 ctypes.byref(h)), "ac_build")
        self._h = h
        self.n_keywords = len(keywords)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def info(self) -> Dict[str, float]:
        inf = L.Info()
        L.check(L.load().ac_info(self._h, ctypes.byref(inf)), "ac_info")
        return inf.as_dict()

    def tune(self, text, stream=None) -> Dict[str, int]:
        """Time every filtered-policy choice on `text` (uint8 CUDA tensor) and
        use the fastest for later texts of similar length."""
        _check_text(text)
        cfg = L.Launch()
        L.check(L.load().ac_tune(self._h, ctypes.c_void_p(text.data_ptr()), text.numel(), _stream_ptr(stream),
                                 ctypes.byref(cfg)), "ac_tune")
        return cfg.as_dict()

    def tune_batch(self, texts, text_offsets, total_bytes: Optional[int] = None, stream=None) -> Dict[str, int]:
        """Time every filtered-policy choice on one packed batch and use the
        fastest for later batches of similar total length."""
        _check_text(texts)
        n_texts = text_offsets.numel() - 1
        total = texts.numel() if total_bytes is None else total_bytes
        cfg = L.Launch()
        L.check(L.load().ac_tune_batch(self._h, ctypes.c_void_p(texts.data_ptr()),
                                       ctypes.c_void_p(text_offsets.data_ptr()), n_texts, total,
                                       _stream_ptr(stream), ctypes.byref(cfg)), "ac_tune_batch")
        return cfg.as_dict()

    def default_launch(self, n_bytes: int) -> Dict[str, int]:
        cfg = L.Launch()
        L.check(L.load().ac_default_launch(self._h, n_bytes, ctypes.byref(cfg)), "ac_default_launch")
        return cfg.as_dict()

    def close(self) -> None:
        if self._h:
            L.load().ac_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- single text -------------------------------------------------------------
    def count(self, text, launch: Optional[L.Launch] = None, stream=None) -> int:
        """Number of matches in a uint8 CUDA tensor (no match buffers)."""
        _check_text(text)
        return L.check(L.load().ac_match_ex(self._h, ctypes.c_void_p(text.data_ptr()), text.numel(), None,
                                            ctypes.byref(launch) if launch is not None else None,
                                            _stream_ptr(stream)), "ac_match")

    def match_into(self, text, offsets, pattern_ids, launch: Optional[L.Launch] = None, stream=None) -> int:
        """Match into caller-owned int64/int32 CUDA tensors; returns the true count."""
        _check_text(text)
        m = L.Matches(offsets.data_ptr(), pattern_ids.data_ptr(), min(offsets.numel(), pattern_ids.numel()))
        return L.check(L.load().ac_match_ex(self._h, text.data_ptr(), text.numel(), ctypes.byref(m),
                                            ctypes.byref(launch) if launch is not None else None,
                                            _stream_ptr(stream)), "ac_match")

    def match(self, text, capacity: Optional[int] = None, launch: Optional[L.Launch] = None, stream=None):
        """All matches of a uint8 CUDA tensor as (offsets int64, pattern_ids int32)
        CUDA tensors, unordered.  Retries once with an exact buffer if the first
        guess was too small."""
        import torch
        cap = capacity if capacity is not None else max(1024, text.numel() // 512)
        while True:
            off = torch.empty(max(cap, 1), dtype=torch.int64, device=text.device)
            pid = torch.empty(max(cap, 1), dtype=torch.int32, device=text.device)
            n = self.match_into(text, off[:cap], pid[:cap], launch=launch, stream=stream)
            if n <= cap:
                return off[:n], pid[:n]
            cap = n

    def match_async(self, text, offsets, pattern_ids, d_count, launch: Optional[L.Launch] = None,
                    stream=None) -> None:
        """Enqueue only; the count lands in ``d_count`` (int64 CUDA tensor)."""
        _check_text(text)
        m = L.Matches(ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(pattern_ids.data_ptr()),
                      min(offsets.numel(), pattern_ids.numel()))
        L.check(L.load().ac_match_async(self._h, ctypes.c_void_p(text.data_ptr()), text.numel(),
                                        ctypes.byref(m),
                                        ctypes.byref(launch) if launch is not None else None,
                                        ctypes.c_void_p(d_count.data_ptr()), _stream_ptr(stream)),
                "ac_match_async")

    def match_async_noalloc(self, text, offsets, pattern_ids, d_count, launch: Optional[L.Launch] = None,
                            stream=None) -> None:
        """As ``match_async``, with the library's fixed device array as
        scratch (no device allocation; calls on one GPU must not overlap)."""
        _check_text(text)
        m = L.Matches(ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(pattern_ids.data_ptr()),
                      min(offsets.numel(), pattern_ids.numel()))
        L.check(L.load().ac_match_async_noalloc(self._h, ctypes.c_void_p(text.data_ptr()), text.numel(),
                                                ctypes.byref(m),
                                                ctypes.byref(launch) if launch is not None else None,
                                                ctypes.c_void_p(d_count.data_ptr()), _stream_ptr(stream)),
                "ac_match_async_noalloc")

    # -- CPU matcher and CPU/GPU dispatch ---------------------------------------
    def match_host(self, text, n_threads: int = 0, capacity: Optional[int] = None):
        """Host text -> host (offsets, pattern_ids) on the library's CPU matcher."""
        off, pid, _ = _host_call(L.load().ac_match_host, self._h, text, capacity, n_threads)
        return off, pid

    def match_dispatch(self, text, capacity: Optional[int] = None, stream=None):
        """Host text -> host (offsets, pattern_ids, ran_on) on the CPU below the
        dispatch threshold, else on the GPU (ran_on: AC_RAN_CPU / AC_RAN_GPU)."""
        ran = ctypes.c_int32(0)
        off, pid, _ = _host_call(L.load().ac_match_dispatch, self._h, text, capacity, _stream_ptr(stream),
                                 ctypes.byref(ran))
        return off, pid, ran.value

    @property
    def dispatch_threshold(self) -> int:
        return int(L.check(L.load().ac_dispatch_threshold(self._h), "ac_dispatch_threshold"))

    @dispatch_threshold.setter
    def dispatch_threshold(self, nbytes: int) -> None:
        L.check(L.load().ac_set_dispatch_threshold(self._h, int(nbytes)), "ac_set_dispatch_threshold")

    def calibrate_dispatch(self, sample, stream=None) -> int:
        """Measures the CPU/GPU crossover on prefixes of a host sample and sets
        the dispatch threshold to it; returns the threshold."""
        buf = _host_bytes(sample)
        thr = ctypes.c_int64(0)
        L.check(L.load().ac_calibrate_dispatch(self._h, buf.ctypes.data, buf.size, _stream_ptr(stream),
                                               ctypes.byref(thr)), "ac_calibrate_dispatch")
        return thr.value

    # -- batches -----------------------------------------------------------------
    def match_batch_into(self, texts, text_offsets, text_ids, offsets, pattern_ids, per_text=None,
                         launch: Optional[L.Launch] = None, stream=None, total_bytes: Optional[int] = None) -> int:
        _check_text(texts)
        n_texts = text_offsets.numel() - 1
        total = texts.numel() if total_bytes is None else total_bytes
        cap = min(offsets.numel(), pattern_ids.numel(), text_ids.numel())
        m = L.BatchMatches(ctypes.c_void_p(text_ids.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                           ctypes.c_void_p(pattern_ids.data_ptr()), cap,
                           ctypes.c_void_p(per_text.data_ptr()) if per_text is not None else None)
        return L.check(L.load().ac_match_batch(self._h, texts.data_ptr(), text_offsets.data_ptr(), n_texts, total,
                                               ctypes.byref(m),
                                               ctypes.byref(launch) if launch is not None else None,
                                               _stream_ptr(stream)), "ac_match_batch")

    def match_batch_async(self, texts, text_offsets, text_ids, offsets, pattern_ids, d_count, per_text=None,
                          launch: Optional[L.Launch] = None, stream=None, total_bytes: Optional[int] = None) -> None:
        """Enqueue a batch scan only; the total count lands in ``d_count``
        (int64 CUDA tensor).  Capturable in a HIP graph once the stream has
        run a batch at least as large."""
        _check_text(texts)
        n_texts = text_offsets.numel() - 1
        total = texts.numel() if total_bytes is None else total_bytes
        cap = min(offsets.numel(), pattern_ids.numel(), text_ids.numel())
        m = L.BatchMatches(ctypes.c_void_p(text_ids.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                           ctypes.c_void_p(pattern_ids.data_ptr()), cap,
                           ctypes.c_void_p(per_text.data_ptr()) if per_text is not None else None)
        L.check(L.load().ac_match_batch_async(self._h, ctypes.c_void_p(texts.data_ptr()),
                                              ctypes.c_void_p(text_offsets.data_ptr()), n_texts, total,
                                              ctypes.byref(m),
                                              ctypes.byref(launch) if launch is not None else None,
                                              ctypes.c_void_p(d_count.data_ptr()), _stream_ptr(stream)),
                "ac_match_batch_async")

    def match_batch(self, texts, text_offsets, capacity: Optional[int] = None,
                    launch: Optional[L.Launch] = None, stream=None):
        """Match a packed batch; returns (text_ids, offsets, pattern_ids, per_text_count)."""
        import torch
        n_texts = text_offsets.numel() - 1
        cap = capacity if capacity is not None else max(1024, texts.numel() // 512)
        while True:
            dev = texts.device
            tid = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            off = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
            pid = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            per = torch.empty(max(n_texts, 1), dtype=torch.int64, device=dev)
            n = self.match_batch_into(texts, text_offsets, tid[:cap], off[:cap], pid[:cap], per,
                                      launch=launch, stream=stream)
            if n <= cap:
                return tid[:n], off[:n], pid[:n], per[:n_texts]
            cap = n


def _check_text(t) -> None:
    import torch
    if t.dtype != torch.uint8 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("text must be a contiguous uint8 CUDA tensor")


def sorted_pairs(offsets, pattern_ids) -> Tuple[np.ndarray, np.ndarray]:
    """Host copy of a match set sorted by (offset, id), for comparisons."""
    off = offsets.cpu().numpy().astype(np.int64)
    pid = pattern_ids.cpu().numpy().astype(np.int32)
    order = np.lexsort((pid, off))
    return off[order], pid[order]
