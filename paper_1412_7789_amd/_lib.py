"""ctypes declarations of the C ABI in ``include/pfac.h`` (libpfac.so)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PFAC_LIBRARY points the binding at another build (the sanitized one)
LIB_PATH = os.environ.get("PFAC_LIBRARY") or os.path.join(HERE, "libpfac.so")

AC_OK, AC_EINVAL, AC_ENOMEM, AC_EHIP, AC_ENOTSUP = 0, -1, -2, -3, -4
AC_POLICY_AUTO, AC_POLICY_FILTERED, AC_POLICY_DIRECT = 0, 1, 2
AC_FILTER_AUTO, AC_FILTER_BYTES17, AC_FILTER_BITS20, AC_FILTER_BYTES16, AC_FILTER_BITS19 = 0, 1, 2, 3, 4
AC_FILTER_DUAL19 = 5
AC_FILTER_PAIR20 = 6
AC_TABLE_CLASS_MAP, AC_TABLE_DENSE, AC_TABLE_NODE, AC_TABLE_LABEL = 1, 2, 3, 4
AC_TABLE_OUT_OFF, AC_TABLE_OUT_PID, AC_TABLE_DEPTH, AC_TABLE_FILTER_BASE = 5, 6, 7, 100
AC_TABLE_PREFIX, AC_TABLE_TAIL, AC_TABLE_TAIL_INFO = 8, 9, 10

# every symbol include/pfac.h declares
EXPORTS = [
    "ac_build", "ac_build_csr", "ac_free", "ac_match", "ac_match_ex", "ac_match_async",
    "ac_match_batch", "ac_match_batch_async", "ac_info", "ac_default_launch",
    "ac_last_error", "ac_compile", "ac_plan_info", "ac_plan_export", "ac_plan_hash",
    "ac_plan_free", "ac_last_scan_ms", "ac_last_scan_split", "ac_probe_read", "ac_plan_prefix_buckets",
    "ac_plan_hash2", "ac_tune", "ac_match_async_noalloc",
    "ac_match_host", "ac_plan_match_host", "ac_match_dispatch", "ac_set_dispatch_threshold",
    "ac_dispatch_threshold", "ac_calibrate_dispatch", "ac_tune_batch", "ac_release_stream",
]
AC_RAN_CPU, AC_RAN_GPU = 1, 2
# every symbol include/pfac_serve.h declares
SERVE_EXPORTS = [
    "ac_server_create", "ac_server_destroy", "ac_server_add_automaton", "ac_server_submit",
    "ac_server_wait", "ac_server_poll", "ac_server_release", "ac_server_replay", "ac_server_get_stats",
    "ac_serve_charge", "ac_serve_plan",
]
AC_SERVE_BATCHED, AC_SERVE_FIFO = 0, 1
AC_LAUNCH_TIME_SCAN = 1


class BuildOpts(ctypes.Structure):
    _fields_ = [("dense_budget_bytes", ctypes.c_int64), ("hash_multiplier", ctypes.c_uint32),
                ("reserved", ctypes.c_int32 * 7)]


class Matches(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_void_p), ("pattern_id", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class BatchMatches(ctypes.Structure):
    _fields_ = [("text_id", ctypes.c_void_p), ("offset", ctypes.c_void_p), ("pattern_id", ctypes.c_void_p),
                ("capacity", ctypes.c_int64), ("per_text_count", ctypes.c_void_p)]


class Launch(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("filter", ctypes.c_int32), ("block", ctypes.c_int32),
                ("segs", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32), ("table_in_lds", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("stride", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Info(ctypes.Structure):
    _fields_ = [("n_patterns", ctypes.c_int32), ("n_states", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("min_len", ctypes.c_int32), ("max_len", ctypes.c_int32), ("prefix_len", ctypes.c_int32),
                ("n_dense_states", ctypes.c_int32), ("dense_depth", ctypes.c_int32),
                ("n_prefixes", ctypes.c_int32), ("n_windows2", ctypes.c_int32),
                ("dense_bytes", ctypes.c_int64), ("compact_bytes", ctypes.c_int64),
                ("output_bytes", ctypes.c_int64), ("filter_bytes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double),
                ("prefix_table_bytes", ctypes.c_int64), ("tail_bytes", ctypes.c_int64),
                ("n_windows4", ctypes.c_int32), ("n_quads4", ctypes.c_int32), ("n_quads2", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class ServerOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("max_batch_bytes", ctypes.c_int64), ("max_batch_texts", ctypes.c_int32),
                ("matches_per_kib", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_requests", ctypes.c_int32), ("count", ctypes.c_int64),
                ("offset", ctypes.POINTER(ctypes.c_int64)), ("pattern_id", ctypes.POINTER(ctypes.c_int32)),
                ("submit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("batches", ctypes.c_int64), ("text_bytes", ctypes.c_int64),
                ("admission_waits", ctypes.c_int64), ("rescans", ctypes.c_int64), ("peak_charged", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 3)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpfac.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.environ.get("PFAC_NO_TORCH"):
        try:
            # torch's HIP runtime must be the one loaded: the library then shares
            # it (and its device context) instead of loading a second copy
            import torch  # noqa: F401
        except ImportError:
            pass
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_1412_7789_amd.build, or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "ac_build": (ctypes.c_int, [vp, vp, i32, vp, vp]),
        "ac_build_csr": (ctypes.c_int, [vp, vp, i32, vp, vp]),
        "ac_free": (None, [vp]),
        "ac_match": (i64, [vp, vp, i64, vp, vp]),
        "ac_match_ex": (i64, [vp, vp, i64, vp, vp, vp]),
        "ac_match_async": (ctypes.c_int, [vp, vp, i64, vp, vp, vp, vp]),
        "ac_match_async_noalloc": (ctypes.c_int, [vp, vp, i64, vp, vp, vp, vp]),
        "ac_match_host": (i64, [vp, vp, i64, vp, vp, i64, i32]),
        "ac_plan_match_host": (i64, [vp, vp, i64, vp, vp, i64, i32]),
        "ac_match_dispatch": (i64, [vp, vp, i64, vp, vp, i64, vp, vp]),
        "ac_set_dispatch_threshold": (ctypes.c_int, [vp, i64]),
        "ac_dispatch_threshold": (i64, [vp]),
        "ac_calibrate_dispatch": (ctypes.c_int, [vp, vp, i64, vp, vp]),
        "ac_tune_batch": (ctypes.c_int, [vp, vp, vp, i32, i64, vp, vp]),
        "ac_match_batch": (i64, [vp, vp, vp, i32, i64, vp, vp, vp]),
        "ac_match_batch_async": (ctypes.c_int, [vp, vp, vp, i32, i64, vp, vp, vp, vp]),
        "ac_info": (ctypes.c_int, [vp, vp]),
        "ac_default_launch": (ctypes.c_int, [vp, i64, vp]),
        "ac_tune": (ctypes.c_int, [vp, vp, i64, vp, vp]),
        "ac_last_error": (ctypes.c_char_p, []),
        "ac_compile": (ctypes.c_int, [vp, vp, i32, vp, vp]),
        "ac_plan_info": (ctypes.c_int, [vp, vp]),
        "ac_plan_export": (i64, [vp, i32, vp, i64]),
        "ac_plan_hash": (u32, [vp, u32]),
        "ac_plan_hash2": (u32, [vp, u32]),
        "ac_plan_prefix_buckets": (None, [vp, u32, vp, vp]),
        "ac_plan_free": (None, [vp]),
        "ac_last_scan_ms": (ctypes.c_float, []),
        "ac_last_scan_split": (None, [vp, vp]),
        "ac_probe_read": (ctypes.c_int, [vp, i64, vp, vp]),
        "ac_release_stream": (ctypes.c_int, [vp]),
        "ac_server_create": (ctypes.c_int, [vp, vp]),
        "ac_server_destroy": (None, [vp]),
        "ac_server_add_automaton": (ctypes.c_int, [vp, vp]),
        "ac_server_submit": (i64, [vp, i32, vp, i64]),
        "ac_server_wait": (ctypes.c_int, [vp, i64, vp]),
        "ac_server_poll": (ctypes.c_int, [vp, i64, vp]),
        "ac_server_release": (None, [vp, i64]),
        "ac_server_replay": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "ac_server_get_stats": (ctypes.c_int, [vp, vp]),
        "ac_serve_charge": (i64, [vp, i64]),
        "ac_serve_plan": (i32, [vp, i32, vp, vp, i64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PfacError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().ac_last_error()
        super().__init__(f"{where} failed ({code}): {msg.decode() if msg else ''}")
        self.code = code


def check(rc: int, where: str) -> int:
    if rc < 0:
        raise PfacError(rc, where)
    return rc
