"""Shared helpers of the GPU parity tests (no matching arithmetic)."""

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
