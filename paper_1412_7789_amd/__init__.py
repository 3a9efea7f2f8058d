"""MI355X (gfx950) failure-less Aho-Corasick (PFAC) multi-pattern matcher.

The matching runs in ``libpfac.so`` (HIP kernels behind the C ABI declared in
``include/pfac.h``); this package only marshals arguments.  Importing it does
not load the library; the first call does, and raises ``ImportError`` if the
library was not built.
"""

from ._lib import (  # noqa: F401
    AC_POLICY_AUTO, AC_POLICY_FILTERED, AC_POLICY_DIRECT,
    AC_FILTER_AUTO, AC_FILTER_BYTES17, AC_FILTER_BITS20, AC_FILTER_BYTES16, AC_FILTER_BITS19, AC_FILTER_DUAL19, AC_FILTER_PAIR20,
    AC_LAUNCH_TIME_SCAN, AC_RAN_CPU, AC_RAN_GPU, AC_SERVE_BATCHED, AC_SERVE_FIFO, EXPORTS, SERVE_EXPORTS, LIB_PATH, PfacError, load,
)
from .api import (Automaton, Plan, last_scan_ms, last_scan_split, launch_config, probe_read,  # noqa: F401
                  release_stream, sorted_pairs)
from .serve import Server, serve_charge, serve_plan, server_opts  # noqa: F401
