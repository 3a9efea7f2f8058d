"""CPU oracle for the failure-less Aho-Corasick matcher.  TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  It shares no code with the GPU library and imports
nothing from it; the only module both sides use is ``workloads`` (seeded input
generation, no matching arithmetic).

Contents:

* ``ac``     - a plain serial Aho-Corasick machine with Goto, Failure and
               Output functions (paper, Section II, Fig. 4), in C
               (``ac_oracle.c``) behind ctypes.
* ``brute``  - the definition of the result, written out: every (offset, id)
               with ``text[offset : offset + |k_id|] == k_id``.  Pure Python,
               for tiny inputs only.
* ``build``  - compiles ``ac_oracle.c`` with gcc.
"""

from .ac import Oracle, oracle_match, load_library  # noqa: F401
from .brute import brute_match, find_all  # noqa: F401
