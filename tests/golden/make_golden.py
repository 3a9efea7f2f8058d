"""Write the stored digests in ``tests/golden/digests.txt``.

Calls only the CPU oracle (``oracle/``) and the seeded generators
(``workloads``); nothing here touches the GPU library.  Each line is

    <workload name> <match count> <sha256 of the sorted result>

where the result is serialised as the int64 start offsets followed by the
int32 keyword ids, little-endian, sorted by (offset, id).

Run:  python tests/golden/make_golden.py
"""

import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle_match  # noqa: E402
from workloads import config_sweep, config_tiny, paper_workload  # noqa: E402

OUT = os.path.join(HERE, "digests.txt")


def digest(off, pid) -> str:
    h = hashlib.sha256()
    h.update(off.astype("<i8").tobytes())
    h.update(pid.astype("<i4").tobytes())
    return h.hexdigest()


def workloads():
    yield config_tiny()
    yield config_sweep(1 << 22)
    yield paper_workload(5, 5125)
    yield paper_workload(10, 410)


def main() -> None:
    lines = ["# written by tests/golden/make_golden.py from the CPU oracle only"]
    for w in workloads():
        off, pid = oracle_match(w.keywords, w.text)
        lines.append(f"{w.name} {len(off)} {digest(off, pid)}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
