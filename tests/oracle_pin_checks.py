"""Pin checks run against an oracle library given on the command line.

Used by ``test_oracle_mutants.py``: each planted mistake in a copy of the
oracle's C source must make at least one of these checks fail (exit status 1)
or crash/hang the child process.  Exit status 0 means every check passed.
"""

import os
import random
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle.ac import Oracle  # noqa: E402
from oracle.brute import brute_match  # noqa: E402


def pairs(res):
    off, pid = res
    return list(zip(off.tolist(), pid.tolist()))


def run(lib_path: str) -> bool:
    def om(kws, text):
        o = Oracle(kws, lib_path=lib_path)
        try:
            return pairs(o.match(text))
        finally:
            o.close()

    ok = True
    # Fig. 4 keyword set, worked scan
    ok &= om([b"AB", b"ABG", b"BEDE", b"ED"], b"ABGBEDED") == [(0, 0), (0, 1), (3, 2), (4, 3), (6, 3)]
    ok &= om([b"abab"], b"ababab") == [(0, 0), (2, 0)]
    ok &= om([b"a", b"ab", b"abc", b"bc", b"c"], b"abc") == [(0, 0), (0, 1), (0, 2), (1, 3), (2, 4)]
    rng = random.Random(5)
    for alphabet in ([97, 98], [97, 98, 99, 100], list(range(256))):
        for _ in range(60):
            kws = [bytes(rng.choice(alphabet) for _ in range(rng.randint(1, 6)))
                   for _ in range(rng.randint(1, 8))]
            text = bytes(rng.choice(alphabet) for _ in range(rng.randint(0, 80)))
            ok &= om(kws, text) == pairs(brute_match(kws, text))
    return bool(ok)


if __name__ == "__main__":
    sys.exit(0 if run(sys.argv[1]) else 1)
