"""The paper's own experiment (Section III/IV) on the GPU: permutations of
a..z as keywords over text made of 131-byte lines (the alphabet five times
and a newline), at the text sizes the paper quotes.  The GPU match set must
equal the oracle's, and the closed forms hold: the identity permutation
occurs 5 times per line, a rotation by r four times per line, any other
permutation never."""

import sys

import numpy as np
import pytest

from oracle import oracle_match
from tests.helpers import assert_same
from workloads import paper_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

pf = None


def setup_module(module):
    global pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1412_7789_amd as _pf
    _pf.load()
    pf = _pf


def expected_count(keyword: bytes, lines: int) -> int:
    alpha = b"abcdefghijklmnopqrstuvwxyz"
    if keyword == alpha:
        return 5 * lines
    for r in range(1, 26):
        if keyword == alpha[r:] + alpha[:r]:
            return 4 * lines
    return 0


@pytest.mark.parametrize("n_patterns", [5, 10])
@pytest.mark.parametrize("lines", [10, 125, 410, 5125])
def test_paper_sizes_match_oracle_and_closed_form(n_patterns, lines):
    w = paper_workload(n_patterns, lines)
    print("paper", n_patterns, lines, len(w.text), file=sys.stderr, flush=True)
    a = pf.Automaton(w.keywords)
    off, pid = a.match(torch.from_numpy(w.text).cuda())
    got = (off.cpu().numpy(), pid.cpu().numpy())
    assert_same(got, oracle_match(w.keywords, w.text), f"paper {n_patterns}x{lines}")
    counts = np.bincount(got[1], minlength=n_patterns)
    for p, k in enumerate(w.keywords):
        assert counts[p] == expected_count(k, lines), (p, k)
    # the identity's occurrences sit at 131 j + 26 t
    ident = np.sort(got[0][got[1] == 0])
    exp = np.sort((131 * np.arange(lines)[:, None] + 26 * np.arange(5)[None, :]).ravel())
    assert (ident == exp).all()
