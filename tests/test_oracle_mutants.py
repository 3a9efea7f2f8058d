"""Plant plausible mistakes in a copy of the oracle and check the pins fail.

Each mutant is a textual edit of ``oracle/ac_oracle.c`` compiled into a
temporary library; ``oracle_pin_checks.py`` then runs in a child process (a
mutant may crash or loop) and must not pass.  The committed oracle itself must
pass the same checks.
"""

import os
import subprocess
import sys

import pytest

from oracle.build import SRC, build

HERE = os.path.dirname(os.path.abspath(__file__))
CHECKS = os.path.join(HERE, "oracle_pin_checks.py")

MUTANTS = {
    "output_union_dropped": (
        "for (int32_t k = 0; k < m->st[f].n_out; ++k) {",
        "for (int32_t k = 0; k < 0; ++k) {"),
    "start_offset_off_by_one": (
        "pairs[2 * cnt] = i - m->len[p] + 1;",
        "pairs[2 * cnt] = i - m->len[p];"),
    "match_restarts_at_root": (
        "        while (go(m, st, a) < 0) st = m->st[st].fail;\n        st = go(m, st, a);",
        "        while (go(m, st, a) < 0) st = 0;\n        st = go(m, st, a);"),
    "failure_takes_parent_link": (
        "                int32_t f = go(m, st, a);",
        "                int32_t f = st;"),
    "failure_chain_single_step": (
        "                while (go(m, st, a) < 0) st = m->st[st].fail;\n                int32_t f",
        "                if (go(m, st, a) < 0) st = 0;\n                int32_t f"),
    "bisection_off_by_one": (
        "if (s->edge[mid].label < a) lo = mid + 1;",
        "if (s->edge[mid].label <= a) lo = mid + 1;"),
    "sort_by_pid_first": (
        "if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;\n    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;",
        "if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;\n    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;"),
    "last_keyword_byte_skipped": (
        "for (int64_t j = 0; j < L; ++j) {",
        "for (int64_t j = 0; j + 1 < L || j == 0; ++j) {"),
}


def _run_checks(lib: str) -> int:
    try:
        return subprocess.run([sys.executable, CHECKS, lib], timeout=60,
                              capture_output=True).returncode
    except subprocess.TimeoutExpired:
        return -999


def test_committed_oracle_passes_checks(oracle_lib, tmp_path):
    lib = build(out=str(tmp_path / "liboracle_ok.so"))
    assert _run_checks(lib) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found once in the oracle"
    mutant = tmp_path / f"{name}.c"
    mutant.write_text(src.replace(old, new))
    lib = build(src=str(mutant), out=str(tmp_path / f"lib{name}.so"), extra=["-w"])
    assert _run_checks(lib) != 0, f"mutant {name} survived the pins"
