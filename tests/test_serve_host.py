"""Host-side rules of the request server (no GPU): the admission charge and
the batch-formation rule that the engine applies to waiting requests."""

import pytest

import paper_1412_7789_amd as pf
from paper_1412_7789_amd import _lib as L


@pytest.fixture(scope="module", autouse=True)
def lib():
    return pf.load()


def test_charge_is_text_plus_reserved_match_slots():
    # at least 256 slots of 16 bytes; 4 slots per KiB by default
    assert pf.serve_charge(0) == 256 * 16
    assert pf.serve_charge(1000) == 1000 + 256 * 16
    assert pf.serve_charge(1 << 20) == (1 << 20) + 4096 * 16
    o = pf.server_opts(matches_per_kib=8)
    assert pf.serve_charge(1 << 20, o) == (1 << 20) + 8192 * 16


def test_oldest_request_leads_and_same_automaton_joins():
    big = 1 << 40
    assert pf.serve_plan([2, 1, 2, 0, 2], [10, 20, 30, 40, 50], big) == [0, 2, 4]
    assert pf.serve_plan([1], [5], big) == [0]
    assert pf.serve_plan([], [], big) == []


def test_fifo_mode_takes_one_request():
    o = pf.server_opts(mode=L.AC_SERVE_FIFO)
    assert pf.serve_plan([0, 0, 0], [10, 10, 10], 1 << 40, o) == [0]


def test_admission_wait_when_oldest_does_not_fit():
    c = pf.serve_charge(1 << 20)
    assert pf.serve_plan([0, 0], [1 << 20, 10], c - 1) == []
    # the oldest fits, the next one does not, a later small one does
    small = pf.serve_charge(10)
    assert pf.serve_plan([0, 0, 0], [1 << 20, 1 << 20, 10], c + small) == [0, 2]


def test_batch_limits():
    o = pf.server_opts(max_batch_texts=3)
    assert pf.serve_plan([0] * 6, [1] * 6, 1 << 40, o) == [0, 1, 2]
    o = pf.server_opts(max_batch_bytes=100)
    # a first request above the byte limit is served alone
    assert pf.serve_plan([0, 0], [500, 10], 1 << 40, o) == [0]
    assert pf.serve_plan([0, 0, 0, 0], [60, 50, 30, 20], 1 << 40, o) == [0, 2]


def test_bad_options_are_rejected():
    with pytest.raises(pf.PfacError):
        pf.serve_charge(10, pf.server_opts(mode=7))
    with pytest.raises(pf.PfacError):
        pf.serve_charge(10, pf.server_opts(n_streams=-1))
    with pytest.raises(pf.PfacError):
        pf.serve_charge(-1)
