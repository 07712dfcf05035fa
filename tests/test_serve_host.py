"""CPU tests of the serving admission policy (no GPU): FIFO order, the HBM
budget, slot limits, bounded bypass of a blocked head, and rejection of
requests that can never fit."""
import pytest

from paper_2308_01999_amd.serve import Admission


def test_fifo_within_budget_and_slots():
    a = Admission(budget_bytes=100, slots=2)
    for rid, fp in [(0, 30), (1, 30), (2, 30)]:
        a.add(rid, fp)
    assert a.pick() == (0, 30)
    assert a.pick() == (1, 30)
    assert a.pick() is None          # both slots busy
    a.release(30)
    assert a.pick() == (2, 30)
    assert a.used == 60 and a.busy == 2


def test_budget_blocks_until_release():
    a = Admission(budget_bytes=100, slots=8)
    a.add(0, 70)
    a.add(1, 70)
    assert a.pick() == (0, 70)
    assert a.pick() is None          # 140 > 100
    a.release(70)
    assert a.pick() == (1, 70)


def test_bounded_bypass_of_blocked_head():
    a = Admission(budget_bytes=100, slots=16, max_bypass=2)
    a.add(0, 60)
    assert a.pick() == (0, 60)
    a.add(1, 80)                     # head: does not fit while 0 runs
    for rid in range(2, 6):
        a.add(rid, 10)
    assert a.pick() == (2, 10)       # bypass 1
    assert a.pick() == (3, 10)       # bypass 2
    assert a.pick() is None          # no more bypass while the head waits
    a.release(60)
    a.release(10)
    a.release(10)
    assert a.pick() == (1, 80)       # head admitted first
    assert a.pick() == (4, 10)
    assert a.pick() == (5, 10)


def test_oversized_request_rejected():
    a = Admission(budget_bytes=100, slots=1)
    with pytest.raises(ValueError):
        a.add(0, 101)
