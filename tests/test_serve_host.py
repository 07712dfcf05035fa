"""CPU tests of the serving admission policy (no GPU): FIFO order, the HBM
budget, slot limits, bounded bypass of a blocked head, slots reserved for
small requests, and rejection of requests that can never fit."""
import pytest

from paper_2308_01999_amd import serve
from paper_2308_01999_amd.serve import Admission


def test_fifo_within_budget_and_slots():
    a = Admission(budget_bytes=100, slots=2)
    for rid, fp in [(0, 30), (1, 30), (2, 30)]:
        a.add(rid, fp)
    assert a.pick() == (0, 30, False)
    assert a.pick() == (1, 30, False)
    assert a.pick() is None          # both slots busy
    a.release(30)
    assert a.pick() == (2, 30, False)
    assert a.used == 60 and a.busy == 2


def test_budget_blocks_until_release():
    a = Admission(budget_bytes=100, slots=8)
    a.add(0, 70)
    a.add(1, 70)
    assert a.pick() == (0, 70, False)
    assert a.pick() is None          # 140 > 100
    a.release(70)
    assert a.pick() == (1, 70, False)


def test_bounded_bypass_of_blocked_head():
    a = Admission(budget_bytes=100, slots=16, max_bypass=2)
    a.add(0, 60)
    assert a.pick() == (0, 60, False)
    a.add(1, 80)                     # head: does not fit while 0 runs
    for rid in range(2, 6):
        a.add(rid, 10)
    assert a.pick() == (2, 10, False)       # bypass 1
    assert a.pick() == (3, 10, False)       # bypass 2
    assert a.pick() is None          # no more bypass while the head waits
    a.release(60)
    a.release(10)
    a.release(10)
    assert a.pick() == (1, 80, False)       # head admitted first
    assert a.pick() == (4, 10, False)
    assert a.pick() == (5, 10, False)


def test_small_slots_serve_small_requests_past_large_ones():
    a = Admission(budget_bytes=1000, slots=1, small_slots=2)
    a.add(0, 100)                    # large: takes the general slot
    a.add(1, 100)                    # large: waits for the general slot
    for rid in (2, 3, 4):
        a.add(rid, 10, small=True)
    assert a.pick() == (0, 100, False)
    # the head (1) waits for a general slot; small requests take the small
    # slots without using up its bypass allowance
    assert a.pick() == (2, 10, True)
    assert a.pick() == (3, 10, True)
    assert a.pick() is None          # small slots full, general slot busy
    assert a.head_bypassed == 0
    a.release(10, small_slot=True)
    assert a.pick() == (4, 10, True)
    a.release(100)
    assert a.pick() == (1, 100, False)
    assert a.busy == 1 and a.busy_small == 2


def test_small_request_may_use_a_general_slot():
    a = Admission(budget_bytes=1000, slots=2, small_slots=1)
    for rid in (0, 1, 2):
        a.add(rid, 10, small=True)
    assert a.pick() == (0, 10, True)
    assert a.pick() == (1, 10, False)
    assert a.pick() == (2, 10, False)
    a.add(3, 500)
    assert a.pick() is None          # no general slot left for the large request


def test_small_requests_passing_a_head_blocked_by_memory_count():
    a = Admission(budget_bytes=100, slots=2, small_slots=2, max_bypass=1)
    a.add(0, 60)
    assert a.pick() == (0, 60, False)
    a.add(1, 60)                     # head: a general slot is free, memory is not
    a.add(2, 10, small=True)
    a.add(3, 10, small=True)
    assert a.pick() == (2, 10, True)  # passes the head: counts
    assert a.pick() is None          # allowance used up
    a.release(60)
    assert a.pick() == (1, 60, False)
    assert a.pick() == (3, 10, True)


def test_oversized_request_rejected():
    a = Admission(budget_bytes=100, slots=1)
    with pytest.raises(ValueError):
        a.add(0, 101)


def test_footprint_counts_slot_scratch():
    # a slot keeps its handle workspace and a sampler prefix buffer of one
    # double per 64 amplitudes of the largest state it may sample
    assert serve.sampler_scratch_bytes(28) == (1 << 28) // 8
    assert serve.sampler_scratch_bytes(10) == 256           # 16 doubles, rounded up to 256 B
    assert serve.slot_reserve(28) == (64 << 20) + (32 << 20)
    assert serve.state_bytes(28, "c64") == 2 << 30 and serve.state_bytes(10, "c128") == 16 << 10
    total = 3 << 30
    left = serve.request_budget(total, 4, 28)
    assert left == total - 4 * ((64 << 20) + (32 << 20))
    # with the reserve set aside, a 28-qubit complex64 state (2 GiB) and a
    # 27-qubit one (1 GiB) no longer fit together in 3 GiB
    a = Admission(left, 4)
    a.add(0, serve.state_bytes(28, "c64"))
    a.add(1, serve.state_bytes(27, "c64"))
    assert a.pick() == (0, 2 << 30, False)
    assert a.pick() is None
    with pytest.raises(ValueError):
        serve.request_budget(256 << 20, 4, 28)


def test_budget_from_environment(monkeypatch):
    monkeypatch.setenv("SV_HBM_BUDGET_BYTES", str(3 << 30))
    assert serve.default_budget() == 3 << 30
    monkeypatch.setenv("SV_HBM_BUDGET_BYTES", "x")
    assert serve.default_budget() == 64 << 30
    monkeypatch.delenv("SV_HBM_BUDGET_BYTES")
    assert serve.default_budget() == 64 << 30


def test_rejected_request_leaves_no_state():
    # submit() registers a request only once admission has accepted it
    srv = serve.Server.__new__(serve.Server)
    import threading
    srv.cv = threading.Condition()
    srv.pending = {}
    srv.dtype = "c64"
    srv.max_qubits = 28
    srv.small_qubits = 0
    srv.fuse_pool = None
    srv.adm = Admission(1 << 20, 1)
    with pytest.raises(ValueError):
        srv.submit(serve.Request(7, 20, [], [], None))     # 8 MiB > 1 MiB
    assert srv.pending == {} and not srv.adm.queue
    with pytest.raises(ValueError):
        srv.submit(serve.Request(8, 29, [], [], None))     # above max_qubits
    assert srv.pending == {}
    srv.submit(serve.Request(9, 10, [], [], None))
    assert list(srv.pending) == [9] and list(srv.adm.queue) == [(9, 8 << 10, False)]


def test_submit_starts_fusion_on_the_pool():
    # an admitted request is fused on the host pool right away (libsv's
    # host fuser runs without a GPU); a rejected one starts nothing
    from concurrent.futures import ThreadPoolExecutor
    import threading

    import workloads as W
    srv = serve.Server.__new__(serve.Server)
    srv.cv = threading.Condition()
    srv.pending = {}
    srv.dtype = "c64"
    srv.max_qubits = 28
    srv.small_qubits = 0
    srv.kmax = 5
    srv.fuse_pool = ThreadPoolExecutor(max_workers=1)
    srv.adm = Admission(1 << 20, 1)
    gates = W.brickwork(10, 6, 3)
    srv.submit(serve.Request(1, 10, gates, [], None))
    futs = srv.pending[1].fused
    assert len(futs) == len(serve.fusion_pieces(10, gates))
    for fut in futs:
        f = fut.result(timeout=60)
        try:
            assert 0 < f.count <= len(gates)
        finally:
            f.free()
    with pytest.raises(ValueError):
        srv.submit(serve.Request(2, 20, gates, [], None))   # 8 MiB > 1 MiB
    assert 2 not in srv.pending
    srv.fuse_pool.shutdown(wait=True)


def test_fusion_pieces_cover_the_gate_list_in_order():
    import workloads as W
    gates = W.brickwork(16, 60, 4)
    pieces = serve.fusion_pieces(16, gates)
    assert 1 < len(pieces) <= serve.MAX_CHUNKS
    assert [g for p in pieces for g in p] == gates
    assert max(len(p) for p in pieces) - min(len(p) for p in pieces) <= len(pieces)
    # large states and short lists are fused whole
    assert serve.fusion_pieces(serve.CHUNK_QUBITS + 1, gates) == [gates]
    short = gates[: serve.CHUNK_GATES]
    assert serve.fusion_pieces(16, short) == [short]
