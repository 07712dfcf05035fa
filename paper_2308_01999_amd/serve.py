"""Continuous-batching server for circuit requests on one GPU.

Requests (a named-gate circuit on n qubits, Pauli strings to evaluate, and
uniforms to sample with) arrive over time.  Each is fused on a host thread
pool as soon as it arrives, so fusion overlaps its wait for admission and
the device work of other requests: a small request in a few pieces at
once, each applied as soon as it is fused; a large one whole, with coupled
fusion, which saves it sweeps.  A dispatcher admits them in
arrival order as soon as a slot is free and the request's state fits the
HBM budget; later requests may pass a blocked head only a bounded number of
times, so large requests do not starve.  Some slots may be kept for small
requests (a few qubits' worth of memory and milliseconds of work), which
then never wait behind large states for a slot.  Each slot is a worker
thread with its own torch stream and libsv handle, so the work of admitted
requests overlaps on the device.  A request's state stays resident in HBM from
admission until its results are read back, then its memory is returned to
the budget and the next request is admitted.

All computation happens in libsv (host fusion in its C++, everything else
in its kernels); this module only schedules.  Every reduction in libsv is
deterministic, so a request's results are bitwise the same whether it runs
alone or among others.
"""
from __future__ import annotations

import collections
import os
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import Handle, State, fuse, sv_apply_fused, sv_expect_pauli, sv_sample

STATE_BYTES = {"c64": 8, "c128": 16}
WORKSPACE_BYTES = 64 << 20    # libsv's default handle workspace (one per slot)


def state_bytes(n: int, dtype: str) -> int:
    """Device bytes of an n-qubit state."""
    return (1 << n) * STATE_BYTES[dtype]


def sampler_scratch_bytes(n: int) -> int:
    """The sampler's per-handle prefix buffer for an n-qubit state: one
    double per 64 amplitudes, rounded up to 256 B.  libsv grows it to the
    largest state a handle has sampled and keeps it until the handle is
    destroyed."""
    return (((1 << n) // 64) * 8 + 255) & ~255


def slot_reserve(max_qubits: int) -> int:
    """Device bytes a slot holds whatever it serves: its handle workspace and
    its sampler buffer grown to the largest admissible state."""
    return WORKSPACE_BYTES + sampler_scratch_bytes(max_qubits)


def request_budget(total_bytes: int, slots: int, max_qubits: int) -> int:
    """What is left of a device-memory budget for request states once every
    slot's reserve is set aside."""
    left = total_bytes - slots * slot_reserve(max_qubits)
    if left <= 0:
        raise ValueError(f"a budget of {total_bytes} B does not cover {slots} slots of {slot_reserve(max_qubits)} B")
    return left


# Requests of up to CHUNK_QUBITS qubits (whose sweeps are short) are fused in
# contiguous pieces of about CHUNK_GATES gates, at most MAX_CHUNKS, each on
# its own pool thread: fusion, which dominates such a request's time, then
# takes a fraction as long, and the first piece is applied while the others
# are still being fused.  A piece boundary can cost a block or two; larger
# states, whose sweeps dominate, are fused whole.
CHUNK_QUBITS = 20
CHUNK_GATES = 400
MAX_CHUNKS = 4
# Requests of at least COUPLED_QUBITS qubits are fused with coupled fusion
# (phase gates deferred into the phase couplings of later blocks): about a
# fifth fewer sweeps of a large state for twice the host time, which such a
# request's sweeps dwarf.
COUPLED_QUBITS = 21


def fusion_pieces(n: int, gates: list) -> list:
    """The contiguous pieces of a request's gate list that are fused
    separately (one piece above CHUNK_QUBITS qubits)."""
    if n > CHUNK_QUBITS or len(gates) <= CHUNK_GATES:
        return [gates]
    k = min(MAX_CHUNKS, -(-len(gates) // CHUNK_GATES))
    size = -(-len(gates) // k)
    return [gates[i:i + size] for i in range(0, len(gates), size)]


def default_budget() -> int:
    """SV_HBM_BUDGET_BYTES if set (the same cap libsv applies to its own
    allocations), else 64 GiB."""
    v = os.environ.get("SV_HBM_BUDGET_BYTES", "")
    return int(v) if v.isdigit() else 64 << 30


@dataclass
class Request:
    rid: int
    n: int
    gates: list
    terms: list
    uniforms: np.ndarray
    arrival: float = 0.0          # host monotonic time of arrival (set on submit)
    fused: list | None = None     # futures of the fused pieces, made on the fusion pool (set on submit)


@dataclass
class Result:
    rid: int
    expectations: np.ndarray
    samples: np.ndarray
    fused_blocks: int
    arrival: float
    admitted: float
    done: float
    error: str = ""               # set if libsv rejected or failed the request

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Admission:
    """Pure admission policy (no GPU): FIFO with bounded bypass under a
    byte budget and slot counts.  `slots` general slots take any request;
    `small_slots` more take only requests marked small, so small requests
    never wait behind large ones for a slot.  A request that cannot start
    may be passed by later ones at most max_bypass times while it waits for
    memory or for a general slot (a small request taking a small slot the
    head could not use does not count).  Unit-tested on the CPU."""

    def __init__(self, budget_bytes: int, slots: int, max_bypass: int = 8, small_slots: int = 0):
        self.budget = budget_bytes
        self.slots = slots
        self.small_slots = small_slots
        self.max_bypass = max_bypass
        self.used = 0
        self.busy = 0          # general slots in use
        self.busy_small = 0    # small slots in use
        self.queue = collections.deque()  # (rid, footprint, small)
        self.head_bypassed = 0

    def add(self, rid: int, footprint: int, small: bool = False) -> None:
        if footprint > self.budget:
            raise ValueError(f"request {rid} needs {footprint} B, more than the budget {self.budget} B")
        self.queue.append((rid, footprint, bool(small)))

    def _slot_for(self, small: bool):
        """'small', 'general' or None: the free slot a request would take."""
        if small and self.busy_small < self.small_slots:
            return "small"
        if self.busy < self.slots:
            return "general"
        return None

    def pick(self):
        """Next request to admit as (rid, footprint, small_slot), or None.
        Reserves its slot and bytes."""
        if not self.queue:
            return None
        rid, fp, small = self.queue[0]
        cls = self._slot_for(small)
        if cls is not None and self.used + fp <= self.budget:
            self.queue.popleft()
            self.head_bypassed = 0
            return self._take(rid, fp, cls)
        for i in range(1, len(self.queue)):
            r2, f2, s2 = self.queue[i]
            c2 = self._slot_for(s2)
            if c2 is None or self.used + f2 > self.budget:
                continue
            # passing the head costs it a turn only if the head could have
            # used what this request takes: memory, or a general slot
            counts = cls is not None or c2 == "general"
            if counts and self.head_bypassed >= self.max_bypass:
                continue
            del self.queue[i]
            if counts:
                self.head_bypassed += 1
            return self._take(r2, f2, c2)
        return None

    def _take(self, rid, fp, cls):
        self.used += fp
        if cls == "small":
            self.busy_small += 1
        else:
            self.busy += 1
        return rid, fp, cls == "small"

    def release(self, footprint: int, small_slot: bool = False) -> None:
        self.used -= footprint
        if small_slot:
            self.busy_small -= 1
        else:
            self.busy -= 1


class Server:
    """Serves requests on `slots` concurrent streams within `budget_bytes`
    of device memory (default: SV_HBM_BUDGET_BYTES, else 64 GiB), complex64
    (or complex128) states, fusion width kmax (0: no fusion, one sweep per
    gate).  `small_slots` more streams serve only requests of at most
    small_qubits qubits, so those never queue behind large states for a
    slot.  Each slot's handle workspace and sampler buffer (sized for the
    largest state it may serve) are set aside first; requests are admitted
    by their state size against the rest.  Requests above max_qubits are
    rejected."""

    def __init__(self, slots: int = 4, budget_bytes: int | None = None, dtype: str = "c64", kmax: int = 5,
                 max_bypass: int = 8, max_qubits: int = 28, small_slots: int = 0, small_qubits: int = 16,
                 fuse_threads: int = 4):
        import torch
        self.dtype = dtype
        self.kmax = kmax
        self.max_qubits = max_qubits
        self.small_qubits = min(small_qubits, max_qubits)
        total = default_budget() if budget_bytes is None else budget_bytes
        left = request_budget(total, slots, max_qubits)
        if small_slots:
            left = request_budget(left, small_slots, self.small_qubits)
        self.adm = Admission(left, slots, max_bypass, small_slots)
        self.cv = threading.Condition()
        self.pending = {}        # rid -> Request
        self.results = {}        # rid -> Result
        self.ready = {False: collections.deque(), True: collections.deque()}  # admitted, per slot class
        self.stop = False
        self.fuse_pool = ThreadPoolExecutor(max_workers=fuse_threads) if kmax > 0 else None
        n_workers = slots + small_slots
        self.handles = [Handle(stream=torch.cuda.Stream()) for _ in range(n_workers)]
        self.workers = [threading.Thread(target=self._worker, args=(i, i >= slots), daemon=True)
                        for i in range(n_workers)]
        self.dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        for w in self.workers:
            w.start()
        self.dispatcher.start()

    def footprint(self, n: int) -> int:
        return state_bytes(n, self.dtype)

    def submit(self, req: Request) -> None:
        """Queues a request; raises ValueError (and keeps nothing of it) if it
        can never be admitted."""
        if req.n > self.max_qubits:
            raise ValueError(f"request {req.rid} has {req.n} qubits, more than the server's {self.max_qubits}")
        req.arrival = time.monotonic()
        with self.cv:
            self.adm.add(req.rid, self.footprint(req.n), req.n <= self.small_qubits)
            if self.fuse_pool is not None:
                coupled = req.n >= COUPLED_QUBITS
                req.fused = [self.fuse_pool.submit(fuse, part, self.kmax, 0, coupled)
                             for part in fusion_pieces(req.n, req.gates)]
            self.pending[req.rid] = req
            self.cv.notify_all()

    def _dispatch(self) -> None:
        with self.cv:
            while not self.stop:
                picked = self.adm.pick()
                if picked is None:
                    self.cv.wait(timeout=0.05)
                    continue
                rid, _, small_slot = picked
                self.ready[small_slot].append((rid, time.monotonic()))
                self.cv.notify_all()

    def _worker(self, slot: int, small_slot: bool) -> None:
        import torch
        h = self.handles[slot]
        ready = self.ready[small_slot]
        while True:
            with self.cv:
                while not ready and not self.stop:
                    self.cv.wait(timeout=0.05)
                if self.stop and not ready:
                    return
                rid, admitted = ready.popleft()
                req = self.pending.pop(rid)
            try:
                with torch.cuda.stream(h.stream):
                    res = self._run(h, req, admitted)
            except Exception as e:  # report the failure, keep serving others
                res = Result(req.rid, np.zeros(0), np.zeros(0, dtype=np.uint64), 0, req.arrival, admitted,
                             time.monotonic(), error=str(e))
            with self.cv:
                self.results[rid] = res
                self.adm.release(self.footprint(req.n), small_slot)
                self.cv.notify_all()

    def _run(self, h: Handle, req: Request, admitted: float) -> Result:
        pieces = list(req.fused) if req.fused is not None else None
        st = None
        try:
            st = State(h, req.n, self.dtype)
            if pieces is not None:
                # each piece as soon as it is fused, in order
                nb = 0
                while pieces:
                    f = pieces.pop(0).result()
                    try:
                        sv_apply_fused(st.s, f.f)
                        nb += f.count
                    finally:
                        f.free()
            else:
                st.run(req.gates)  # one sweep per gate
                nb = len(req.gates)
            exps = sv_expect_pauli(st.s, req.terms)
            smp = sv_sample(st.s, req.uniforms)
        finally:
            for fut in pieces or []:
                try:
                    fut.result().free()
                except Exception:
                    pass
            if st is not None:
                st.close()
        return Result(req.rid, exps, smp, nb, req.arrival, admitted, time.monotonic())

    def wait(self, rids, timeout: float = 600.0) -> dict:
        end = time.monotonic() + timeout
        with self.cv:
            while not all(r in self.results for r in rids):
                left = end - time.monotonic()
                if left <= 0:
                    raise TimeoutError("requests did not finish in time")
                self.cv.wait(timeout=min(left, 0.1))
            return {r: self.results[r] for r in rids}

    def close(self) -> None:
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        self.dispatcher.join()
        for w in self.workers:
            w.join()
        if self.fuse_pool is not None:
            self.fuse_pool.shutdown(wait=True)
        for h in self.handles:
            h.close()


def replay(server: Server, requests, time_scale: float = 1.0) -> dict:
    """Submits `requests` (workloads.Request) at their arrival times (scaled)
    and waits for all; returns rid -> Result."""
    t0 = time.monotonic()
    for r in requests:
        delay = t0 + r.arrival * time_scale - time.monotonic()
        if delay > 0:
            time.sleep(delay)
        server.submit(Request(r.rid, r.n, r.gates, r.terms, np.asarray(r.uniforms)))
    return server.wait([r.rid for r in requests])
