#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Workload: the 30-qubit brickwork random circuit of depth 20 (U3 on every
qubit, then CZ bricks on alternating offsets; angles from seed 0), fused into
dense blocks of up to 5 qubits, on complex64 (headline) and complex128
states.  One step is one pass of the whole hot path over that circuit:
host gate fusion -> reset to |0..0> -> every fused block swept over the
state -> <Z_i> for all 30 qubits -> 2^20 samples from seeded uniforms.

``value`` is the fused-gate HBM bandwidth: the algorithmic bytes of the
fused-block sweeps (each block reads and writes the whole state once,
2 * 2^n * bytes-per-amplitude) divided by the time the GPU spends in them,
measured with HIP events on the handle's stream around every block of every
timed step.  ``ms_per_step`` is the wall time of a whole step.

Prints one JSON line.  ``--gpus`` above 1 is refused: the library keeps a
whole state on one GPU and has no multi-GPU sharding.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged over the 30-qubit
# launches of the headline circuit), each scaled by what the same counter
# reads for a plain copy of known size (FETCH_SIZE reads half the bytes a
# copy fetches, so x2.0; WRITE_SIZE reads them all, x1.0).  Valid only for the
# kernel sources the counters were taken on: their SHA-256 are recorded and
# checked at run time.
_K5_SOURCES = {"paper_2308_01999_amd/csrc/sv_apply.hip":
               "cf79059f6f509d8abd8860f662118b5c5ff6710a5ea28dc36f83deb7742e688b",
               "paper_2308_01999_amd/csrc/sv_tile.h":
               "14df7118bbe9218d6f281185a9817e4518b765bfcec4ed09243b2a5b993b5984"}
PMC_TRAFFIC = {
    # 30-qubit brickwork sweep, dispatch-weighted over all tile variants (728
    # launches of each dtype in one pass: 14 steps of 52 blocks)
    "k_tile_c64_k5": {"n": 30, "fetch_kib": 4194384.0, "write_kib": 8389899.5,
                      "fetch_scale": 2.0, "write_scale": 1.0, "sources": _K5_SOURCES},
    "k_tile_c128_k5": {"n": 30, "fetch_kib": 8388720.9, "write_kib": 16780158.6,
                       "fetch_scale": 2.0, "write_scale": 1.0, "sources": _K5_SOURCES},
}


def pmc_traffic(kernel, n):
    """Calibrated HBM bytes per launch of `kernel` at n qubits from the
    recorded counters, or None if none were taken for it or its sources have
    changed since."""
    import hashlib
    rec = PMC_TRAFFIC.get(kernel)
    if rec is None or rec["n"] != n:
        return None
    for path, digest in rec["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return int(rec["fetch_kib"] * 1024 * rec["fetch_scale"] + rec["write_kib"] * 1024 * rec["write_scale"])


def dominant_kernel_name(dt, k, n):
    """Kernel that libsv launches for an uncontrolled fused k-qubit block on
    an n-qubit state (mirrors the path choice in sv_apply.hip)."""
    if dt == "c64" and k in (4, 5) and n >= 12:
        return f"k_tile_c64_k{k}"
    if dt == "c128" and k == 5 and n >= 11:
        return "k_tile_c128_k5"
    if dt == "c64" and k == 6 and n >= 13:
        return "k_tile_c64_k6"
    if dt == "c128" and k == 6 and n >= 12:
        return "k_tile_c128_k6"
    if dt == "c64" and k in (4, 5):
        return f"k_apply_mfma_c64_k{k}"
    return f"k_apply_dense<{'float' if dt == 'c64' else 'double'}, {k}>"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    # untimed steps; they also let the handle time its k = 5 tile variants
    # on every target set of the circuit and settle on the fastest
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--kmax", type=int, default=5)
    ap.add_argument("--shots", type=int, default=1 << 20)
    ap.add_argument("--no-c128", action="store_true", help="skip the complex128 leg")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target length of the oracle sample")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-circuit leg")
    ap.add_argument("--batch-circuits", type=int, default=4096)
    ap.add_argument("--baseline-sample", type=int, default=48,
                    help="circuits of the batch run through the plain complex128 per-circuit path")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-small-slots", type=int, default=2,
                    help="extra serving slots for requests of up to 16 qubits")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="also serve at 0.25/0.5/0.75/0.9 of capacity and compare capacity with 1 slot")
    ap.add_argument("--sweep-requests", type=int, default=500)
    ap.add_argument("--no-kmax-sweep", action="store_true",
                    help="skip the unfused / kmax 4, 5, 6 comparison on the same circuit")
    ap.add_argument("--gate-sweep", action="store_true",
                    help="also time single k-qubit gates (k = 1..6) on random target sets, both dtypes")
    ap.add_argument("--seeds", type=int, default=10,
                    help="also run the headline circuit at seeds 0..K-1 (fused, one timed pass each, both dtypes)")
    ap.add_argument("--sweep-sets", type=int, default=100)
    ap.add_argument("--sweep-n64", type=int, default=None,
                    help="qubits of the gate sweep's complex64 state (default: --n; the paper's Fig. 2: 33)")
    ap.add_argument("--sweep-n128", type=int, default=None,
                    help="qubits of the gate sweep's complex128 state (default: --n; the paper's Fig. 2: 32)")
    ap.add_argument("--no-diagonal", action="store_true",
                    help="skip the diagonal / permutation gate leg (and the QFT with diagonal fusion)")
    ap.add_argument("--large", action="store_true",
                    help="also time the fused depth-12 random CNOT/CP circuit on 34 qubits (complex64) and "
                         "33 qubits (complex128): 128 GiB states")
    ap.add_argument("--full-oracle", action="store_true",
                    help="also compare the whole 30-qubit states (fused and unfused, both dtypes) with the "
                         "oracle's, streamed through host memory (the oracle takes minutes on the host)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain device copies of known size (for HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy(torch):
    """Plain device-to-device copies of a known size: a reference for the
    HBM byte counters of a profiler (2 GiB read + 2 GiB written per copy)."""
    a = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b
    return {"copy_bytes_read": 1 << 31, "copy_bytes_written": 1 << 31, "launches": 3,
            "kernel": "torch elementwise mul(a, 1.0) on 2^29 float32",
            "streaming_ceilings": streaming_ceilings(torch)}


def streaming_ceilings(torch, reps=5):
    """HBM rates of plain streaming kernels (torch's own) on 8 GiB of random
    float32, median of `reps` launches timed with HIP events after one
    untimed launch: in place read + write (the shape of a gate sweep), out of
    place copy, read only (a sum) and write only (a fill).  A reference for
    the sweeps' rates on the same device, not a peak."""
    import numpy as np
    n = 1 << 31
    a = torch.rand(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {}
    cases = (("in_place_read_write", lambda: a.mul_(1.0), 2 * 4 * n),
             ("copy", lambda: b.copy_(a), 2 * 4 * n),
             ("read_only_sum", lambda: a.sum(), 4 * n),
             ("write_only_fill", lambda: b.fill_(0.5), 4 * n))
    for name, fn, nbytes in cases:
        fn()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        out[name] = {"avg_ms": round(med, 3), "GBps": round(nbytes / (med * 1e-3) / 1e9, 1),
                     "frac_of_8TBps": round(nbytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del a, b
    torch.cuda.empty_cache()
    return out


def run_leg(P, W, torch, H, gates, n, dt, kmax, shots, steps, warmup):
    """Runs warmup + timed steps on one dtype; returns measurements."""
    import numpy as np
    st = P.State(H, n, dt)
    abytes = 8 if dt == "c64" else 16
    zterms = W.z_terms(n)
    u = W.uniforms(shots, 1)
    stream = H.stream
    # the uniforms and outcomes stay in device memory for the timed sampler
    with torch.cuda.stream(stream):
        du = torch.from_numpy(u).to("cuda")
        dsmp = torch.empty(shots, dtype=torch.int64, device="cuda")
    stream.synchronize()
    sample_dev_ms_total = 0.0
    per_block = None
    block_k = None
    apply_ms_total = 0.0
    fuse_ms_total = 0.0
    expect_ms_total = 0.0
    sample_ms_total = 0.0

    def step(timed):
        nonlocal per_block, block_k, apply_ms_total, fuse_ms_total, expect_ms_total, sample_ms_total
        nonlocal sample_dev_ms_total
        t0 = time.perf_counter()
        f = P.fuse(gates, kmax)
        t1 = time.perf_counter()
        P.sv_set_basis_state(st.s, 0)
        nb = f.count
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
        for i in range(nb):
            evs[i].record(stream)
            P.sv_apply_fused_range(st.s, f.f, i, 1)
        evs[nb].record(stream)
        evs[nb].synchronize()
        t2 = time.perf_counter()
        z = P.sv_expect_pauli(st.s, zterms)
        es0, es1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t3 = time.perf_counter()
        es0.record(stream)
        P.sv_sample_device(st.s, du.data_ptr(), shots, dsmp.data_ptr())
        es1.record(stream)
        t4 = time.perf_counter()
        es1.synchronize()
        smp = dsmp
        times = [evs[i].elapsed_time(evs[i + 1]) for i in range(nb)]
        ks = [len(t) for t, _ in f.blocks()] if block_k is None else block_k
        f.free()
        if timed:
            if per_block is None:
                per_block = [0.0] * nb
            for i in range(nb):
                per_block[i] += times[i]
            apply_ms_total += sum(times)
            fuse_ms_total += (t1 - t0) * 1e3
            expect_ms_total += (t3 - t2) * 1e3
            sample_ms_total += (t4 - t3) * 1e3
            sample_dev_ms_total += es0.elapsed_time(es1)
        block_k = ks
        return z, smp

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        z, smp = step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nrm = st.norm()
    # the same sampler with the uniforms and outcomes in host memory (over
    # the host link): outside the timed steps, once warm
    P.sv_sample(st.s, u)
    t5 = time.perf_counter()
    host_smp = P.sv_sample(st.s, u)
    sample_host_io_ms = (time.perf_counter() - t5) * 1e3
    host_equals_device = bool(np.array_equal(host_smp, smp.cpu().numpy().view(np.uint64)))
    dim = 1 << n
    sweep_bytes = 2 * dim * abytes
    nb = len(block_k)
    fused_bytes = nb * sweep_bytes * steps
    kmax_idx = [i for i in range(nb) if block_k[i] == max(block_k)]
    avg_kmax_ms = sum(per_block[i] for i in kmax_idx) / (len(kmax_idx) * steps)
    by_k = {}
    for k in sorted(set(block_k)):
        idx = [i for i in range(nb) if block_k[i] == k]
        by_k[str(k)] = {"blocks": len(idx), "avg_ms": round(sum(per_block[i] for i in idx) / (len(idx) * steps), 4)}
    out = {
        "dtype": dt,
        "fused_blocks": nb,
        "block_sizes": by_k,
        "fused_gate_GBps": fused_bytes / (apply_ms_total * 1e-3) / 1e9,
        "apply_ms_per_step": apply_ms_total / steps,
        "ms_per_step": wall * 1e3 / steps,
        "fuse_host_ms_per_step": fuse_ms_total / steps,
        "expect_ms_per_step": expect_ms_total / steps,
        "sample_ms_per_step": sample_ms_total / steps,
        "sample_device_ms_per_step": sample_dev_ms_total / steps,
        "sample_host_io_ms": sample_host_io_ms,
        "sample_host_io_equals_device": host_equals_device,
        "dominant_kernel": {"k": max(block_k), "launches_per_step": len(kmax_idx), "avg_ms": avg_kmax_ms,
                            "bytes_per_launch": sweep_bytes,
                            "GBps": sweep_bytes / (avg_kmax_ms * 1e-3) / 1e9},
        "norm_after": nrm,
        "z_first": [round(float(v), 6) for v in z[:3]],
    }
    state = st
    return out, state


def seeds_leg(P, W, torch, H, n, depth, kmax, seeds):
    """The headline circuit at seeds 0..seeds-1 (the brickwork construction
    with other angles: the same qubit windows, so the handle's tile choices
    from the timed legs carry over), fused at kmax, one pass each from
    |0..0>, timed with HIP events on the handle's stream, complex64 and
    complex128: GB/s of the fused sweeps per seed."""
    import numpy as np
    out = {}
    for dt, s in (("c64", 8), ("c128", 16)):
        st = P.State(H, n, dt)
        sweep = 2 * (1 << n) * s
        vals = []
        for seed in range(seeds):
            f = P.fuse(W.brickwork(n, depth, seed), kmax)
            P.sv_set_basis_state(st.s, 0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            P.sv_apply_fused(st.s, f.f)
            e1.record(H.stream)
            e1.synchronize()
            vals.append(f.count * sweep / (e0.elapsed_time(e1) * 1e-3) / 1e9)
            f.free()
        st.close()
        out[dt] = {"seeds": seeds, "mean_GBps": round(float(np.mean(vals)), 1),
                   "min_GBps": round(float(np.min(vals)), 1), "max_GBps": round(float(np.max(vals)), 1),
                   "mean_frac_of_8TBps": round(float(np.mean(vals)) / HBM_PEAK_GBS, 4)}
        torch.cuda.synchronize()
    return out


def kmax_leg(P, W, torch, H, gates, n):
    """The same circuit unfused (one sweep per gate, controlled gates touching
    only their 2^(n-c) amplitudes) and fused at kmax = 4, 5, 6, complex64 and
    complex128: one warm pass, then one pass timed with HIP events on the
    handle's stream around all its sweeps."""
    out = {}
    for dt, s in (("c64", 8), ("c128", 16)):
        st = P.State(H, n, dt)
        res = {}
        for kmax in (0, 4, 5, 6):
            if kmax == 0:
                entries = P.gate_entries(gates)
                nbytes = sum(2 * (1 << (n - len(e[2]))) * s for e in entries)
                sweeps = len(entries)

                def go():
                    for t, m, c, cv, adj in entries:
                        st.apply_matrix(m, t, c, cv, adjoint=adj)
            else:
                f = P.fuse(gates, kmax)
                sweeps = f.count
                nbytes = sweeps * 2 * (1 << n) * s

                def go():
                    P.sv_apply_fused(st.s, f.f)
            go()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            go()
            e1.record(H.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            if kmax:
                f.free()
            res["unfused" if kmax == 0 else f"kmax{kmax}"] = {
                "sweeps": sweeps, "apply_ms": round(ms, 2), "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}
        base = res["unfused"]["apply_ms"]
        for k in ("kmax4", "kmax5", "kmax6"):
            res[k]["speedup_vs_unfused"] = round(base / res[k]["apply_ms"], 2)
        out[dt] = res
        st.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def graph_leg(P, W, torch, H, n=14, depth=20, reps=200):
    """A small fused program (the brickwork circuit at n qubits, complex64,
    k <= 5 blocks) run repeatedly: eager (one launch per block) against a
    recorded HIP graph replay.  Host wall time per run, averaged over reps,
    after 20 untimed runs (which also settle the k = 5 tile variants)."""
    gates = W.brickwork(n, depth, 0)
    st = P.State(H, n, "c64")
    f = P.fuse(gates, 5)

    def timed(run):
        for _ in range(20):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e6

    eager_us = timed(lambda: P.sv_apply_fused(st.s, f.f))
    g = P.Graph(st, gates, 5)
    graph_us = timed(g.launch)
    out = {"workload": f"{n}-qubit brickwork depth {depth}, complex64, {f.count} fused blocks, run {reps} times",
           "eager_us_per_run": round(eager_us, 1), "graph_us_per_run": round(graph_us, 1),
           "speedup": round(eager_us / graph_us, 2)}
    g.close()
    f.free()
    st.close()
    return out


def host_facts():
    """nproc, CPU model and RAM of the host the oracle runs on."""
    model, ram = "", 0.0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024 / 1e9
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "ram_GB": round(ram, 1)}


def oracle_blocks_rate(P, gates, n, kmax, seconds):
    """The oracle applying the fused blocks of `gates` to a 2^n complex128
    state in host memory until about `seconds` of work: (GB/s counting
    2 * 2^n * 16 B per block, blocks done, blocks, seconds)."""
    import oracle
    f = P.fuse(gates, kmax)
    blocks = f.blocks()
    f.free()
    psi = oracle.basis_state(n, 0)
    done = 0
    t0 = time.perf_counter()
    for targets, m in blocks:
        oracle.apply(psi, m, targets)
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    del psi
    return done * 2 * (1 << n) * 16 / el / 1e9, done, len(blocks), el


def cpu_baseline(W, P, gates, n, depth, kmax, seconds, per_circuit):
    """The oracle (as it stands) applying the same fused blocks to a 2^n
    complex128 state on the host, on all of its threads until about
    `seconds` of work is done; then on one thread, on the same circuit at
    n - 4 qubits (a 30-qubit block takes minutes on one core).  Also the
    oracle's whole-circuit times measured by the error legs."""
    import oracle
    threads = oracle.threads()
    gbs, done, nb, el = oracle_blocks_rate(P, gates, n, kmax, seconds)
    n1 = n - 4
    oracle.set_threads(1)
    try:
        gbs1, done1, nb1, el1 = oracle_blocks_rate(P, W.brickwork(n1, depth, 0), n1, kmax, seconds / 2)
    finally:
        oracle.set_threads(threads)
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} of {nb} fused blocks (k<={kmax}) of the {n}-qubit brickwork "
                      f"depth-{depth} circuit applied by the complex128 oracle to a 2^{n} state in host memory; "
                      f"{el:.1f} s; bytes counted as 2*2^{n}*16 per block",
            "one_core": {"value": round(gbs1, 3), "unit": "GB/s", "cores": 1,
                         "sample": f"first {done1} of {nb1} fused blocks of the {n1}-qubit brickwork depth-{depth} "
                                   f"circuit on one thread; {el1:.1f} s"},
            "host": host_facts(),
            "per_circuit_s": per_circuit}


def config1_errors(P, W, H):
    """The 12-qubit brickwork circuit (depth 20, seed 0) unfused and fused to
    <= 5-qubit blocks, complex128 and complex64, against the oracle: the
    largest amplitude difference, the state fidelity and the largest <Z_i>
    difference; and the oracle's time for the whole circuit."""
    import numpy as np
    import oracle
    n, depth = 12, 20
    gates = W.brickwork(n, depth, 0)
    t0 = time.perf_counter()
    ref = oracle.run(n, gates)
    zref = np.array([oracle.expect_pauli(ref, t) for t in W.z_terms(n)])
    t_oracle = time.perf_counter() - t0
    out = {"workload": f"{n}-qubit brickwork, depth {depth}, seed 0", "oracle_s": round(t_oracle, 4)}
    for dt in ("c128", "c64"):
        for kmax in (0, 5):
            st = P.State(H, n, dt)
            st.run(gates, max_fused_qubits=kmax or None)
            got = st.to_numpy().astype(np.complex128)
            z = P.sv_expect_pauli(st.s, W.z_terms(n))
            st.close()
            out[f"{dt}_{'fused5' if kmax else 'unfused'}"] = {
                "max_abs_damp": float(np.max(np.abs(got - ref))),
                "fidelity": oracle.fidelity(ref, got),
                "max_abs_dz": float(np.max(np.abs(z - zref)))}
    return out


def full_oracle_errors(P, W, H, gates, n, states):
    """The oracle's whole state for `gates` (its gates applied one by one on
    the host, progress printed) against each GPU state in `states` (label ->
    libsv state), streamed in chunks: max |d amp| and the fidelity."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    ref = oracle.basis_state(n, 0)
    for g, gate in enumerate(gates):
        oracle.apply_gate(ref, gate)
        if g % 50 == 0:
            print(f"[bench] oracle gate {g}/{len(gates)} {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    t_or = time.perf_counter() - t0
    out = {"workload": f"{n}-qubit brickwork depth 20 seed 0, whole states", "oracle_s": round(t_or, 1),
           "oracle_threads": oracle.threads()}
    chunk = 1 << 24
    for label, (st, dt) in states.items():
        buf = np.empty(chunk, dtype=np.complex64 if dt == "c64" else np.complex128)
        ov, ng, nr, dmax = 0.0 + 0.0j, 0.0, 0.0, 0.0
        for first in range(0, 1 << n, chunk):
            P.sv_copy_to_host(st.s, buf, first, chunk)
            a = buf.astype(np.complex128)
            r = ref[first: first + chunk]
            ov += np.vdot(r, a)
            ng += np.vdot(a, a).real
            nr += np.vdot(r, r).real
            dmax = max(dmax, float(np.max(np.abs(a - r))))
        out[label] = {"max_abs_damp": dmax, "fidelity": float(abs(ov) ** 2 / (ng * nr))}
        print(f"[bench] full-state comparison {label}: {out[label]}", file=sys.stderr, flush=True)
    del ref
    return out


def config2_errors(P, W, torch, st, n, depth):
    """The timed leg's final state against the oracle's values for the same
    30-qubit circuit (tests/golden/config2_30q_d20_seed0.npz, written by the
    oracle alone): the amplitudes at 65540 seeded indices (largest
    difference; ||d psi||^2 estimated from them, whose complement bounds the
    fidelity from below) and all <Z_i>."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "config2_30q_d20_seed0.npz")
    if n != 30 or depth != 20 or not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in ("idx", "amp", "z", "norm")}
    idx = torch.from_numpy(g["idx"].astype(np.int64)).to(st.tensor.device)
    got = st.tensor[idx].cpu().numpy().astype(np.complex128)
    d = got - g["amp"]
    dpsi2 = float(np.sum(np.abs(d) ** 2)) * float(1 << n) / idx.numel()
    e = P.sv_expect_pauli(st.s, W.z_terms(n))
    return {"sampled_amplitudes": int(idx.numel()), "max_abs_damp": float(np.max(np.abs(d))),
            "est_dpsi2": dpsi2, "est_fidelity_lower_bound": 1.0 - dpsi2,
            "max_abs_dz": float(np.max(np.abs(e - g["z"]))),
            "norm_diff": float(P.sv_norm(st.s) - float(g["norm"]))}


def copy_ceiling(torch, n):
    """In-place read+write bandwidth of torch's elementwise kernel on a
    2^n complex64-sized buffer of uniform random floats (HBM transfer time
    depends on the data: a mostly-zero buffer streams faster than a dense
    state does): the achievable ceiling for in-place sweeps."""
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    a = torch.rand(1 << (n + 1), dtype=torch.float32, device="cuda", generator=g)
    a.mul_(1.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        a.mul_(1.0)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a
    torch.cuda.empty_cache()
    return 2 * (1 << n) * 8 / (ms * 1e-3) / 1e9


def gate_sweep(P, W, torch, H, qubits, sets, reps=3, warm=3, warm_k5=10):
    """Single dense k-qubit gates (Haar random) on `sets` random target sets
    per k, after the paper's gate-application measurement (Sec. II-B, Fig. 2:
    bandwidth from many random target sets).  Each set is applied `warm`
    times untimed (the handle settles its k = 5 tile variant), then `reps`
    times timed with HIP events on the handle's stream.  Median, p10 and p90
    GB/s per k and dtype, and medians per target class: all targets below
    n/2 ("low"), all at or above ("high"), or both ("mixed").  The state is
    dense (a brickwork layer first: every amplitude non-zero), since sweep
    time depends on the data.  For k = 5 the handle first passes its
    untimed warm-up sweeps, and each set gets warm_k5 untimed applications
    (three timings of each of the three tile variants, then the choice).
    qubits: the state's qubit count per dtype."""
    import numpy as np
    out = {}
    for dt, ab in (("c64", 8), ("c128", 16)):
        n = qubits[dt]
        st = P.State(H, n, dt)
        st.run(W.brickwork(n, 1, 11))
        rng = np.random.default_rng(1000)
        res = {}
        for k in range(1, 7):
            bws, cls = [], []
            if k == 5:
                m0 = W.haar_unitary(5, np.random.default_rng(1))
                for _ in range(P.TILE_WARM_SWEEPS):
                    st.apply_matrix(m0, (0, 1, 2, 3, 4))
            for j in range(sets):
                ts = W.random_targets(n, k, np.random.default_rng(1000 * k + j))
                m = W.haar_unitary(k, rng)
                for _ in range(warm_k5 if k == 5 else warm):
                    st.apply_matrix(m, ts)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(H.stream)
                for _ in range(reps):
                    st.apply_matrix(m, ts)
                e1.record(H.stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1) / reps
                bws.append(2 * (1 << n) * ab / (ms * 1e-3) / 1e9)
                cls.append("low" if max(ts) < n // 2 else "high" if min(ts) >= n // 2 else "mixed")
            r = {"median_GBps": round(float(np.median(bws)), 1),
                 "p10_GBps": round(float(np.percentile(bws, 10)), 1),
                 "p90_GBps": round(float(np.percentile(bws, 90)), 1)}
            for c in ("low", "mixed", "high"):
                v = [x for x, y in zip(bws, cls) if y == c]
                if v:
                    r[c] = {"sets": len(v), "median_GBps": round(float(np.median(v)), 1)}
            res[str(k)] = r
            print(f"[bench] gate sweep {dt} {n}q k={k}: median {r['median_GBps']} GB/s", file=sys.stderr, flush=True)
        res["n_qubits"] = n
        out[dt] = res
        st.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def diagonal_leg(P, W, torch, H, n, reps=10):
    """Generalized permutation gates at n qubits on a dense state: diagonal
    gates on 2 and 10 targets (random phases) and a permutation on 3 targets,
    HBM GB/s over `reps` back-to-back sweeps each (HIP events on the handle's
    stream); then the n-qubit QFT fused with dense blocks only (k <= 5)
    against dense plus diagonal blocks (k <= 5, diagonal k <= 10) and against
    coupled fusion (k <= 5, the controlled phases carried as couplings of
    the dense blocks): sweeps and apply time of one timed pass after one
    untimed pass."""
    import numpy as np
    out = {}
    rng = np.random.default_rng(17)
    for dt, ab in (("c64", 8), ("c128", 16)):
        st = P.State(H, n, dt)
        st.run(W.brickwork(n, 1, 13))
        sweep = 2 * (1 << n) * ab
        res = {}
        for label, perm, targets in (("diag_k2", None, (3, 17)), ("diag_k10", None, tuple(range(0, 30, 3))[:10]),
                                     ("perm_k3", [int(p) for p in rng.permutation(8)], (2, 11, 25))):
            diag = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << len(targets)))
            for _ in range(2):
                st.apply_gen_permutation(perm, diag, targets)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            for _ in range(reps):
                st.apply_gen_permutation(perm, diag, targets)
            e1.record(H.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res[label] = {"avg_ms": round(ms, 3), "GBps": round(sweep / (ms * 1e-3) / 1e9, 1)}
        gates = W.qft(n)
        for label, kd, coupled in (("qft_dense_only", 0, False), ("qft_dense_and_diagonal", 10, False),
                                   ("qft_coupled", 0, True)):
            f = P.fuse(gates, 5, kd, coupled)
            ndiag = sum(1 for _, m in f.blocks() if m.ndim == 1)
            P.sv_apply_fused(st.s, f.f)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            P.sv_apply_fused(st.s, f.f)
            e1.record(H.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            res[label] = {"sweeps": f.count, "diagonal_sweeps": ndiag, "apply_ms": round(ms, 2),
                          "GBps": round(f.count * sweep / (ms * 1e-3) / 1e9, 1)}
            f.free()
        res["qft_speedup"] = round(res["qft_dense_only"]["apply_ms"] / res["qft_dense_and_diagonal"]["apply_ms"], 2)
        res["qft_coupled_speedup"] = round(res["qft_dense_only"]["apply_ms"] / res["qft_coupled"]["apply_ms"], 2)
        out[dt] = res
        st.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def table1_leg(P, W, torch, H, n, reps=5):
    """The other single-GPU operations of the paper's Table I at n qubits on
    a dense state, each timed over `reps` calls with HIP events on the
    handle's stream (blocking calls: host wall time): Pauli rotations (an
    X/Y/Z string, a Z-only string), measurement probabilities of 3 qubits,
    Z-product parity probabilities, collapse, batched measurement with
    collapse, and a 3-qubit dense-observable expectation.  GB/s counts the
    algorithmic bytes: reads of 2^n amplitudes for the reductions, read and
    write for the rotation, the write plus the kept reads for a collapse."""
    import numpy as np
    out = {}
    rng = np.random.default_rng(23)
    for dt, ab in (("c64", 8), ("c128", 16)):
        st = P.State(H, n, dt)
        st.run(W.brickwork(n, 1, 29))
        state = (1 << n) * ab
        res = {}

        def timed_async(fn):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            for _ in range(reps):
                fn()
            e1.record(H.stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

        def timed_blocking(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            return (time.perf_counter() - t0) / reps * 1e3

        term = [(1, "X"), (7, "Y"), (19, "Z"), (26, "X")]
        ms = timed_async(lambda: P.sv_apply_pauli_rotation(st.s, 0.3, term))
        res["pauli_rotation_xyz"] = {"avg_ms": round(ms, 3), "GBps": round(2 * state / (ms * 1e-3) / 1e9, 1)}
        ms = timed_async(lambda: P.sv_apply_pauli_rotation(st.s, 0.3, [(q, "Z") for q in range(0, n, 2)]))
        res["pauli_rotation_z"] = {"avg_ms": round(ms, 3), "GBps": round(2 * state / (ms * 1e-3) / 1e9, 1)}
        q3 = [2, 14, 27]
        ms = timed_blocking(lambda: P.sv_measure_probabilities(st.s, q3))
        res["measure_probabilities_3q"] = {"avg_ms": round(ms, 3), "GBps": round(state / (ms * 1e-3) / 1e9, 1)}
        ms = timed_blocking(lambda: P.sv_zbasis_probabilities(st.s, list(range(0, n, 3))))
        res["zbasis_probabilities"] = {"avg_ms": round(ms, 3), "GBps": round(state / (ms * 1e-3) / 1e9, 1)}
        p = P.sv_measure_probabilities(st.s, [29])
        ms = timed_async(lambda: P.sv_collapse(st.s, [29], 0, 1.0))
        res["collapse_1q"] = {"avg_ms": round(ms, 3), "GBps": round(1.5 * state / (ms * 1e-3) / 1e9, 1),
                              "note": "bytes: the whole state written, the kept half read"}
        m = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
        ms = timed_blocking(lambda: P.sv_expect_matrix(st.s, m, [3, 12, 21]))
        res["expect_matrix_3q"] = {"avg_ms": round(ms, 3), "GBps": round(state / (ms * 1e-3) / 1e9, 1)}
        del p
        ms = timed_async(lambda: P.sv_swap_index_bits(st.s, [(1, 25), (4, 17)]))
        res["swap_index_bits_2pairs"] = {"avg_ms": round(ms, 3), "GBps": round(2 * 0.75 * state / (ms * 1e-3) / 1e9, 1),
                                         "note": "bytes: the 3/4 of amplitudes the swap moves, read and written"}
        order = list(range(n))[::-1]
        svd = P.SV_C64 if dt == "c64" else P.SV_C128
        host_buf = np.empty(1 << 26, dtype=np.complex64 if dt == "c64" else np.complex128)
        ms = timed_blocking(lambda: P.sv_accessor_get(st.s, svd, order, begin=0, end=1 << 26, out=host_buf))
        res["accessor_get_reversed_2^26"] = {"avg_ms": round(ms, 3),
                                             "GBps_host": round((1 << 26) * ab / (ms * 1e-3) / 1e9, 1),
                                             "note": "into a reused host array; the 2^26 requested amplitudes are "
                                                     "every 16th of the state, one per 128-B line"}
        out[dt] = res
        st.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def large_leg(P, W, torch, H):
    """The depth-12 random CNOT/CP circuit (U3 on every qubit, then a random
    matching into far-apart CNOT or CP pairs, per layer) fused to k <= 5
    blocks on 34 qubits (complex64) and 33 qubits (complex128), 128 GiB
    each, from a random basis state: one untimed pass, then one pass timed
    with HIP events on the handle's stream around every block."""
    out = {}
    for n, dt, ab in ((34, "c64", 8), (33, "c128", 16)):
        free, _ = torch.cuda.mem_get_info()
        need = (1 << n) * ab + (2 << 30)
        if free < need:
            out[dt] = {"skipped": f"needs {need >> 30} GiB of free device memory, {free >> 30} GiB free"}
            continue
        gates = W.random_cx_cp(n, 12, 0)
        f = P.fuse(gates, 5)
        ks = [len(t) for t, _ in f.blocks()]
        st = P.State(H, n, dt)
        P.sv_set_basis_state(st.s, W.random_basis_state(n, 0))
        P.sv_apply_fused(st.s, f.f)
        torch.cuda.synchronize()
        P.sv_set_basis_state(st.s, W.random_basis_state(n, 0))
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(f.count + 1)]
        for i in range(f.count):
            evs[i].record(H.stream)
            P.sv_apply_fused_range(st.s, f.f, i, 1)
        evs[f.count].record(H.stream)
        evs[f.count].synchronize()
        times = [evs[i].elapsed_time(evs[i + 1]) for i in range(f.count)]
        nrm = st.norm()
        sweep = 2 * (1 << n) * ab
        by_k = {}
        for k in sorted(set(ks)):
            t = [x for x, kk in zip(times, ks) if kk == k]
            by_k[str(k)] = {"blocks": len(t), "avg_ms": round(sum(t) / len(t), 3),
                            "GBps": round(sweep / (sum(t) / len(t) * 1e-3) / 1e9, 1)}
        out[dt] = {"n_qubits": n, "gates": len(gates), "fused_blocks": f.count, "apply_ms": round(sum(times), 1),
                   "fused_gate_GBps": round(f.count * sweep / (sum(times) * 1e-3) / 1e9, 1),
                   "block_sizes": by_k, "norm_after": nrm}
        f.free()
        # the same circuit and the QFT of a basis state with coupled fusion
        # (controlled phases carried as couplings of the dense blocks)
        for label, g in (("cxcp_coupled", gates), ("qft_coupled", W.qft(n))):
            fc = P.fuse(g, 5, coupled=True)
            P.sv_set_basis_state(st.s, W.random_basis_state(n, 0))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            P.sv_apply_fused(st.s, fc.f)
            e1.record(H.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            out[dt][label] = {"gates": len(g), "fused_blocks": fc.count, "apply_ms": round(ms, 1),
                              "GBps": round(fc.count * sweep / (ms * 1e-3) / 1e9, 1)}
            fc.free()
        # 2^20 samples of the QFT's output state from seeded uniforms, in
        # device memory (one untimed call, then one timed)
        with torch.cuda.stream(H.stream):
            du = torch.from_numpy(W.uniforms(1 << 20, 7)).to("cuda")
            dsmp = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
        H.stream.synchronize()
        P.sv_sample_device(st.s, du.data_ptr(), 1 << 20, dsmp.data_ptr())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(H.stream)
        P.sv_sample_device(st.s, du.data_ptr(), 1 << 20, dsmp.data_ptr())
        e1.record(H.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        out[dt]["sample_2^20"] = {"ms": round(ms, 2),
                                  "state_read_GBps": round((1 << n) * ab / (ms * 1e-3) / 1e9, 1),
                                  "note": "uniforms and outcomes in device memory; the state after the QFT"}
        del du, dsmp
        st.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def batched_leg(P, W, torch, H, count, steps, warmup, sample, check_per_n=4):
    """4096 independent complex64 brickwork circuits (qubits uniform in
    8..20, depth uniform in 10..40), each returning <Z_i Z_i+1> for all i, in
    one recorded run: the autotuner chooses, per qubit count, the persistent
    kernel (and its fusion width) or the level path (and its tile shape);
    per-circuit latency from the device wall clock.  Baseline: a sample of the same
    circuits run one at a time through the plain complex128 path (one
    sv_apply_matrix per gate, then sv_expect_pauli), timed on the host.
    Errors: the first `check_per_n` circuits of every qubit count against
    the oracle (state fidelity, <Z_i Z_i+1>)."""
    import numpy as np
    import oracle
    items = W.batched(count, seed=0)
    ns = [it.n for it in items]
    circuits = [it.gates for it in items]
    terms = [[(1 << q) | (1 << (q + 1)) for q in range(it.n - 1)] for it in items]
    t0 = time.perf_counter()
    b = P.Batch(H, ns, circuits, terms, max_fused_qubits=0)
    prep = time.perf_counter() - t0
    for _ in range(warmup):
        b.run()
    lats, kts = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        exps, lat, ks = b.run()
        lats.append(lat)
        kts.append(ks)
    wall = (time.perf_counter() - t0) / steps
    lat = np.concatenate(lats)
    widths = {str(n): b.fusion_width(n) for n in sorted(set(ns))}
    plans = {str(n): {k: v for k, v in b.plan(n).items() if k != "tuned"} for n in sorted(set(ns))}
    tune_s, build_s = b.host_times()
    blocks = b.blocks()
    state_gb = sum((1 << n) * 8 for n in ns) / 1e9
    # every fused block reads and writes its state once
    sweep_bytes = sum(int(nb) * 2 * (1 << n) * 8 for nb, n in zip(blocks, ns))
    # errors against the oracle on a sample spread over every qubit count
    check = []
    for n in sorted(set(ns)):
        check += [i for i in range(count) if ns[i] == n][:check_per_n]
    fids, dzz, t_or = [], [], {}
    for i in check:
        n = ns[i]
        t1 = time.perf_counter()
        ref = oracle.run(n, circuits[i])
        zr = np.array([oracle.expect_pauli(ref, [(q, "Z"), (q + 1, "Z")]) for q in range(n - 1)])
        t_or.setdefault(n, []).append(time.perf_counter() - t1)
        fids.append(oracle.fidelity(ref, b.state(i).astype(np.complex128)))
        dzz.append(float(np.max(np.abs(exps[i] - zr))))
    b.close()
    # baseline: plain complex128 per-circuit path on a sample
    rng = np.random.default_rng(1)
    pick = sorted(rng.choice(count, size=min(sample, count), replace=False).tolist())
    base_lat = []
    for i in pick:
        it = items[i]
        st = P.State(H, it.n, "c128")
        zz = [[(q, "Z"), (q + 1, "Z")] for q in range(it.n - 1)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st.run(it.gates)
        st.expect(zz)
        base_lat.append(time.perf_counter() - t1)
        st.close()
    base_lat = np.array(base_lat)
    return {
        "workload": f"{count} complex64 brickwork circuits, qubits uniform 8-20, depth uniform 10-40, "
                    f"<Z_i Z_i+1> for all i, one recorded run (path, fusion width and tile shape per qubit count "
                    f"from the autotuner)",
        "circuits": count,
        "states_GB": round(state_gb, 3),
        "kernel_ms": round(1e3 * float(np.median(kts)), 3),
        "wall_ms_per_batch": round(1e3 * wall, 3),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "latency_clock": "device wall clock, from the run's start to each circuit's state and expectations written",
        "circuits_per_s": round(count / float(np.median(kts)), 1),
        "sweep_GB": round(sweep_bytes / 1e9, 2),
        "effective_GBps": round(sweep_bytes / float(np.median(kts)) / 1e9, 1),
        "fusion_widths": widths,
        "plans": plans,
        "fused_blocks_total": int(blocks.sum()),
        "host_prep_s": round(prep, 3),
        "host_prep_split_s": {"autotuner": round(tune_s, 3), "fuse_pack_upload": round(build_s, 3),
                              "note": "autotuner 0 when every plan came from the process or SV_AUTOTUNE_CACHE"},
        "vs_oracle": {"circuits": len(check), "qubits": f"{min(ns)}-{max(ns)}", "min_fidelity": min(fids),
                      "max_abs_dzz": max(dzz)},
        "oracle_s_per_circuit": {str(n): round(float(np.mean(v)), 4) for n, v in sorted(t_or.items())},
        "baseline_c128_per_circuit": {
            "sample": len(pick),
            "p50_ms": round(1e3 * float(np.percentile(base_lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(base_lat, 99)), 3),
            "circuits_per_s": round(len(pick) / float(base_lat.sum()), 1),
            "latency_clock": "host wall clock of each circuit alone (no queueing)",
            "path": "one circuit at a time, unfused sv_apply_matrix per gate, then sv_expect_pauli",
        },
    }


def _serve_stats(res, reqs, span):
    import numpy as np
    lat = np.array([res[r.rid].latency for r in reqs])
    svc = np.array([res[r.rid].done - res[r.rid].admitted for r in reqs])
    return {"requests": len(reqs),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
            "service_p50_ms": round(1e3 * float(np.percentile(svc, 50)), 2),
            "circuits_per_s": round(len(reqs) / span, 2)}


def serving_capacity(Server, replay, W, slots, small_slots, dtype="c64", kmax=5, count=32, seed=11):
    """Requests per second a server sustains when a calibration set of the
    stream's requests is submitted at once."""
    srv = Server(slots=slots, small_slots=small_slots, budget_bytes=96 << 30, dtype=dtype, kmax=kmax)
    cal = W.serving_requests(count, rate_per_s=1e9, seed=seed)
    replay(srv, cal[: max(4, slots)], time_scale=0.0)  # warm the slots
    t0 = time.monotonic()
    replay(srv, cal, time_scale=0.0)
    cap = len(cal) / (time.monotonic() - t0)
    srv.close()
    return cap


def serving_leg(P, W, torch, n_requests, slots, small_slots, check=16):
    """Poisson stream of circuit requests (qubits log-uniform 10..28, depth
    10..100, random U3 + CZ/CNOT pairs; 16 random Pauli strings and 1024
    samples each) through the continuous-batching server (complex64 states,
    FP64 reductions; `slots` general slots plus `small_slots` for requests
    of up to 16 qubits).  The offered load is 0.75 of the capacity measured
    by submitting a calibration set at once.  Latency: host monotonic time
    from a request's arrival to its results.  Baseline: a complex128 FIFO
    that serves one request at a time, offered 0.75 of its own capacity.
    Errors: the first `check` requests of up to 20 qubits against the oracle
    (expectations; samples by the epsilon-interval rule with the served
    state's probabilities, rebuilt by the same fused program)."""
    import numpy as np
    import oracle
    from paper_2308_01999_amd.serve import Server, fusion_pieces, replay
    capacity = serving_capacity(Server, replay, W, slots, small_slots)
    rate = 0.75 * capacity
    reqs = W.serving_requests(n_requests, rate_per_s=rate, seed=0)
    srv = Server(slots=slots, small_slots=small_slots, budget_bytes=96 << 30, dtype="c64", kmax=5)
    t0 = time.monotonic()
    res = replay(srv, reqs)
    span = time.monotonic() - t0
    srv.close()
    main = _serve_stats(res, reqs, span)
    # baseline: complex128, one request at a time, unfused, below its capacity
    base_n = min(16, n_requests)
    bcap = serving_capacity(Server, replay, W, 1, 0, dtype="c128", kmax=0, count=8)
    breqs = W.serving_requests(base_n, rate_per_s=0.75 * bcap, seed=0)
    bsrv = Server(slots=1, budget_bytes=96 << 30, dtype="c128", kmax=0)
    t0 = time.monotonic()
    bres = replay(bsrv, breqs)
    bspan = time.monotonic() - t0
    bsrv.close()
    # errors against the oracle
    h = P.Handle()
    dexp, eps_ok, t_or, checked = [], [], [], 0
    for r in reqs:
        if checked >= check:
            break
        if r.n > 20:
            continue
        checked += 1
        t1 = time.perf_counter()
        ref = oracle.run(r.n, r.gates)
        er = np.array([oracle.expect_pauli(ref, t) for t in r.terms])
        t_or.append(time.perf_counter() - t1)
        dexp.append(float(np.max(np.abs(res[r.rid].expectations - er))))
        # the served state rebuilt from the same fused pieces the server ran
        st = P.State(h, r.n, "c64")
        for part in fusion_pieces(r.n, r.gates):
            f = P.fuse(part, 5)
            P.sv_apply_fused(st.s, f.f)
            f.free()
        p_g = np.abs(st.to_numpy().astype(np.complex128)) ** 2
        same = np.array_equal(st.sample(np.asarray(r.uniforms)), res[r.rid].samples)
        st.close()
        u = np.asarray(r.uniforms)
        _, cdf = oracle.sample(ref, u[:1], return_cdf=True)
        eps = float(np.sum(np.abs(p_g - np.abs(ref) ** 2))) + 1e-12
        got = res[r.rid].samples.astype(np.int64)
        lo = np.where(got > 0, cdf[np.maximum(got - 1, 0)], 0.0)
        x = u * cdf[-1]
        eps_ok.append(bool(same and ((lo - eps <= x) & (x < cdf[got] + eps)).all()))
    h.close()
    return {
        "workload": "Poisson requests: qubits log-uniform 10-28, depth 10-100, U3 + CZ/CNOT on random pairs, "
                    "16 Pauli strings + 1024 samples each; complex64, fused k<=5, FP64 reductions",
        "slots": slots,
        "small_slots": small_slots,
        "capacity_req_per_s": round(capacity, 2),
        "offered_req_per_s": round(rate, 2),
        **main,
        "latency_clock": "host monotonic, arrival to results; service = admission to results",
        "qubits_mean": round(float(np.mean([r.n for r in reqs])), 2),
        "vs_oracle": {"requests": checked, "max_qubits": 20, "max_abs_dexpect": max(dexp),
                      "eps_rule_pass_rate": sum(eps_ok) / max(1, len(eps_ok))},
        "oracle_s_per_request_mean": round(float(np.mean(t_or)), 4),
        "baseline_c128_fifo": {
            "capacity_req_per_s": round(bcap, 2),
            "offered_req_per_s": round(0.75 * bcap, 2),
            **_serve_stats(bres, breqs, bspan),
            "path": "one request at a time, complex128 states, one sv_apply_matrix sweep per gate",
        },
    }


def serving_sweep(P, W, torch, n_requests, slots, small_slots):
    """Serving at offered loads of 0.25, 0.5, 0.75 and 0.9 of the measured
    capacity, and the capacity with one slot against `slots` (the same
    complex64, kmax 5 stream): more slots only raise capacity if the slots'
    work overlaps on the device."""
    from paper_2308_01999_amd.serve import Server, replay
    capacity = serving_capacity(Server, replay, W, slots, small_slots)
    points = []
    for frac in (0.25, 0.5, 0.75, 0.9):
        reqs = W.serving_requests(n_requests, rate_per_s=frac * capacity, seed=0)
        srv = Server(slots=slots, small_slots=small_slots, budget_bytes=96 << 30, dtype="c64", kmax=5)
        t0 = time.monotonic()
        res = replay(srv, reqs)
        span = time.monotonic() - t0
        srv.close()
        points.append({"load": frac, "offered_req_per_s": round(frac * capacity, 2), **_serve_stats(res, reqs, span)})
        print(f"[bench] serving sweep load {frac}: {points[-1]}", file=sys.stderr, flush=True)
    caps = {}
    for sl, sm in ((1, 0), (slots, 0), (slots, small_slots)):
        caps[f"{sl}+{sm}"] = round(serving_capacity(Server, replay, W, sl, sm, count=48), 2)
    return {"capacity_req_per_s": round(capacity, 2), "points": points,
            "capacity_by_slots": caps,
            "capacity_note": "general+small slots; calibration set of 48 requests submitted at once"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library keeps a whole "
              f"state on one device and has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2308_01999_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    n, depth, kmax = args.n, args.depth, args.kmax
    gates = W.brickwork(n, depth, 0)
    H = P.Handle()
    print(f"[bench] c64 leg: n={n} depth={depth} kmax={kmax}", file=sys.stderr, flush=True)
    r64, st64 = run_leg(P, W, torch, H, gates, n, "c64", kmax, args.shots, args.steps, args.warmup)
    # errors of the results against the oracle (outside every timed region)
    errors = {"config2_c64": config2_errors(P, W, torch, st64, n, depth)}
    extra = {}
    if not args.no_c128:
        print("[bench] c128 leg", file=sys.stderr, flush=True)
        r128, st128 = run_leg(P, W, torch, H, gates, n, "c128", kmax, args.shots, args.steps, args.warmup)
        errors["config2_c128"] = config2_errors(P, W, torch, st128, n, depth)
        # fidelity of the complex64 result against the complex128 GPU result,
        # streamed in chunks through host memory
        import numpy as np
        ov = 0.0 + 0.0j
        n64 = n128 = 0.0
        chunk = 1 << 24
        a = np.empty(chunk, dtype=np.complex64)
        b = np.empty(chunk, dtype=np.complex128)
        for first in range(0, 1 << n, chunk):
            P.sv_copy_to_host(st64.s, a, first, chunk)
            P.sv_copy_to_host(st128.s, b, first, chunk)
            a128 = a.astype(np.complex128)
            ov += np.vdot(b, a128)
            n64 += np.vdot(a128, a128).real
            n128 += np.vdot(b, b).real
        r128["fidelity_c64_vs_c128"] = float(abs(ov) ** 2 / (n64 * n128))
        extra["c128"] = r128
    # the fused states stay for the full-state comparison, if asked for
    st64_keep = st64 if args.full_oracle else None
    st128_keep = st128 if (args.full_oracle and not args.no_c128) else None
    if st64_keep is None:
        st64.close()
    if not args.no_c128 and st128_keep is None:
        st128.close()
    torch.cuda.synchronize()
    dk = r64["dominant_kernel"]
    achieved = dk["GBps"]
    kname = dominant_kernel_name("c64", dk["k"], n)
    traffic = pmc_traffic(kname, n)
    line = {
        "metric": "fused-gate HBM GB/s at 30q c64/c128; batched-circuit p50/p99 latency",
        "value": round(r64["fused_gate_GBps"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit brickwork random circuit, depth {depth}, seed 0, fused to <= {kmax}-qubit "
                               f"blocks, complex64 state (fp32 arithmetic, fp64 reductions), <Z_i> for all qubits, "
                               f"{args.shots} samples",
                   "n_qubits": n, "depth": depth, "max_fused_qubits": kmax, "state_dtype": "complex64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kname, "bytes_per_launch": dk["bytes_per_launch"],
                     "avg_launch_ms": round(dk["avg_ms"], 4)},
        "c64": r64,
        **extra,
    }
    if "c128" in extra:
        # the same figure for the complex128 leg's dominant kernel
        dk2 = extra["c128"]["dominant_kernel"]
        k2 = dominant_kernel_name("c128", dk2["k"], n)
        line["roofline_c128"] = {"bound": "hbm", "achieved": round(dk2["GBps"], 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(dk2["GBps"] / HBM_PEAK_GBS, 4),
                                 "traffic": pmc_traffic(k2, n), "kernel": k2,
                                 "bytes_per_launch": dk2["bytes_per_launch"], "avg_launch_ms": round(dk2["avg_ms"], 4)}
    if args.full_oracle:
        # the timed legs' states (fused) and unfused runs of the same circuit
        print("[bench] full-state comparison with the oracle", file=sys.stderr, flush=True)
        states = {}
        for dt in ("c64", "c128"):
            su = P.State(H, n, dt)
            su.run(gates)
            states[f"{dt}_unfused"] = (su, dt)
        states["c64_fused5"] = (st64_keep, "c64")
        if st128_keep is not None:
            states["c128_fused5"] = (st128_keep, "c128")
        errors["config2_full"] = full_oracle_errors(P, W, H, gates, n, states)
        for su, _ in states.values():
            su.close()
    print("[bench] 12-qubit configuration against the oracle", file=sys.stderr, flush=True)
    errors["config1"] = config1_errors(P, W, H)
    line["oracle_errors"] = errors
    if not args.no_kmax_sweep:
        print("[bench] unfused / kmax sweep", file=sys.stderr, flush=True)
        # on the main handle, whose k = 5 tile choices for this circuit are settled
        line["fusion_widths"] = kmax_leg(P, W, torch, H, gates, n)
    if args.seeds > 0 and not args.no_c128:
        print(f"[bench] seeds 0-{args.seeds - 1}", file=sys.stderr, flush=True)
        line["seeds"] = seeds_leg(P, W, torch, H, n, depth, kmax, args.seeds)
    H.close()
    print("[bench] graph leg", file=sys.stderr, flush=True)
    H5 = P.Handle()
    line["graph_replay"] = graph_leg(P, W, torch, H5)
    H5.close()
    if not args.no_batched:
        print("[bench] batched leg", file=sys.stderr, flush=True)
        H2 = P.Handle()
        line["batched"] = batched_leg(P, W, torch, H2, args.batch_circuits, max(1, args.steps), 1,
                                      args.baseline_sample)
        H2.close()
    if not args.no_serving:
        print("[bench] serving leg", file=sys.stderr, flush=True)
        line["serving"] = serving_leg(P, W, torch, args.serve_requests, args.serve_slots, args.serve_small_slots)
    if args.serving_sweep:
        print("[bench] serving sweep", file=sys.stderr, flush=True)
        line["serving_sweep"] = serving_sweep(P, W, torch, args.sweep_requests, args.serve_slots,
                                              args.serve_small_slots)
    line["copy_ceiling_GBps"] = round(copy_ceiling(torch, n), 1)
    line["frac_of_copy_ceiling"] = round(r64["fused_gate_GBps"] / line["copy_ceiling_GBps"], 4)
    if not args.no_diagonal:
        print("[bench] diagonal / permutation leg", file=sys.stderr, flush=True)
        HD = P.Handle()
        line["diagonal_gates"] = diagonal_leg(P, W, torch, HD, n)
        HD.close()
    if not args.no_diagonal:
        print("[bench] Table I operations leg", file=sys.stderr, flush=True)
        HT = P.Handle()
        line["table1_ops"] = table1_leg(P, W, torch, HT, n)
        HT.close()
    if args.large:
        print("[bench] large-state leg", file=sys.stderr, flush=True)
        HL = P.Handle()
        line["large"] = large_leg(P, W, torch, HL)
        HL.close()
    if args.gate_sweep:
        print("[bench] gate sweep", file=sys.stderr, flush=True)
        H3 = P.Handle()
        qubits = {"c64": args.sweep_n64 or n, "c128": args.sweep_n128 or n}
        line["gate_sweep"] = gate_sweep(P, W, torch, H3, qubits, args.sweep_sets)
        H3.close()
    if args.calibrate_copy:
        line["copy_calibration"] = calibrate_copy(torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        per_circuit = {"config1_12q_c128": errors["config1"]["oracle_s"]}
        if "batched" in line:
            per_circuit["batched_by_qubits"] = line["batched"]["oracle_s_per_circuit"]
        if "serving" in line:
            per_circuit["serving_mean_up_to_20q"] = line["serving"]["oracle_s_per_request_mean"]
        line["cpu_baseline"] = cpu_baseline(W, P, gates, n, depth, kmax, args.cpu_seconds, per_circuit)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
