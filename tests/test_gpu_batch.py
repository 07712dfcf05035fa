"""GPU parity of the batched path: every circuit of a mixed batch (resident
and streamed states on the persistent kernel, fused at each width and by
the autotuner; 13-20 qubit states on the level path, which sweeps each
block as a five-qubit gate through the single-state tile sweep) against the
oracle, and each circuit's result alone versus in the mix (bitwise equal,
since all reductions run in a fixed order)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

C64_FID = 1.0 - 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_01999_amd as P
    return P


@pytest.fixture(scope="module")
def H(P):
    h = P.Handle()
    yield h
    h.close()


def _mixed(seed, sizes, depth_lo=4, depth_hi=12):
    rng = np.random.default_rng(seed)
    ns, circuits, terms = [], [], []
    for i, n in enumerate(sizes):
        d = int(rng.integers(depth_lo, depth_hi + 1))
        ns.append(n)
        circuits.append(W.brickwork(n, d, 1000 * seed + i))
        zz = [1 << q | 1 << (q + 1) for q in range(n - 1)]
        terms.append(zz + [1 << (n - 1)])
    return ns, circuits, terms


def _check(P, batch, ns, circuits, terms, exps):
    for i, (n, g, zm) in enumerate(zip(ns, circuits, terms)):
        ref = oracle.run(n, g)
        got = batch.state(i).astype(np.complex128)
        fid = oracle.fidelity(ref, got)
        assert fid >= C64_FID, (i, n, fid)
        zr = []
        for m in zm:
            term = [(q, "Z") for q in range(n) if (m >> q) & 1]
            zr.append(oracle.expect_pauli(ref, term))
        assert np.max(np.abs(exps[i] - np.array(zr))) <= 1e-4, (i, n)


@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 5])
def test_batch_fixed_width_matches_oracle(P, H, kmax):
    sizes = [2, 3, 5, 8, 11, 12, 13, 14, 16, 4, 9, 12, 13]
    ns, circuits, terms = _mixed(kmax, sizes)
    b = P.Batch(H, ns, circuits, terms, max_fused_qubits=kmax)
    exps, lat, ks = b.run()
    _check(P, b, ns, circuits, terms, exps)
    assert (lat > 0).all() and ks > 0
    assert lat.max() <= ks * 1.5 + 1e-3
    b.close()


def test_batch_autotuned_width_matches_oracle(P, H):
    sizes = [8, 10, 12, 13, 14, 15] * 3
    ns, circuits, terms = _mixed(77, sizes, 10, 20)
    b = P.Batch(H, ns, circuits, terms, max_fused_qubits=0)
    for n in set(sizes):
        assert 3 <= b.fusion_width(n) <= 5
    exps, lat, ks = b.run()
    _check(P, b, ns, circuits, terms, exps)
    b.close()


def test_batch_alone_equals_in_mix(P, H):
    sizes = [8, 14, 10, 16, 12, 9, 13, 15]
    ns, circuits, terms = _mixed(5, sizes)
    mix = P.Batch(H, ns, circuits, terms, max_fused_qubits=5)
    exps, _, _ = mix.run()
    states = [mix.state(i) for i in range(len(ns))]
    for i in (0, 3, 6):
        alone = P.Batch(H, [ns[i]], [circuits[i]], [terms[i]], max_fused_qubits=5)
        e1, _, _ = alone.run()
        np.testing.assert_array_equal(e1[0], exps[i])
        np.testing.assert_array_equal(alone.state(0), states[i])
        alone.close()
    # a second run of the same batch gives the same results
    exps2, _, _ = mix.run()
    for a, c in zip(exps, exps2):
        np.testing.assert_array_equal(a, c)
    mix.close()


@pytest.mark.parametrize("level", [13, 15, 17])
@pytest.mark.parametrize("kmax", [0, 5])
def test_batch_level_path_matches_oracle(P, level, kmax):
    # 17-20 qubit states (the large part of the benchmark batch) with
    # resident and smaller streamed ones; level 13 also moves every streamed
    # state of 13-16 qubits to the level path
    sizes = [20, 8, 17, 13, 19, 12, 18, 14, 16, 20, 15, 17]
    ns, circuits, terms = _mixed(31 + level + kmax, sizes, 4, 14)
    h = P.Handle()
    h.set_batch_level_qubits(level)
    b = P.Batch(h, ns, circuits, terms, max_fused_qubits=kmax)
    for n in set(sizes):
        if n >= level:
            assert b.fusion_width(n) == 5
    exps, lat, ks = b.run()
    _check(P, b, ns, circuits, terms, exps)
    assert (lat > 0).all() and ks > 0
    assert lat.max() <= ks * 1.5 + 1e-3
    # a replay of the recorded run gives the same results bit for bit
    exps2, _, _ = b.run()
    for a, c in zip(exps, exps2):
        np.testing.assert_array_equal(a, c)
    b.close()
    h.close()


def test_batch_level_path_z_sums_many_terms(P):
    # shallow circuits (expectations of order one) on the level path with up
    # to 32 random Z strings each, over every qubit: the last block's sums
    # take each term from one coefficient of a per-thread transform over
    # four tile-local index bits and a sign over the others, so terms on
    # every bit position, on several at once and on none of the transform's
    # bits are all needed; one circuit has no terms at all (the norm only)
    rng = np.random.default_rng(77)
    sizes = [13, 15, 17, 20, 14, 19]
    counts = [32, 32, 17, 32, 0, 9]
    ns, circuits, terms = [], [], []
    for i, (n, t) in enumerate(zip(sizes, counts)):
        ns.append(n)
        circuits.append(W.brickwork(n, 1 + i % 2, 500 + i))
        masks = [1 << q for q in range(min(t, n))]
        while len(masks) < t:
            m = int(rng.integers(1, 1 << n))
            masks.append(m)
        terms.append(masks[:t])
    h = P.Handle()
    h.set_batch_level_qubits(13)
    b = P.Batch(h, ns, circuits, terms, max_fused_qubits=5)
    exps, _, _ = b.run()
    for i, (n, g, zm) in enumerate(zip(ns, circuits, terms)):
        assert len(exps[i]) == len(zm)
        if not zm:
            continue
        ref = oracle.run(n, g)
        zr = np.array([oracle.expect_pauli(ref, [(q, "Z") for q in range(n) if (m >> q) & 1]) for m in zm])
        assert np.max(np.abs(zr)) > 0.1, (i, n)  # the terms are not all near zero
        assert np.max(np.abs(exps[i] - zr)) <= 2e-6, (i, n, np.max(np.abs(exps[i] - zr)))
    b.close()
    h.close()


def test_batch_level_path_alone_equals_in_mix(P):
    sizes = [17, 20, 9, 18, 13, 19, 15, 20, 12]
    ns, circuits, terms = _mixed(6, sizes, 6, 16)
    h = P.Handle()
    mix = P.Batch(h, ns, circuits, terms, max_fused_qubits=5)
    exps, _, _ = mix.run()
    states = [mix.state(i) for i in range(len(ns))]
    for i in (0, 1, 3, 5):
        alone = P.Batch(h, [ns[i]], [circuits[i]], [terms[i]], max_fused_qubits=5)
        e1, _, _ = alone.run()
        np.testing.assert_array_equal(e1[0], exps[i])
        np.testing.assert_array_equal(alone.state(0), states[i])
        alone.close()
    mix.close()
    h.close()


def test_batch_level_setting_bounds(P, H):
    h = P.Handle()
    for bad in (12, 32, 0):
        with pytest.raises(P.SVError):
            h.set_batch_level_qubits(bad)
    h.set_batch_level_qubits(P.SV_BATCH_LEVEL_NONE)
    sizes = [17, 18]
    ns, circuits, terms = _mixed(8, sizes)
    b = P.Batch(h, ns, circuits, terms, max_fused_qubits=3)
    assert b.fusion_width(17) == 3  # persistent kernel at the fixed width
    exps, _, _ = b.run()
    _check(P, b, ns, circuits, terms, exps)
    b.close()
    h.close()


def test_batch_rejects_bad_input(P, H):
    with pytest.raises(P.SVError):
        P.Batch(H, [31], [W.brickwork(2, 1, 0)], [[1]], 5)
    with pytest.raises(P.SVError):
        P.Batch(H, [4], [W.brickwork(4, 1, 0)], [[1 << 4]], 5)
    with pytest.raises(P.SVError):
        P.Batch(H, [4], [W.brickwork(5, 1, 0)], [[1]], 5)
    with pytest.raises(P.SVError):
        P.Batch(H, [4], [W.brickwork(4, 1, 0)], [[1]], 6)


def test_batch_short_circuits_finish_first(P, H):
    # more large circuits than workgroups: the cheap circuits (the first 5%
    # of the work) are queued first, so every one of them completes before
    # most large ones; in largest-first order they would wait for a full
    # wave of large circuits.  The persistent kernel holds about 46 KiB of LDS per
    # workgroup, so at most 3 fit on a CU: 1000 large circuits outnumber its
    # workgroups on 256 CUs whatever its register use.
    rng = np.random.default_rng(9)
    small = [W.brickwork(8, int(rng.integers(4, 9)), 10_000 + i) for i in range(1200)]
    large = [W.brickwork(14, int(rng.integers(10, 17)), 20_000 + i) for i in range(1000)]
    import torch
    assert len(large) > 3 * torch.cuda.get_device_properties(0).multi_processor_count
    circuits = small + large
    ns = [8] * len(small) + [14] * len(large)
    terms = [[1] for _ in circuits]
    b = P.Batch(H, ns, circuits, terms, max_fused_qubits=5)
    b.run()
    _, lat, ks = b.run()
    b.close()
    lat_small, lat_large = lat[: len(small)], lat[len(small):]
    assert lat_small.max() < np.median(lat_large), (lat_small.max(), np.median(lat_large), ks)


def test_batch_autotuner_plans(P):
    # every size of a mixed batch gets a tuned plan: the persistent kernel's
    # width below the level-path size (15), a tile shape on the level path
    # (sizes tuned by earlier batches of this process keep theirs); the
    # results match the oracle
    sizes = [9, 12, 13, 14, 15, 16, 17, 19] * 2
    ns, circuits, terms = _mixed(91, sizes, 6, 14)
    h = P.Handle()
    b = P.Batch(h, ns, circuits, terms, max_fused_qubits=0)
    for n in set(sizes):
        p = b.plan(n)
        assert p["tuned"] == 1, (n, p)
        assert p["level_path"] == (1 if n >= 15 else 0), (n, p)
        if not p["level_path"]:
            assert 3 <= p["max_fused_qubits"] <= 5, (n, p)
        if p["level_path"]:
            assert p["max_fused_qubits"] == 5 and p["tiles_per_wg"] in (1, 2, 4, 8) and p["spread"] in (0, 1), (n, p)
            assert p["tiles_per_wg"] <= 1 << (n - 12)
        else:
            assert p["tiles_per_wg"] == 0 and p["spread"] == 0, (n, p)
    assert b.plan(25) == {"max_fused_qubits": 0, "level_path": 0, "tiles_per_wg": 0, "spread": 0, "tuned": 0}
    tune_s, build_s = b.host_times()
    assert tune_s >= 0.0 and build_s > 0.0
    exps, lat, ks = b.run()
    _check(P, b, ns, circuits, terms, exps)
    # a later batch with these sizes takes the same plans without timing
    b2 = P.Batch(h, ns[:8], circuits[:8], terms[:8], max_fused_qubits=0)
    assert b2.host_times()[0] == 0.0
    for n in sizes[:8]:
        assert b2.plan(n) == b.plan(n)
    e2, _, _ = b2.run()
    for i in range(8):
        np.testing.assert_array_equal(e2[i], exps[i])
    b2.close()
    # a fixed width takes no timing and the default level shape
    b3 = P.Batch(h, ns, circuits, terms, max_fused_qubits=4)
    assert b3.host_times()[0] == 0.0
    assert b3.plan(17) == {"max_fused_qubits": 5, "level_path": 1, "tiles_per_wg": 4, "spread": 1, "tuned": 0}
    assert b3.plan(12) == {"max_fused_qubits": 4, "level_path": 0, "tiles_per_wg": 0, "spread": 0, "tuned": 0}
    b3.close()
    b.close()
    h.close()


_CACHE_SCRIPT = r"""
import json, os, sys
sys.path.insert(0, os.getcwd())
import paper_2308_01999_amd as P
import workloads as W
h = P.Handle()
ns = [10, 14, 15, 17]
circuits = [W.brickwork(n, 8, 100 + n) for n in ns]
terms = [[1, 1 << (n - 1)] for n in ns]
b = P.Batch(h, ns, circuits, terms, max_fused_qubits=0)
exps, _, _ = b.run()
print(json.dumps({"tune_s": b.host_times()[0], "plans": {str(n): b.plan(n) for n in ns},
                  "exps": [[float(v) for v in e] for e in exps]}))
b.close()
h.close()
"""


def test_batch_tune_cache_file_across_processes(P, tmp_path):
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, SV_AUTOTUNE_CACHE=str(cache))

    def run():
        r = subprocess.run([sys.executable, "-c", _CACHE_SCRIPT], cwd=root, env=env, capture_output=True,
                           text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-3000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = run()
    assert first["tune_s"] > 0.0
    doc = json.load(open(cache))
    entries = {e["n"]: e for e in doc["entries"]}
    assert {10, 14, 15, 17} <= set(entries)
    assert entries[10]["kmax"] in (3, 4, 5) and entries[17]["tiles_per_wg"] in (1, 2, 4, 8)
    # the level path's sizes were timed together: one shape
    assert (entries[15]["tiles_per_wg"], entries[15]["spread"]) == (entries[17]["tiles_per_wg"], entries[17]["spread"])
    assert first["plans"]["15"]["level_path"] == 1 and first["plans"]["14"]["level_path"] == 0
    assert entries[14]["kmax"] != -1 and entries[14]["tiles_per_wg"] == -1  # persistent kernel only
    assert entries[17]["kmax"] == -1
    arch = entries[10]["arch"]
    # a second process reads the file: no timing, the same plans and results
    second = run()
    assert second["tune_s"] == 0.0
    assert second["plans"] == first["plans"]
    assert second["exps"] == first["exps"]
    # choices written by hand are taken as they are
    lines = [
        {"arch": arch, "dtype": "c64", "n": 10, "kmax": 3, "persistent_ms": 1.0, "tiles_per_wg": -1, "spread": -1,
         "level_ms": -1},
        {"arch": arch, "dtype": "c64", "n": 14, "kmax": 4, "persistent_ms": 1.0, "tiles_per_wg": 1, "spread": 0,
         "level_ms": 2.0},
        {"arch": arch, "dtype": "c64", "n": 15, "kmax": -1, "persistent_ms": -1, "tiles_per_wg": 8, "spread": 1,
         "level_ms": 1.0},
        {"arch": arch, "dtype": "c64", "n": 17, "kmax": -1, "persistent_ms": -1, "tiles_per_wg": 1, "spread": 0,
         "level_ms": 1.0},
    ]
    cache.write_text('{"sv_autotune": 1, "entries": [\n' + ",\n".join(json.dumps(x) for x in lines) + "\n]}\n")
    third = run()
    assert third["tune_s"] == 0.0
    p = third["plans"]
    assert p["10"] == {"max_fused_qubits": 3, "level_path": 0, "tiles_per_wg": 0, "spread": 0, "tuned": 1}
    assert p["14"] == {"max_fused_qubits": 4, "level_path": 0, "tiles_per_wg": 0, "spread": 0, "tuned": 1}
    assert p["15"] == {"max_fused_qubits": 5, "level_path": 1, "tiles_per_wg": 8, "spread": 1, "tuned": 1}
    assert p["17"] == {"max_fused_qubits": 5, "level_path": 1, "tiles_per_wg": 1, "spread": 0, "tuned": 1}
    for n, e in zip((10, 14, 15, 17), third["exps"]):
        ref = oracle.run(n, W.brickwork(n, 8, 100 + n))
        want = [oracle.expect_pauli(ref, [(0, "Z")]), oracle.expect_pauli(ref, [(n - 1, "Z")])]
        assert np.max(np.abs(np.array(e) - np.array(want))) <= 1e-4, (n, e, want)
