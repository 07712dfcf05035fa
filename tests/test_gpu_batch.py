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
