"""GPU test of the serving loop: requests of mixed sizes arriving while
others run are admitted under a tight HBM budget; each result matches the
oracle and is bitwise the same as when the request runs alone."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_01999_amd as P
    return P


def _eps_ok(psi_gpu_p, psi_ref, u, got):
    p_o = np.abs(psi_ref) ** 2
    _, cdf = oracle.sample(psi_ref, u[:1], return_cdf=True)
    N = cdf[-1]
    eps = float(np.sum(np.abs(psi_gpu_p - p_o))) + 1e-12
    got = got.astype(np.int64)
    lo = np.where(got > 0, cdf[np.maximum(got - 1, 0)], 0.0)
    r = u * N
    return bool(((lo - eps <= r) & (r < cdf[got] + eps)).all())


def test_serving_mix_matches_alone_and_oracle(P):
    from paper_2308_01999_amd import serve
    from paper_2308_01999_amd.serve import Server, replay, slot_reserve
    reqs = W.serving_requests(14, rate_per_s=400.0, seed=3, n_lo=6, n_hi=16, d_lo=4, d_hi=20,
                              n_terms=6, n_shots=256)
    # a few of the largest states at once, beside each slot's reserve
    states = 3 * (1 << 16) * 8
    # two general slots and two kept for requests of up to 12 qubits
    srv = Server(slots=2, small_slots=2, small_qubits=12,
                 budget_bytes=states + 2 * slot_reserve(16) + 2 * slot_reserve(12), dtype="c64", kmax=5,
                 max_qubits=16)
    mixed = replay(srv, reqs)
    srv.close()
    assert all(not m.error for m in mixed.values()), [m.error for m in mixed.values()]
    alone_srv = Server(slots=1, budget_bytes=states + slot_reserve(16), dtype="c64", kmax=5, max_qubits=16)
    for r in reqs:
        one = replay(alone_srv, [r])[r.rid]
        m = mixed[r.rid]
        np.testing.assert_array_equal(one.expectations, m.expectations)
        np.testing.assert_array_equal(one.samples, m.samples)
    alone_srv.close()
    h = P.Handle()
    for r in reqs:
        ref = oracle.run(r.n, r.gates)
        er = np.array([oracle.expect_pauli(ref, t) for t in r.terms])
        assert np.max(np.abs(mixed[r.rid].expectations - er)) <= 1e-4
        assert mixed[r.rid].latency > 0
        # the served samples against the oracle's CDF by the epsilon rule,
        # with epsilon from the served state: the same fused pieces rebuilt
        # on a fresh state, which samples bitwise the same outcomes
        st = P.State(h, r.n, "c64")
        for part in serve.fusion_pieces(r.n, r.gates):
            f = P.fuse(part, 5)
            P.sv_apply_fused(st.s, f.f)
            f.free()
        psi = st.to_numpy().astype(np.complex128)
        np.testing.assert_array_equal(st.sample(np.asarray(r.uniforms)), mixed[r.rid].samples)
        st.close()
        assert _eps_ok(np.abs(psi) ** 2, ref, np.asarray(r.uniforms), mixed[r.rid].samples), r.rid
    h.close()
    # results arrive for every request; latency covers queueing
    assert all(m.done >= m.admitted >= m.arrival for m in mixed.values())


def test_large_request_with_coupled_fusion_matches_oracle(P):
    # a request above the coupled-fusion size: served expectations against
    # the oracle, samples by the epsilon rule on the served state (rebuilt
    # with the same coupled program, which samples bitwise the same)
    from paper_2308_01999_amd import serve
    from paper_2308_01999_amd.serve import Server, replay, slot_reserve
    n = serve.COUPLED_QUBITS
    reqs = W.serving_requests(1, rate_per_s=100.0, seed=11, n_lo=n, n_hi=n, d_lo=8, d_hi=8,
                              n_terms=6, n_shots=512)
    r = reqs[0]
    srv = Server(slots=1, budget_bytes=(1 << n) * 8 + slot_reserve(n), dtype="c64", kmax=5, max_qubits=n)
    res = replay(srv, reqs)[r.rid]
    srv.close()
    assert not res.error, res.error
    f = P.fuse(r.gates, 5, coupled=True)
    assert res.fused_blocks == f.count
    h = P.Handle()
    st = P.State(h, n, "c64")
    P.sv_apply_fused(st.s, f.f)
    f.free()
    psi = st.to_numpy().astype(np.complex128)
    np.testing.assert_array_equal(st.sample(np.asarray(r.uniforms)), res.samples)
    st.close()
    h.close()
    ref = oracle.run(n, r.gates)
    er = np.array([oracle.expect_pauli(ref, t) for t in r.terms])
    assert np.max(np.abs(res.expectations - er)) <= 1e-4
    assert oracle.fidelity(ref, psi) >= 1 - 1e-5
    assert _eps_ok(np.abs(psi) ** 2, ref, np.asarray(r.uniforms), res.samples)
