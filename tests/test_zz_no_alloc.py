"""The allocation-free sampler (sv_sample_noalloc) against sv_sample, through
the C ABI: both run the same kernels, one with the handle's own buffers and
one with a fixed per-GPU scratch array, so outcomes must agree bit for bit
(index work).  Two calls in a row, the second on a smaller state with fewer
shots, so the second call reads nothing stale from the first; the largest
state it takes and the first one it rejects; the samples also satisfy the
epsilon-interval rule on the oracle's CDF."""
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


@pytest.fixture(scope="module")
def H(P):
    h = P.Handle()
    yield h
    h.close()


def _eps_rule(psi_gpu, psi_ref, u, got):
    p_g = np.abs(psi_gpu.astype(np.complex128)) ** 2
    p_o = np.abs(psi_ref) ** 2
    eps = float(np.sum(np.abs(p_g - p_o))) + 1e-12
    _, cdf = oracle.sample(psi_ref, u[:1], return_cdf=True)
    got = got.astype(np.int64)
    lo = np.where(got > 0, cdf[np.maximum(got - 1, 0)], 0.0)
    r = u * cdf[-1]
    ok = (lo - eps <= r) & (r < cdf[got] + eps)
    assert ok.all(), f"{(~ok).sum()} samples outside their CDF interval"
    assert (p_g[got] > 0).all(), "sampled a zero-probability index"


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_noalloc_sampler_equals_sv_sample_two_calls(P, H, dt):
    cases = [(22, 6, 11, 300_000), (11, 8, 12, 5_000)]  # (n, depth, seed, shots): second call smaller
    states, refs, us, got = [], [], [], []
    for n, depth, seed, shots in cases:
        gates = W.brickwork(n, depth, seed)
        st = P.State(H, n, dt)
        st.run(gates, max_fused_qubits=5)
        states.append(st)
        refs.append(oracle.run(n, gates))
        us.append(W.uniforms(shots, seed + 100))
    order = [0, 4, 7, 1, 3]
    for st, u in zip(states, us):  # two allocation-free calls in a row
        print(f"sv_sample_noalloc {dt} n={st.n} shots={u.size}", flush=True)
        got.append((P.sv_sample_noalloc(st.s, u), P.sv_sample_noalloc(st.s, u[:4096], order)))
    for st, ref, u, (full, marg) in zip(states, refs, us, got):
        want = P.sv_sample(st.s, u)
        assert np.array_equal(full, want), f"n={st.n}: outcomes differ from sv_sample"
        assert np.array_equal(marg, P.sv_sample(st.s, u[:4096], order))
        psi = st.to_numpy()
        _eps_rule(psi, ref, u, full)
        bits = np.zeros_like(full[:4096])
        for a, q in enumerate(order):
            bits |= ((full[:4096] >> np.uint64(q)) & np.uint64(1)) << np.uint64(a)
        assert np.array_equal(marg, bits)
        st.close()


def test_noalloc_sampler_largest_state_and_limit(P, H):
    n = P.SV_SAMPLE_NOALLOC_MAX_QUBITS
    st = P.State(H, n, "c64")
    gates = [("h", [q], []) for q in range(0, n, 3)] + [("u3", [n - 1], [0.7, 0.2, 1.1]), ("cx", [n - 1, 1], [])]
    st.run(gates)
    u = W.uniforms(1 << 16, 5)
    print(f"sv_sample_noalloc c64 n={n} shots={u.size}", flush=True)
    got = P.sv_sample_noalloc(st.s, u)
    assert np.array_equal(got, P.sv_sample(st.s, u))
    st.close()
    big = P.State(H, n + 1, "c64")
    out = np.full(8, 7, dtype=np.uint64)
    import ctypes
    rc = P._L.sv_sample_noalloc(ctypes.c_void_p(big.s), P._dptr(u[:8]), 8, None, 0,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    assert rc == P.SV_ERR_INVALID_VALUE
    assert "at most" in P.sv_last_error()
    assert (out == 7).all()
    big.close()


def test_noalloc_sampler_argument_errors(P, H):
    st = P.State(H, 6, "c128")
    assert P.sv_sample_noalloc(st.s, np.zeros(0)).size == 0
    with pytest.raises(P.SVError):
        P.sv_sample_noalloc(st.s, np.array([0.5, 1.0]))
    with pytest.raises(P.SVError):
        P.sv_sample_noalloc(st.s, np.array([0.5]), [0, 0])
    st.close()
