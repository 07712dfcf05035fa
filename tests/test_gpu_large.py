"""Full-size states of the large configuration: 34 qubits complex64 and 33
qubits complex128 (128 GiB each), in the launch configuration the benchmark
uses (fused blocks of up to 5 qubits through the tiled kernels).  A host
oracle of that size would take hours, so these tests check what holds at
any size:
  - the QFT of a random basis state against its closed form on sampled
    amplitudes, the norm, and 2^20 samples of its uniform distribution by
    the epsilon rule;
  - H on every qubit plus CZ signs: all probabilities are equal bit for bit
    in the GPU's own arithmetic (every output amplitude is a single product
    of equal-magnitude factors), so each of 2^20 samples is floor(u 2^n) up
    to one index;
  - a random CNOT/controlled-phase circuit followed by its mirror returns to
    the start state (amplitude, norm, every sample);
  - a GHZ state built along a random qubit order that includes the top index
    bits: its two amplitudes, <Z Z> across the top bits, and its samples.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = [(34, "c64"), (33, "c128")]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, total = torch.cuda.mem_get_info()
    if free < (134 << 30):
        pytest.skip("needs 134 GiB of free device memory")
    import paper_2308_01999_amd as P
    return P


@pytest.fixture(scope="module")
def H(P):
    h = P.Handle()
    yield h
    h.close()


def _release():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _amps(P, st, idx):
    dt = P.NP_DTYPES[st.dt]
    out = np.empty(len(idx), dtype=np.complex128)
    one = np.empty(1, dtype=dt)
    for j, i in enumerate(idx):
        P.sv_copy_to_host(st.s, one, int(i), 1)
        out[j] = one[0]
    return out


@pytest.mark.parametrize("n,dt", CASES)
def test_qft_closed_form_and_uniform_sampling(P, H, n, dt):
    x = W.random_basis_state(n, 1234 + n)
    st = P.State(H, n, dt, basis=x)
    nb = st.run(W.qft(n), max_fused_qubits=5)
    assert nb > 0
    rng = np.random.default_rng(n)
    ys = rng.integers(0, 1 << n, size=4096, dtype=np.uint64).tolist() + [0, 1, (1 << n) - 1]
    got = _amps(P, st, ys)
    ref = np.array([np.exp(2j * math.pi * ((x * y) % (1 << n)) / (1 << n)) for y in ys]) / math.sqrt(1 << n)
    rel = np.max(np.abs(got - ref)) * math.sqrt(1 << n)
    assert rel <= (1e-9 if dt == "c128" else 2e-4), rel
    nrm = st.norm()
    assert abs(nrm - 1.0) <= (1e-10 if dt == "c128" else 1e-4)
    # every exact probability is 2^-n, so the exact CDF is C_i = (i + 1) 2^-n
    # and the epsilon rule bounds how far an outcome may sit from
    # floor(u 2^n): |C - C_gpu| <= sum |dp| <= 2 ||d psi|| + ||d psi||^2, with
    # ||d psi|| estimated from the sampled amplitudes (safety factor 10)
    dnorm = math.sqrt(float(np.mean(np.abs(got - ref) ** 2)) * (1 << n))
    eps = 10 * (2 * dnorm + dnorm ** 2) + 1e-12
    u = W.uniforms(1 << 20, 77)
    s = st.sample(u).astype(np.float64)
    dev = np.abs(s - np.floor(u * (1 << n)))
    assert dev.max() <= eps * (1 << n) + 2, (dev.max(), eps)
    st.close()
    _release()


@pytest.mark.parametrize("n,dt", CASES)
def test_uniform_superposition_samples_exact(P, H, n, dt):
    rng = np.random.default_rng(50 + n)
    order = [int(v) for v in rng.permutation(n)]
    gates = [W.Gate("h", (q,), ()) for q in order]
    for _ in range(n):
        a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
        gates.append(W.Gate("cz", (a, b), ()))
    gates.append(W.Gate("cz", (n - 1, n - 2), ()))
    st = P.State(H, n, dt)
    st.run(gates, max_fused_qubits=5)
    a = _amps(P, st, [0, (1 << n) - 1, 12345, 1 << (n - 1)])
    assert np.ptp(np.abs(a)) == 0.0, a  # equal magnitudes bit for bit
    assert abs(abs(a[0]) - 2.0 ** (-n / 2)) <= (4e-15 if dt == "c128" else 1e-6) * 2.0 ** (-n / 2)
    u = W.uniforms(1 << 20, 78)
    s = st.sample(u).astype(np.float64)
    dev = np.abs(s - np.floor(u * (1 << n)))
    assert dev.max() <= 1, dev.max()
    st.close()
    _release()


@pytest.mark.parametrize("n,dt", CASES)
def test_random_cx_cp_mirror_returns_to_start(P, H, n, dt):
    x = W.random_basis_state(n, 99 + n)
    gates = W.random_cx_cp(n, 12, 7 + n)
    assert any(max(g.qubits) == n - 1 for g in gates if len(g.qubits) == 2)
    st = P.State(H, n, dt, basis=x)
    st.run(gates + W.inverse(gates), max_fused_qubits=5)
    a = _amps(P, st, [x, (x + 1) % (1 << n)])
    tol = 1e-10 if dt == "c128" else 2e-4
    assert abs(a[0] - 1.0) <= tol and abs(a[1]) <= tol, a
    assert abs(st.norm() - 1.0) <= (1e-10 if dt == "c128" else 1e-4)
    s = st.sample(W.uniforms(1 << 16, 3))
    assert (s == x).all()
    st.close()
    _release()


@pytest.mark.parametrize("n,dt", CASES)
def test_ghz_across_top_bits(P, H, n, dt):
    order = [int(v) for v in np.random.default_rng(n).permutation(n)]
    st = P.State(H, n, dt)
    st.run(W.ghz(n, order), max_fused_qubits=5)
    a = _amps(P, st, [0, (1 << n) - 1, 1 << (n - 1), 12345])
    tol = 1e-12 if dt == "c128" else 1e-6
    assert abs(a[0] - 1 / math.sqrt(2)) <= tol and abs(a[1] - 1 / math.sqrt(2)) <= tol
    assert abs(a[2]) <= tol and abs(a[3]) <= tol
    e = st.expect([[(n - 1, "Z"), (n - 2, "Z")], [(0, "Z"), (n - 1, "Z")], [(n - 1, "Z")],
                   [(q, "X") for q in range(n)]])
    np.testing.assert_allclose(e, [1.0, 1.0, 0.0, 1.0], atol=(1e-10 if dt == "c128" else 1e-5))
    s = st.sample(W.uniforms(1 << 16, 5))
    assert set(np.unique(s).tolist()) <= {0, (1 << n) - 1}
    st.close()
    _release()
