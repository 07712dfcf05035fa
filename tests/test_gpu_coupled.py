"""GPU parity of coupled fusion (sv_fuse_gate_list_coupled): blocks whose
phase couplings carry the controlled phases deferred from earlier blocks,
applied by the five-qubit tile sweeps with the coupling folded in (states of
>= 14 qubits, smaller blocks padded to five qubits) or by the plain sweeps
after a separate coupling pass (smaller states), against the oracle on the
same circuits; every tile variant; recorded programs; the QFT closed form."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

C128_TOL = 1e-10
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


def _check(got, ref, dt):
    got = got.astype(np.complex128)
    if dt == "c128":
        err = float(np.max(np.abs(got - ref)))
        assert err <= C128_TOL, f"max |d amp| = {err}"
    else:
        fid = oracle.fidelity(ref, got)
        assert fid >= C64_FID, f"fidelity = {fid}"
        assert float(np.max(np.abs(got - ref))) <= 1e-5


def _circuit(name, n, seed):
    return {"qft": lambda: W.qft(n), "diagheavy": lambda: W.diagonal_heavy(n, 120, seed),
            "cxcp": lambda: W.random_cx_cp(n, 8, seed), "brickwork": lambda: W.brickwork(n, 8, seed),
            "cxcp_qft": lambda: W.random_cx_cp(n, 4, seed) + W.qft(n)}[name]()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 13, 14, 17])
@pytest.mark.parametrize("circuit", ["qft", "diagheavy", "cxcp", "brickwork", "cxcp_qft"])
def test_coupled_fusion_matches_oracle(P, H, dt, n, circuit):
    gates = _circuit(circuit, n, 100 + n)
    x = W.random_basis_state(n, n)
    ref = oracle.run(n, gates, basis=x)
    st = P.State(H, n, dt, basis=x)
    st.run(gates, max_fused_qubits=5, coupled=True)
    _check(st.to_numpy(), ref, dt)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_coupled_fusion_every_tile_variant(P, dt, mode):
    # the coupled sweeps take the tile variant the handle uses for the plain
    # ones; force each and compare with the oracle
    n = 16
    gates = W.random_cx_cp(n, 6, 7) + W.qft(n)
    x = W.random_basis_state(n, 8)
    ref = oracle.run(n, gates, basis=x)
    h = P.Handle()
    h.set_tile_mode(mode)
    st = P.State(h, n, dt, basis=x)
    st.run(gates, max_fused_qubits=5, coupled=True)
    _check(st.to_numpy(), ref, dt)
    st.close()
    h.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_coupled_program_replays_from_a_graph(P, H, dt):
    n = 15
    gates = W.diagonal_heavy(n, 100, 3) + W.qft(n)
    x = W.random_basis_state(n, 4)
    eager = P.State(H, n, dt, basis=x)
    eager.run(gates, max_fused_qubits=5, coupled=True)
    want = eager.to_numpy()
    eager.close()
    st = P.State(H, n, dt, basis=x)
    g = P.Graph(st, gates, 5, coupled=True)
    for _ in range(3):
        P.sv_set_basis_state(st.s, x)
        g.launch()
        np.testing.assert_array_equal(st.to_numpy(), want)
    g.close()
    st.close()
    _check(want, oracle.run(n, gates, basis=x), dt)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [20, 24])
def test_coupled_qft_closed_form(P, H, dt, n):
    # the QFT of |x>: amplitude y is exp(2 pi i x y / 2^n) / 2^(n/2)
    x = W.random_basis_state(n, n + 1)
    st = P.State(H, n, dt, basis=x)
    nb = st.run(W.qft(n), max_fused_qubits=5, coupled=True)
    assert nb <= math.ceil(n / 5) + math.ceil(n // 2 / 2) + 1
    y = np.arange(1 << n, dtype=np.int64)
    ref = np.exp(2j * math.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    got = st.to_numpy().astype(np.complex128)
    tol = C128_TOL if dt == "c128" else 2e-6 / math.sqrt(1 << n) * 64
    assert np.max(np.abs(got - ref)) <= tol
    st.close()
