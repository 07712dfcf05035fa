"""GPU parity: libsv (through its C ABI) against the CPU oracle on the same
seeded inputs, plus closed forms and properties at sizes the oracle cannot
hold.  Tolerances: complex128 max |d amp| <= 1e-10; complex64 state fidelity
>= 1 - 1e-5 at depth 20; expectations |d| <= 1e-9 (c128) / 1e-4 (c64);
samples by the epsilon-interval rule (a GPU outcome i for uniform u is valid
if C_{i-1} - eps <= u N < C_i + eps on the oracle's CDF, eps = sum |p_gpu -
p_oracle| + 1e-12)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
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


def _state(P, H, n, dt, basis=0):
    return P.State(H, n, dt, basis=basis)


def _check_state(gpu, ref, dt):
    gpu = gpu.astype(np.complex128)
    if dt == "c128":
        err = float(np.max(np.abs(gpu - ref)))
        assert err <= C128_TOL, f"max |d amp| = {err}"
    else:
        fid = oracle.fidelity(ref, gpu)
        assert fid >= C64_FID, f"fidelity = {fid}"


def _eps_rule(psi_gpu, psi_ref, u, got):
    p_g = np.abs(psi_gpu.astype(np.complex128)) ** 2
    p_o = np.abs(psi_ref) ** 2
    eps = float(np.sum(np.abs(p_g - p_o))) + 1e-12
    _, cdf = oracle.sample(psi_ref, u[:1], return_cdf=True)
    N = cdf[-1]
    got = got.astype(np.int64)
    lo = np.where(got > 0, cdf[np.maximum(got - 1, 0)], 0.0)
    hi = cdf[got]
    r = u * N
    ok = (lo - eps <= r) & (r < hi + eps)
    assert ok.all(), f"{(~ok).sum()} samples outside their CDF interval"
    assert (p_g[got] > 0).all(), "sampled a zero-probability index"


# --------------------------------------------------------------- gate level

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,seed", [(3, 0), (7, 1), (12, 2), (16, 3), (13, 4)])
def test_random_dense_gates_with_controls(P, H, dt, n, seed):
    ops = W.random_dense_circuit(n, 24, min(6, n), 500 + seed)
    x = W.random_basis_state(n, seed)
    ref = oracle.basis_state(n, x)
    st = _state(P, H, n, dt, basis=x)
    for t, c, cv, m in ops:
        oracle.apply(ref, m, t, c, cv)
        st.apply_matrix(m, t, c, cv)
    _check_state(st.to_numpy(), ref, dt)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_each_gate_size_low_mixed_high_targets(P, H, dt, k):
    n = 14
    rng = np.random.default_rng(k)
    for targets in [tuple(range(k)), tuple(range(n - k, n)), tuple(int(v) for v in rng.choice(n, k, replace=False))]:
        m = W.haar_unitary(k, rng)
        psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        psi0 /= np.linalg.norm(psi0)
        st = _state(P, H, n, dt, basis=None)
        st_np = psi0.astype(P.NP_DTYPES[st.dt])
        P.sv_copy_from_host(st.s, st_np)
        ref = st_np.astype(np.complex128)
        oracle.apply(ref, m, targets)
        st.apply_matrix(m, targets)
        out = st.to_numpy().astype(np.complex128)
        tol = 1e-12 if dt == "c128" else 2e-6
        assert np.max(np.abs(out - ref)) <= tol, targets
        st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("k", [7, 8, 10])
def test_large_gates(P, H, dt, k):
    n = 12
    rng = np.random.default_rng(40 + k)
    targets = tuple(int(v) for v in rng.choice(n, k, replace=False))
    m = W.haar_unitary(k, rng)
    ref = oracle.run(n, W.brickwork(n, 2, k))
    st = _state(P, H, n, dt, basis=None)
    P.sv_copy_from_host(st.s, ref.astype(P.NP_DTYPES[st.dt]))
    ref = ref.astype(P.NP_DTYPES[st.dt]).astype(np.complex128)
    oracle.apply(ref, m, targets)
    st.apply_matrix(m, targets)
    out = st.to_numpy().astype(np.complex128)
    assert np.max(np.abs(out - ref)) <= (1e-12 if dt == "c128" else 5e-6)
    st.close()


def test_adjoint_flag(P, H):
    n = 9
    rng = np.random.default_rng(3)
    m = W.haar_unitary(3, rng)
    st = _state(P, H, n, "c128", basis=5)
    st.apply_matrix(m, (1, 7, 4))
    st.apply_matrix(m, (1, 7, 4), adjoint=True)
    out = st.to_numpy()
    ref = oracle.basis_state(n, 5)
    assert np.max(np.abs(out - ref)) <= 1e-14
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("k,n_ctrl,targets", [
    (5, 0, (0, 1, 2, 3, 4)), (5, 0, (14, 3, 9, 11, 6)),  # five-qubit tiles
    (6, 0, (2, 13, 5, 8, 0, 10)),                       # six-qubit tiles
    (4, 0, (12, 1, 7, 4)), (2, 0, (9, 3)),              # padded to five qubits
    (4, 1, (2, 11, 5, 0)), (5, 1, (6, 1, 13, 9, 3)),    # controlled: direct matrix-core path
    (3, 2, (10, 4, 7)),                                 # controlled, vector path
])
def test_adjoint_flag_on_every_sweep(P, H, dt, k, n_ctrl, targets):
    # a non-unitary matrix, so M^dagger differs from M^-1: the result must be
    # the oracle's application of the conjugate transpose
    n = 15
    rng = np.random.default_rng(100 * k + n_ctrl)
    d = 1 << k
    m = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0 * d)
    free = [q for q in range(n) if q not in targets]
    controls = tuple(int(v) for v in rng.choice(free, n_ctrl, replace=False))
    cvals = [int(v) for v in rng.integers(0, 2, size=n_ctrl)]
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 /= np.linalg.norm(psi0)
    st = _state(P, H, n, dt, basis=None)
    st_np = psi0.astype(P.NP_DTYPES[st.dt])
    P.sv_copy_from_host(st.s, st_np)
    ref = st_np.astype(np.complex128)
    oracle.apply(ref, np.conj(m).T, targets, controls, cvals)
    st.apply_matrix(m, targets, controls, cvals, adjoint=True)
    out = st.to_numpy().astype(np.complex128)
    tol = 1e-12 if dt == "c128" else 2e-6
    assert np.max(np.abs(out - ref)) <= tol
    st.close()


# ------------------------------------------------------------- whole circuits

@pytest.mark.parametrize("seed", [0, 1])
def test_config1_brickwork_12q_c128(P, H, seed):
    n, depth = 12, 20
    gates = W.brickwork(n, depth, seed)
    ref = oracle.run(n, gates)
    st = _state(P, H, n, "c128")
    st.run(gates)
    gpu = st.to_numpy()
    _check_state(gpu, ref, "c128")
    z = st.expect(W.z_terms(n))
    zr = np.array([oracle.expect_pauli(ref, t) for t in W.z_terms(n)])
    assert np.max(np.abs(z - zr)) <= 1e-9
    assert abs(st.norm() - 1.0) <= 1e-12
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 5, 6])
def test_fused_brickwork_matches_oracle(P, H, dt, kmax):
    n, depth = 12, 20
    gates = W.brickwork(n, depth, 7)
    ref = oracle.run(n, gates)
    st = _state(P, H, n, dt)
    nb = st.run(gates, max_fused_qubits=kmax)
    assert nb >= 1
    _check_state(st.to_numpy(), ref, dt)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fused_kmax6_on_tiles_matches_oracle(P, H, dt):
    # six-qubit blocks through the k = 6 MFMA tiles (64 KiB tiles, several per
    # state), low, mixed and high windows
    n, depth = 16, 12
    gates = W.brickwork(n, depth, 13)
    ref = oracle.run(n, gates)
    st = _state(P, H, n, dt)
    nb = st.run(gates, max_fused_qubits=6)
    assert nb >= 1
    _check_state(st.to_numpy(), ref, dt)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_brickwork_20q_unfused_and_fused(P, H, dt):
    n, depth = 20, 20
    gates = W.brickwork(n, depth, 11)
    ref = oracle.run(n, gates)
    for kmax in (None, 5):
        st = _state(P, H, n, dt)
        st.run(gates, max_fused_qubits=kmax)
        _check_state(st.to_numpy(), ref, dt)
        st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_random_cx_cp_and_qft(P, H, dt):
    n = 14
    x = W.random_basis_state(n, 21)
    gates = W.random_cx_cp(n, 12, 21) + W.qft(n)
    ref = oracle.run(n, gates, basis=x)
    for kmax in (None, 4, 5):
        st = _state(P, H, n, dt, basis=x)
        st.run(gates, max_fused_qubits=kmax)
        _check_state(st.to_numpy(), ref, dt)
        st.close()


@pytest.mark.parametrize("n", [20, 23])
def test_qft_closed_form(P, H, n):
    x = W.random_basis_state(n, n)
    st = _state(P, H, n, "c128", basis=x)
    st.run(W.qft(n), max_fused_qubits=5)
    y = np.arange(1 << n, dtype=np.int64)
    ref = np.exp(2j * math.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    assert np.max(np.abs(st.to_numpy() - ref)) <= C128_TOL
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_ghz_nonadjacent_and_expectations(P, H, dt):
    n = 22
    order = [int(v) for v in np.random.default_rng(5).permutation(n)]
    st = _state(P, H, n, dt)
    st.run(W.ghz(n, order))
    out = st.to_numpy().astype(np.complex128)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(out - ref)) <= (1e-14 if dt == "c128" else 1e-7)
    tol = 1e-12 if dt == "c128" else 1e-6
    e = st.expect([[(0, "Z"), (n - 1, "Z")], [(3, "Z")], [(q, "X") for q in range(n)],
                   [(0, "Y"), (1, "Y")] + [(q, "X") for q in range(2, n)]])
    np.testing.assert_allclose(e, [1.0, 0.0, 1.0, -1.0], atol=tol)
    u = W.uniforms(4096, 3)
    s = st.sample(u)
    assert set(np.unique(s).tolist()) <= {0, (1 << n) - 1}
    _eps_rule(out, ref, u, s)
    st.close()


def test_cluster_state_stabilisers(P, H):
    n = 16
    st = _state(P, H, n, "c128")
    st.run(W.cluster_1d(n))
    terms = []
    for i in range(n):
        terms.append([(i, "X")] + ([(i - 1, "Z")] if i > 0 else []) + ([(i + 1, "Z")] if i < n - 1 else []))
    e = st.expect(terms)
    np.testing.assert_allclose(e, np.ones(n), atol=1e-12)
    st.close()


# --------------------------------------------------------------- reductions

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 5, 11, 17])
def test_pauli_expectations_vs_oracle(P, H, dt, n):
    rng = np.random.default_rng(70 + n)
    gates = W.brickwork(n, 6, n)
    ref = oracle.run(n, gates)
    st = _state(P, H, n, dt)
    st.run(gates)
    gpu = st.to_numpy().astype(np.complex128)
    terms = W.random_pauli_terms(n, 20, rng) + W.z_terms(n) + W.zz_neighbour_terms(n)
    e = st.expect(terms)
    # compare against the oracle on the GPU's own state (isolates the
    # reduction) and on the oracle's state (end to end)
    e_own = np.array([oracle.expect_pauli(gpu, t) for t in terms])
    e_ref = np.array([oracle.expect_pauli(ref, t) for t in terms])
    assert np.max(np.abs(e - e_own)) <= (1e-12 if dt == "c128" else 1e-6)
    assert np.max(np.abs(e - e_ref)) <= (1e-9 if dt == "c128" else 1e-4)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 11, 22, 23])
def test_many_pauli_strings_in_groups(P, H, dt, n):
    # more distinct X/Y masks than one group of sweeps (64) holds, mixed with
    # Z strings: states of at most 22 qubits run each group as one launch
    # per kind of sweep, larger ones sweep by sweep; both against the
    # oracle on the GPU's own state, and the same terms one at a time agree
    # (up to the norm, which a call takes from its first sweep)
    rng = np.random.default_rng(400 + n)
    st = _state(P, H, n, dt)
    st.run(W.brickwork(n, 3, 40 + n))
    gpu = st.to_numpy().astype(np.complex128)
    count = 150 if n >= 11 else 40
    terms = W.random_pauli_terms(n, count, rng) + W.z_terms(n)
    e = st.expect(terms)
    e_own = np.array([oracle.expect_pauli(gpu, t) for t in terms])
    assert np.max(np.abs(e - e_own)) <= (1e-12 if dt == "c128" else 1e-6)
    for i in range(0, len(terms), max(1, len(terms) // 7)):
        np.testing.assert_allclose(st.expect([terms[i]]), e[i : i + 1], rtol=0, atol=1e-13)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_norm_renormalize_and_determinism(P, H, dt):
    n = 18
    st = _state(P, H, n, dt)
    st.run(W.brickwork(n, 5, 2))
    P.sv_copy_from_host(st.s, (st.to_numpy() * 3.0).astype(P.NP_DTYPES[st.dt]))
    gpu = st.to_numpy().astype(np.complex128)
    n1 = st.norm()
    n2 = st.norm()
    assert n1 == n2  # bitwise reproducible
    assert n1 == pytest.approx(oracle.norm(gpu), rel=1e-13)
    before = P.sv_renormalize(st.s)
    assert before == n1
    assert st.norm() == pytest.approx(1.0, abs=(1e-13 if dt == "c128" else 1e-6))
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [2, 9, 14, 21])
def test_sampling_epsilon_rule(P, H, dt, n):
    gates = W.brickwork(n, 8, 30 + n)
    ref = oracle.run(n, gates)
    st = _state(P, H, n, dt)
    st.run(gates)
    gpu = st.to_numpy()
    u = W.uniforms(50000, n)
    got = st.sample(u)
    _eps_rule(gpu, ref, u, got)
    # the same uniforms give the same outcomes (deterministic)
    np.testing.assert_array_equal(st.sample(u), got)
    st.close()


def test_sampling_hand_tables(P, H):
    g = json.load(open(os.path.join(GOLD, "sampling_table.json")))
    st = _state(P, H, 2, "c128", basis=None)
    P.sv_copy_from_host(st.s, np.array(g["psi_re"]) + 1j * np.array(g["psi_im"]))
    assert st.sample(g["uniforms"]).tolist() == g["expected"]
    assert st.sample(g["uniforms"], [1]).tolist() == g["bit_ordering_[1]"]
    assert st.sample(g["uniforms"], [1, 0]).tolist() == g["bit_ordering_[1,0]"]
    st.close()
    t = json.load(open(os.path.join(GOLD, "sampling_ties.json")))
    for dt in ("c128", "c64"):
        st = _state(P, H, 3, dt, basis=None)
        P.sv_copy_from_host(st.s, np.array(t["psi_re"]).astype(P.NP_DTYPES[st.dt]))
        assert st.sample(t["uniforms"]).tolist() == t["expected"]
        st.close()


def test_sampling_bit_ordering_is_marginal(P, H):
    n = 13
    st = _state(P, H, n, "c128")
    st.run(W.brickwork(n, 6, 4))
    u = W.uniforms(20000, 9)
    full = st.sample(u)
    sub = st.sample(u, [12, 0, 5])
    np.testing.assert_array_equal(sub, ((full >> 12) & 1) | (((full >> 0) & 1) << 1) | (((full >> 5) & 1) << 2))
    st.close()


def test_sampling_zero_probability_blocks(P, H):
    # a state whose mass sits in a few isolated amplitudes across chunk
    # boundaries: every outcome must be one of them
    n = 20
    psi = np.zeros(1 << n, dtype=np.complex128)
    idx = [0, 4095, 4096, 777777, (1 << n) - 1]
    psi[idx] = [0.5, 0.5j, 0.5, -0.5, 0.0]
    st = _state(P, H, n, "c128", basis=None)
    P.sv_copy_from_host(st.s, psi)
    u = W.uniforms(100000, 1)
    got = st.sample(u)
    assert set(np.unique(got).tolist()) <= {0, 4095, 4096, 777777}
    _eps_rule(psi, psi, u, got)
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [5, 14, 18])
def test_sampling_block_and_chunk_boundaries(P, H, dt, n):
    # mass on both sides of 64-amplitude block and chunk boundaries, zeros in
    # between, and amplitudes far too small to move a running sum: every
    # outcome must carry non-zero probability and obey the epsilon rule
    dim = 1 << n
    psi = np.zeros(dim, dtype=np.complex128)
    heavy = sorted({i % dim for i in (0, 63, 64, 127, 4095, 4096, 16383, 16384, dim - 1)})
    psi[heavy] = 1.0
    psi[heavy[1:-1]] = 0.5j
    for i in (1, 65, 4097):
        if i < dim and psi[i] == 0:
            psi[i] = 1e-13  # probability 1e-26: absorbed by the prefix
    psi /= np.linalg.norm(psi)
    st = _state(P, H, n, dt, basis=None)
    P.sv_copy_from_host(st.s, psi.astype(P.NP_DTYPES[st.dt]))
    gpu = st.to_numpy()
    u = np.concatenate([W.uniforms(40000, 2 + n), np.linspace(0.0, 1.0, 4097)[:-1]])
    got = st.sample(u)
    assert (np.abs(gpu[got]) > 0).all()
    _eps_rule(gpu, gpu.astype(np.complex128), u, got)
    st.close()


# ---------------------------------------------------------------- edge cases

def test_invalid_arguments_leave_state_untouched(P, H):
    n = 6
    st = _state(P, H, n, "c128", basis=3)
    with pytest.raises(P.SVError) as e:
        st.apply_matrix(np.eye(2), (6,))
    assert e.value.status == P.SV_ERR_INVALID_VALUE
    with pytest.raises(P.SVError):
        st.apply_matrix(np.eye(4), (1, 1))
    with pytest.raises(P.SVError):
        st.apply_matrix(np.eye(2), (1,), (1,))
    with pytest.raises(P.SVError):
        st.apply_matrix(np.eye(2), (1,), (2,), (2,))
    with pytest.raises(P.SVError):
        st.apply_matrix(np.full((2, 2), np.nan), (1,))
    with pytest.raises(P.SVError):
        st.sample([0.5, 1.0])
    with pytest.raises(P.SVError):
        st.expect([[(0, "Q")]])
    with pytest.raises(P.SVError):
        st.expect([[(0, "X"), (0, "Z")]])
    with pytest.raises(P.SVError):
        P.sv_set_basis_state(st.s, 1 << n)
    out = st.to_numpy()
    assert out[3] == 1.0 and np.count_nonzero(out) == 1
    st.close()


def test_zero_norm_state_is_rejected(P, H):
    st = _state(P, H, 4, "c64", basis=None)
    P.sv_copy_from_host(st.s, np.zeros(16, dtype=np.complex64))
    with pytest.raises(P.SVError):
        st.sample([0.1])
    with pytest.raises(P.SVError):
        st.expect([[(0, "Z")]])
    st.close()


def test_one_qubit_state_and_empty_inputs(P, H):
    st = _state(P, H, 1, "c128")
    st.apply_gate(W.Gate("h", (0,), ()))
    np.testing.assert_allclose(st.to_numpy(), [1 / math.sqrt(2)] * 2, atol=1e-15)
    assert st.sample(np.zeros(0)).size == 0
    assert st.expect([]).size == 0
    assert st.run([], max_fused_qubits=5) == 0
    st.close()


def test_copy_ranges(P, H):
    n = 10
    st = _state(P, H, n, "c64", basis=None)
    data = (np.arange(1 << n) + 1j * np.arange(1 << n)[::-1]).astype(np.complex64)
    P.sv_copy_from_host(st.s, data)
    part = np.zeros(100, dtype=np.complex64)
    P.sv_copy_to_host(st.s, part, 900, 100)
    np.testing.assert_array_equal(part, data[900:1000])
    with pytest.raises(P.SVError):
        P.sv_copy_to_host(st.s, np.zeros(200, dtype=np.complex64), 900, 200)
    st.close()


# ----------------------------------------------------- k = 5 tile shapes

TILE_MODES = ("SV_TILE_NARROW", "SV_TILE_WIDE", "SV_TILE_SPREAD", "SV_TILE_AUTO")


def _tile_mode_states(P, dt, n, layer, mats, targets):
    outs = {}
    for name in TILE_MODES:
        h = P.Handle()
        h.set_tile_mode(getattr(P, name))
        st = P.State(h, n, dt)
        st.run(layer)
        for m in mats:
            st.apply_matrix(m, targets)
        outs[name] = st.to_numpy()
        st.close()
        h.close()
    return outs


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("targets", [(0, 1, 2, 3, 4), (3, 7, 9, 12, 15), (11, 12, 13, 14, 15), (2, 6, 10, 13, 16),
                                     (14, 1, 8, 5, 12)])
def test_k5_tile_shapes_agree_bitwise(P, dt, targets):
    # the narrow (256 threads), wide (512 threads, 64 KiB) and spread (1 KiB
    # runs, low targets swapped for free bits from 12 up, strided tile
    # order) variants of the k = 5 sweep do the same arithmetic per group,
    # so the states agree bit for bit, and match the oracle; AUTO (which
    # times every variant on the first sweeps) gives the same bits too
    n = 17
    rng = np.random.default_rng(sum(targets))
    mats = [W.haar_unitary(5, rng) for _ in range(6)]
    layer = W.brickwork(n, 1, 9)  # every amplitude non-zero
    ref = oracle.run(n, layer)
    for m in mats:
        oracle.apply(ref, m, targets)
    outs = _tile_mode_states(P, dt, n, layer, mats, targets)
    if dt == "c128":
        assert np.max(np.abs(outs["SV_TILE_NARROW"] - ref)) <= 1e-10
    else:
        assert oracle.fidelity(ref, outs["SV_TILE_NARROW"].astype(np.complex128)) >= C64_FID
    for name in TILE_MODES[1:]:
        np.testing.assert_array_equal(outs["SV_TILE_NARROW"], outs[name], err_msg=name)


@pytest.mark.parametrize("dt,n", [("c64", 13), ("c128", 12), ("c64", 16)])
def test_k5_spread_on_small_states(P, dt, n):
    # at 13 (complex64) and 12 (complex128) qubits there are too few free
    # index bits from 12 up to stand in for the low targets, and the spread
    # mode runs the narrow layout; at 16 it swaps four of them for bits
    # 12-15; the bits agree with the other modes either way
    targets = (0, 2, 4, 6, 8)
    rng = np.random.default_rng(n)
    mats = [W.haar_unitary(5, rng) for _ in range(3)]
    layer = W.brickwork(n, 1, 4)
    ref = oracle.run(n, layer)
    for m in mats:
        oracle.apply(ref, m, targets)
    outs = _tile_mode_states(P, dt, n, layer, mats, targets)
    if dt == "c128":
        assert np.max(np.abs(outs["SV_TILE_SPREAD"] - ref)) <= 1e-10
    else:
        assert oracle.fidelity(ref, outs["SV_TILE_SPREAD"].astype(np.complex128)) >= C64_FID
    for name in TILE_MODES[1:]:
        np.testing.assert_array_equal(outs["SV_TILE_NARROW"], outs[name], err_msg=name)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_k5_autotuner_trials_give_the_same_bits(P, dt):
    # enough sweeps on two target sets for the AUTO handle to pass its 64
    # untimed sweeps, time every variant three times per set and settle:
    # whichever variants ran, the state is bit for bit the NARROW one
    n = 17
    sets = [(0, 1, 2, 3, 4), (13, 2, 9, 15, 6)]
    rng = np.random.default_rng(5)
    mats = [W.haar_unitary(5, rng) for _ in range(4)]
    layer = W.brickwork(n, 1, 3)
    outs = {}
    for mode in (P.SV_TILE_NARROW, P.SV_TILE_AUTO):
        h = P.Handle()
        h.set_tile_mode(mode)
        st = P.State(h, n, dt)
        st.run(layer)
        for i in range(64 + 2 * 9 + 8):
            st.apply_matrix(mats[i % 4], sets[(i // 4) % 2])
        outs[mode] = st.to_numpy()
        st.close()
        h.close()
    np.testing.assert_array_equal(outs[P.SV_TILE_NARROW], outs[P.SV_TILE_AUTO])
    assert abs(np.linalg.norm(outs[P.SV_TILE_AUTO].astype(np.complex128)) - 1.0) < 1e-4


def test_tile_mode_rejects_unknown(P, H):
    with pytest.raises(P.SVError):
        H.set_tile_mode(4)
    with pytest.raises(P.SVError):
        H.set_tile_mode(-1)
    H.set_tile_mode(P.SV_TILE_AUTO)


# ------------------------------------------------------ recorded programs

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [6, 12, 16])
def test_graph_replays_match_eager_and_oracle(P, H, dt, n):
    # a fused program recorded into a HIP graph, replayed three times with
    # the program's own eager work (state reset, an eager sweep, a read-back)
    # between replays: every replay equals the eager fused run bit for bit
    gates = W.brickwork(n, 6, 70 + n)
    ref = oracle.run(n, gates)
    st = _state(P, H, n, dt)
    st.run(gates, max_fused_qubits=5)
    eager = st.to_numpy()
    if dt == "c128":
        assert np.max(np.abs(eager - ref)) <= 1e-10
    else:
        assert oracle.fidelity(ref, eager.astype(np.complex128)) >= C64_FID
    g = P.Graph(st, gates, 5)
    for rep in range(3):
        P.sv_set_basis_state(st.s, 0)
        g.launch()
        got = st.to_numpy()
        np.testing.assert_array_equal(got, eager, err_msg=f"replay {rep}")
        # eager work between replays on the same handle
        st.apply_matrix(np.array([[0, 1], [1, 0]]), (n - 1,))
        P.sv_sync(H.h)
    g.close()
    st.close()
