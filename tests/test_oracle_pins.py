"""Pins for the CPU oracle: brute-force Kronecker operators, closed forms,
invariants and hand-worked tables.  Each test is chosen so that a plausible
mistake in the oracle (a wrong sign, a swapped index, a transposed matrix, a
dropped control, a wrong CDF rule) fails at least one of them."""
import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import workloads as W
from tests.kron_ref import PAULI, embed, pauli_operator

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- gate table

def _rz(a):
    return expm(-0.5j * a * PAULI["Z"])


def _ry(a):
    return expm(-0.5j * a * PAULI["Y"])


@pytest.mark.parametrize("seed", range(5))
def test_u3_is_euler_rotation(seed):
    # U3(theta, phi, lambda) = e^{i(phi+lambda)/2} RZ(phi) RY(theta) RZ(lambda)
    th, ph, la = np.random.default_rng(seed).uniform(0, 2 * math.pi, 3)
    m, k, nc = oracle.gate_matrix("u3", (th, ph, la))
    ref = np.exp(0.5j * (ph + la)) * _rz(ph) @ _ry(th) @ _rz(la)
    assert (k, nc) == (1, 0)
    np.testing.assert_allclose(m, ref, atol=1e-14)


def test_named_gate_identities():
    h = oracle.gate_matrix("h")[0]
    x = oracle.gate_matrix("x")[0]
    np.testing.assert_allclose(h, (PAULI["X"] + PAULI["Z"]) / math.sqrt(2), atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("u3", (math.pi / 2, 0, math.pi))[0], h, atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("u3", (math.pi, 0, math.pi))[0], x, atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("u3", (0.7, 0, 0))[0], _ry(0.7), atol=1e-15)
    for name in "xyz":
        np.testing.assert_array_equal(oracle.gate_matrix(name)[0], PAULI[name.upper()])
    assert oracle.gate_matrix("cx")[1:] == (1, 1)
    assert oracle.gate_matrix("cz")[1:] == (1, 1)
    m, k, nc = oracle.gate_matrix("cp", (0.3,))
    assert (k, nc) == (1, 1)
    np.testing.assert_allclose(m, np.diag([1, np.exp(0.3j)]), atol=1e-15)
    sw, k, nc = oracle.gate_matrix("swap")
    assert (k, nc) == (2, 0)
    # SWAP maps |b1 b0> to |b0 b1>: basis 1 <-> 2
    np.testing.assert_array_equal(sw, np.eye(4)[[0, 2, 1, 3]])


@pytest.mark.parametrize("name,params", [("u3", (0.3, 1.1, 2.5)), ("cp", (0.9,)), ("h", ()),
                                         ("y", ()), ("swap", ())])
def test_adjoint_is_inverse(name, params):
    m = oracle.gate_matrix(name, params)[0]
    md = oracle.gate_matrix(name + "_dg", params)[0]
    np.testing.assert_allclose(md @ m, np.eye(m.shape[0]), atol=1e-14)
    np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-14)


def test_unknown_gate_rejected():
    with pytest.raises(ValueError):
        oracle.gate_matrix("foo")
    with pytest.raises(ValueError):
        oracle.gate_matrix("u3", (1.0,))


# ---------------------------------------------------------- gate application

@pytest.mark.parametrize("seed", range(12))
def test_apply_matches_kronecker(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 9))
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    for (t, c, cv, m) in W.random_dense_circuit(n, 6, min(5, n), seed):
        ref = embed(m, t, n, c, cv) @ psi
        oracle.apply(psi, m, t, c, cv)
        np.testing.assert_allclose(psi, ref, atol=1e-13, rtol=0)


def test_apply_controls_default_to_one():
    n = 4
    rng = np.random.default_rng(7)
    psi = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    m = W.haar_unitary(1, rng)
    ref = embed(m, (2,), n, (0, 3), (1, 1)) @ psi
    oracle.apply(psi, m, (2,), (0, 3))
    np.testing.assert_allclose(psi, ref, atol=1e-14)


def test_apply_non_unitary_matrix_acts_linearly():
    # a non-unitary matrix exposes a transposed or conjugated operand
    n = 3
    m = np.arange(16, dtype=np.float64).reshape(4, 4) + 1j * np.arange(16).reshape(4, 4)[::-1]
    psi = np.arange(8, dtype=np.complex128) + 0.5j
    ref = embed(m, (2, 0), n) @ psi
    oracle.apply(psi, m, (2, 0))
    np.testing.assert_allclose(psi, ref, atol=1e-12)


def test_apply_rejects_bad_arguments():
    psi = oracle.basis_state(3)
    with pytest.raises(ValueError):
        oracle.apply(psi, np.eye(2), (3,))
    with pytest.raises(ValueError):
        oracle.apply(psi, np.eye(4), (1, 1))
    with pytest.raises(ValueError):
        oracle.apply(psi, np.eye(2), (1,), (1,))


def _ref_gate_full(name, qs, params, n):
    """Full operator of a workload gate from definitions independent of the
    oracle's table: U3 as an Euler rotation, controlled gates as Pauli /
    phase matrices on the second qubit."""
    if name == "u3":
        th, ph, la = params
        m = np.exp(0.5j * (ph + la)) * _rz(ph) @ _ry(th) @ _rz(la)
        return embed(m, qs, n)
    if name == "h":
        return embed((PAULI["X"] + PAULI["Z"]) / math.sqrt(2), qs, n)
    if name in ("x", "y", "z"):
        return embed(PAULI[name.upper()], qs, n)
    if name == "cx":
        return embed(PAULI["X"], qs[1:], n, qs[:1])
    if name == "cz":
        return embed(PAULI["Z"], qs[1:], n, qs[:1])
    if name == "cp":
        return embed(np.diag([1, np.exp(1j * params[0])]), qs[1:], n, qs[:1])
    if name == "swap":
        a, b = qs
        return embed(PAULI["X"], (a,), n, (b,)) @ embed(PAULI["X"], (b,), n, (a,)) @ embed(PAULI["X"], (a,), n, (b,))
    raise ValueError(name)


@pytest.mark.parametrize("n,depth,seed", [(5, 4, 0), (6, 3, 1), (7, 2, 2)])
def test_brickwork_matches_kronecker_product(n, depth, seed):
    gates = W.brickwork(n, depth, seed)
    u = np.eye(1 << n, dtype=np.complex128)
    for name, qs, params in gates:
        u = _ref_gate_full(name, qs, params, n) @ u
    np.testing.assert_allclose(u @ u.conj().T, np.eye(1 << n), atol=1e-12)
    psi = oracle.run(n, gates)
    np.testing.assert_allclose(psi, u[:, 0], atol=1e-13)


@pytest.mark.parametrize("seed", range(3))
def test_random_cx_cp_matches_kronecker_product(seed):
    n = 6
    gates = W.random_cx_cp(n, 3, 5 + seed)
    x = W.random_basis_state(n, 3 + seed)
    ref = oracle.basis_state(n, x)
    for name, qs, params in gates:
        ref = _ref_gate_full(name, qs, params, n) @ ref
    np.testing.assert_allclose(oracle.run(n, gates, basis=x), ref, atol=1e-13)


def test_qft_and_swap_match_kronecker_product():
    n = 5
    x = 22
    ref = oracle.basis_state(n, x)
    for name, qs, params in W.qft(n):
        ref = _ref_gate_full(name, qs, params, n) @ ref
    np.testing.assert_allclose(oracle.run(n, W.qft(n), basis=x), ref, atol=1e-13)


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_ghz(n):
    psi = oracle.run(n, W.ghz(n))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, ref, atol=1e-15)
    if n >= 2:
        assert oracle.expect_pauli(psi, [(0, "Z"), (n - 1, "Z")]) == pytest.approx(1.0, abs=1e-14)
        assert oracle.expect_pauli(psi, [(0, "Z")]) == pytest.approx(0.0, abs=1e-14)
        assert oracle.expect_pauli(psi, [(q, "X") for q in range(n)]) == pytest.approx(1.0, abs=1e-14)


def test_ghz_nonadjacent_order():
    n = 7
    order = [3, 6, 0, 5, 1, 4, 2]
    psi = oracle.run(n, W.ghz(n, order))
    assert abs(psi[0]) ** 2 == pytest.approx(0.5, abs=1e-15)
    assert abs(psi[-1]) ** 2 == pytest.approx(0.5, abs=1e-15)
    assert oracle.norm(psi) == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("n,x", [(3, 5), (5, 19), (8, 201)])
def test_qft_closed_form(n, x):
    psi = oracle.run(n, W.qft(n), basis=x)
    y = np.arange(1 << n)
    ref = np.exp(2j * math.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    np.testing.assert_allclose(psi, ref, atol=1e-13)
    # numpy's inverse FFT of a basis vector is the same transform
    e = np.zeros(1 << n)
    e[x] = 1
    np.testing.assert_allclose(psi, np.fft.ifft(e) * math.sqrt(1 << n), atol=1e-13)


def test_qft_gate_count_matches_paper():
    g = json.load(open(os.path.join(GOLD, "paper_gate_counts.json")))["qft"]
    assert len(W.qft(g["n"])) == g["gates"]


def test_product_state_closed_form_and_single_qubit_expectations():
    n = 6
    gates = W.brickwork(n, 1, 11)
    psi = oracle.run(n, gates)
    ang = np.random.default_rng(11).uniform(0, 2 * math.pi, size=(1, n, 3))[0]
    # amp(i) = prod_j a_j(b_j) * (-1)^{#CZ pairs with both bits set}
    a0 = np.cos(ang[:, 0] / 2)
    a1 = np.exp(1j * ang[:, 1]) * np.sin(ang[:, 0] / 2)
    ref = np.ones(1 << n, dtype=np.complex128)
    for i in range(1 << n):
        for j in range(n):
            ref[i] *= a1[j] if (i >> j) & 1 else a0[j]
        for j in range(0, n - 1, 2):
            if (i >> j) & 1 and (i >> (j + 1)) & 1:
                ref[i] *= -1
    np.testing.assert_allclose(psi, ref, atol=1e-14)
    for j in range(n):
        assert oracle.expect_pauli(psi, [(j, "Z")]) == pytest.approx(math.cos(ang[j, 0]), abs=1e-13)
    # without the CZ layer: <X_j> = sin th cos ph, <Y_j> = sin th sin ph
    psi1 = oracle.run(n, [g for g in gates if g.name == "u3"])
    for j in range(n):
        th, ph = ang[j, 0], ang[j, 1]
        assert oracle.expect_pauli(psi1, [(j, "X")]) == pytest.approx(math.sin(th) * math.cos(ph), abs=1e-13)
        assert oracle.expect_pauli(psi1, [(j, "Y")]) == pytest.approx(math.sin(th) * math.sin(ph), abs=1e-13)


def test_cluster_state_stabilisers():
    n = 7
    psi = oracle.run(n, W.cluster_1d(n))
    for i in range(n):
        term = [(i, "X")] + ([(i - 1, "Z")] if i > 0 else []) + ([(i + 1, "Z")] if i < n - 1 else [])
        assert oracle.expect_pauli(psi, term) == pytest.approx(1.0, abs=1e-13)
    # Y_i = i X_i Z_i: <Z_{i-1} Y_i Z_{i+1}> = 0 and <X_i> = 0 for inner i
    assert oracle.expect_pauli(psi, [(2, "Z"), (3, "Y"), (4, "Z")]) == pytest.approx(0.0, abs=1e-13)
    assert oracle.expect_pauli(psi, [(3, "X")]) == pytest.approx(0.0, abs=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_pauli_expectation_matches_kronecker(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 7))
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    for term in W.random_pauli_terms(n, 5, rng):
        p = pauli_operator(term, n)
        ref = np.vdot(psi, p @ psi) / np.vdot(psi, psi)
        re, im, nrm = oracle.expect_pauli_full(psi, term)
        assert re == pytest.approx(ref.real, abs=1e-13)
        assert im == pytest.approx(0.0, abs=1e-13)
        assert nrm == pytest.approx(np.vdot(psi, psi).real, rel=1e-14)


def test_mirror_circuit_returns_to_start():
    n = 8
    gates = W.random_cx_cp(n, 4, 2)
    x = W.random_basis_state(n, 9)
    psi = oracle.run(n, gates + W.inverse(gates), basis=x)
    assert abs(psi[x]) == pytest.approx(1.0, abs=1e-13)
    assert oracle.norm(psi) == pytest.approx(1.0, abs=1e-13)


# ------------------------------------------------------------------- norm

def test_norm_closed_form():
    # psi_i = (i+1) + 0j: sum = N(N+1)(2N+1)/6, exact in FP64 for these sizes
    for n in (1, 4, 10, 16):
        N = 1 << n
        psi = np.arange(1, N + 1, dtype=np.float64).astype(np.complex128)
        assert oracle.norm(psi) == N * (N + 1) * (2 * N + 1) // 6
    # compensation: 1 followed by many tiny values
    psi = np.full(1 << 12, 1e-9, dtype=np.complex128)
    psi[0] = 1.0
    assert oracle.norm(psi) == pytest.approx(1.0 + (4095) * 1e-18, rel=1e-16)


@pytest.mark.parametrize("seed", range(3))
def test_unitary_circuits_preserve_norm(seed):
    psi = oracle.run(10, W.brickwork(10, 8, seed))
    assert oracle.norm(psi) == pytest.approx(1.0, abs=1e-12)


# --------------------------------------------------------------- sampling

def test_sampling_hand_table():
    g = json.load(open(os.path.join(GOLD, "sampling_table.json")))
    psi = np.array(g["psi_re"]) + 1j * np.array(g["psi_im"])
    u = np.array(g["uniforms"])
    assert list(oracle.sample(psi, u)) == g["expected"]
    assert list(oracle.sample(psi, u, bit_ordering=[1])) == g["bit_ordering_[1]"]
    assert list(oracle.sample(psi, u, bit_ordering=[1, 0])) == g["bit_ordering_[1,0]"]


def test_sampling_exact_ties_follow_upper_bound_rule():
    g = json.load(open(os.path.join(GOLD, "sampling_ties.json")))
    psi = np.array(g["psi_re"], dtype=np.complex128)
    assert list(oracle.sample(psi, g["uniforms"])) == g["expected"]


def test_sampling_never_returns_zero_probability_and_keeps_order():
    psi = np.zeros(16, dtype=np.complex128)
    psi[[3, 9, 10]] = [0.6, 0.0 + 0.64j, math.sqrt(1 - 0.36 - 0.4096)]
    u = np.random.default_rng(0).random(5000)
    out = oracle.sample(psi, u)
    assert set(out.tolist()) <= {3, 9, 10}
    # input order: each output is the inverse-CDF of its own uniform
    cdf = np.cumsum(np.abs(psi) ** 2)
    for ui, oi in zip(u[:200], out[:200]):
        assert oi == np.searchsorted(cdf, ui * cdf[-1], side="right")


def test_sampling_chi_square():
    from scipy.stats import chisquare
    n = 5
    psi = oracle.run(n, W.brickwork(n, 6, 3))
    p = np.abs(psi) ** 2
    u = W.uniforms(200000, 17)
    out = oracle.sample(psi, u)
    counts = np.bincount(out.astype(np.int64), minlength=1 << n)
    stat, pval = chisquare(counts, p * len(u) / p.sum())
    assert pval > 1e-3


def test_sampling_marginal_bit_ordering():
    n = 4
    psi = oracle.run(n, W.brickwork(n, 3, 4))
    u = W.uniforms(3000, 5)
    full = oracle.sample(psi, u)
    sub = oracle.sample(psi, u, bit_ordering=[3, 1])
    np.testing.assert_array_equal(sub, ((full >> 3) & 1) | (((full >> 1) & 1) << 1))


def test_sampling_rejects_out_of_range_uniform():
    with pytest.raises(ValueError):
        oracle.sample(oracle.basis_state(2), [1.0])
    with pytest.raises(ValueError):
        oracle.sample(oracle.basis_state(2), [float("nan")])


def test_fidelity_helper():
    a = np.array([1, 1j]) / math.sqrt(2)
    assert oracle.fidelity(a, a * np.exp(0.3j)) == pytest.approx(1.0, abs=1e-15)
    assert oracle.fidelity(a, np.array([1, -1j])) == pytest.approx(0.0, abs=1e-15)


# ------------------------------------------- generalized permutation gates

def _rand_state(n, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("case", ["x", "y", "z", "cz", "cx", "swap", "cp"])
def test_gperm_named_gates_match_pauli_operators(case):
    # each gate written by hand as (perm, diag) in the matrix-index
    # convention (bit a of the row index = state of targets[a]), against
    # its full operator built from Pauli matrices by Kronecker products
    n, rng = 4, np.random.default_rng(3)
    cp = 0.7
    table = {
        "x": ([1, 0], [1, 1], (2,), embed(PAULI["X"], (2,), n)),
        "y": ([1, 0], [-1j, 1j], (1,), embed(PAULI["Y"], (1,), n)),
        "z": (None, [1, -1], (3,), embed(PAULI["Z"], (3,), n)),
        # targets (a, b) = (0, 3): row r = a + 2 b
        "cz": (None, [1, 1, 1, -1], (0, 3), embed(PAULI["Z"], (3,), n, (0,))),
        # control a = qubit 1 (matrix bit 0) flips b = qubit 2 (bit 1): rows 1 and 3 trade
        "cx": ([0, 3, 2, 1], [1, 1, 1, 1], (1, 2), embed(PAULI["X"], (2,), n, (1,))),
        "swap": ([0, 2, 1, 3], [1, 1, 1, 1], (0, 2),
                 embed(PAULI["X"], (0,), n, (2,)) @ embed(PAULI["X"], (2,), n, (0,)) @ embed(PAULI["X"], (0,), n, (2,))),
        "cp": (None, [1, 1, 1, np.exp(1j * cp)], (3, 1), embed(np.diag([1, np.exp(1j * cp)]), (1,), n, (3,))),
    }
    perm, diag, targets, full = table[case]
    psi = _rand_state(n, rng)
    ref = full @ psi
    oracle.apply_gperm(psi, perm, diag, targets)
    np.testing.assert_allclose(psi, ref, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_gperm_matches_kronecker_operator(seed):
    # random permutation, arbitrary (non-unitary) complex diagonal, random
    # targets and controls with values, against the full operator of the
    # dense G = D P (row r: diag[r] in column perm[r]) embedded by Kronecker
    # products; the adjoint against the conjugate transpose
    rng = np.random.default_rng(seed)
    n = 6
    k = int(rng.integers(1, 5))
    nc = int(rng.integers(0, 3))
    qs = [int(q) for q in rng.permutation(n)]
    targets, controls = tuple(qs[:k]), tuple(qs[k:k + nc])
    cvals = [int(v) for v in rng.integers(0, 2, nc)]
    perm = None if seed % 3 == 0 else [int(p) for p in rng.permutation(1 << k)]
    diag = rng.normal(size=1 << k) + 1j * rng.normal(size=1 << k)
    g = np.zeros((1 << k, 1 << k), dtype=np.complex128)
    for r in range(1 << k):
        g[r, r if perm is None else perm[r]] = diag[r]
    full = embed(g, targets, n, controls, cvals)
    psi = _rand_state(n, rng)
    a = psi.copy()
    oracle.apply_gperm(a, perm, diag, targets, controls, cvals)
    np.testing.assert_allclose(a, full @ psi, atol=1e-12)
    b = psi.copy()
    oracle.apply_gperm(b, perm, diag, targets, controls, cvals, adjoint=True)
    np.testing.assert_allclose(b, full.conj().T @ psi, atol=1e-12)
    # and the dense form of the oracle agrees with the dense apply
    np.testing.assert_array_equal(oracle.gperm_matrix(perm, diag), g)


def test_gperm_unitary_round_trip_and_rejects_bad_input():
    rng = np.random.default_rng(9)
    n, targets = 5, (4, 0, 2)
    perm = [int(p) for p in rng.permutation(8)]
    diag = np.exp(1j * rng.uniform(0, 2 * np.pi, 8))
    psi = _rand_state(n, rng)
    a = psi.copy()
    oracle.apply_gperm(a, perm, diag, targets)
    oracle.apply_gperm(a, perm, diag, targets, adjoint=True)
    np.testing.assert_allclose(a, psi, atol=1e-13)
    with pytest.raises(ValueError):
        oracle.apply_gperm(psi, [0, 0, 1, 2, 3, 4, 5, 6], diag, targets)
    with pytest.raises(ValueError):
        oracle.apply_gperm(psi, None, diag[:4], targets)
    with pytest.raises(ValueError):
        oracle.apply_gperm(psi, None, diag, (1, 1, 2))


# --------------------------------------------------------- Pauli rotation

@pytest.mark.parametrize("seed", range(6))
def test_pauli_rotation_matches_matrix_exponential(seed):
    # exp(i theta P) against scipy's expm of the Kronecker-built Pauli string,
    # with controls embedded by Kronecker projectors
    rng = np.random.default_rng(seed)
    n = 5
    qs = [int(q) for q in rng.permutation(n)]
    k = int(rng.integers(1, 4))
    term = [(qs[a], "IXYZ"[int(rng.integers(0, 4))]) for a in range(k)]
    nc = int(rng.integers(0, 2))
    controls = tuple(qs[k:k + nc])
    cvals = [int(v) for v in rng.integers(0, 2, nc)]
    theta = float(rng.uniform(-3, 3))
    psi = _rand_state(n, rng)
    if nc:
        local = expm(1j * theta * pauli_operator([(a, o) for a, (_, o) in enumerate(term)], k))
        full = embed(local, tuple(q for q, _ in term), n, controls, cvals)
    else:
        full = expm(1j * theta * pauli_operator(term, n))
    ref = full @ psi
    oracle.apply_pauli_rotation(psi, theta, term, controls, cvals if nc else None)
    np.testing.assert_allclose(psi, ref, atol=1e-12)


def test_pauli_rotation_closed_forms():
    # exp(i t Z)|0> = e^{it}|0>; exp(i t X)|0> = cos t|0> + i sin t|1>;
    # exp(i t Y)|0> = cos t|0> - sin t|1>
    t = 0.3
    for op, a1 in (("Z", 0.0), ("X", 1j * math.sin(t)), ("Y", -math.sin(t))):
        psi = oracle.basis_state(1)
        oracle.apply_pauli_rotation(psi, t, [(0, op)])
        a0 = np.exp(1j * t) if op == "Z" else math.cos(t)
        np.testing.assert_allclose(psi, [a0, a1], atol=1e-15)


# -------------------------------------------------------------- measurement

def test_measure_probs_ghz_product_and_ordering():
    n = 4
    ghz = oracle.run(n, W.ghz(n))
    np.testing.assert_allclose(oracle.measure_probs(ghz, [0, 2]), [0.5, 0, 0, 0.5], atol=1e-15)
    # one U3 layer: P(q = 1) = sin^2(theta_q / 2), independent across qubits
    th = [0.4, 1.1, 2.0]
    psi = oracle.run(3, [W.Gate("u3", (q,), (th[q], 0.3, 0.2)) for q in range(3)])
    p = oracle.measure_probs(psi, [2, 0])
    s2 = [math.sin(t / 2) ** 2 for t in th]
    np.testing.assert_allclose(p, [(1 - s2[2]) * (1 - s2[0]), s2[2] * (1 - s2[0]), (1 - s2[2]) * s2[0], s2[2] * s2[0]],
                               atol=1e-15)
    # bit a of the outcome is qubits[a]: |100> measured on (2, 0) is outcome 1
    np.testing.assert_allclose(oracle.measure_probs(oracle.basis_state(3, 4), [2, 0]), [0, 1, 0, 0])
    rng = np.random.default_rng(2)
    v = _rand_state(6, rng) * 1.7
    assert abs(oracle.measure_probs(v, [5, 1, 3]).sum() - np.vdot(v, v).real) < 1e-13


def _projector(qubits, bits, n):
    # Kronecker product of |b><b| on the measured qubits
    ops = [np.eye(2)] * n
    for q, b in zip(qubits, bits):
        ops[q] = np.diag([1.0 - b, float(b)])
    full = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        full = np.kron(full, ops[q])
    return full


def test_collapse_matches_projectors():
    rng = np.random.default_rng(4)
    n = 5
    psi = _rand_state(n, rng)
    qubits = (3, 0, 4)
    p = oracle.measure_probs(psi, qubits)
    for b in (0, 5, 6):
        bits = [(b >> a) & 1 for a in range(3)]
        ref = _projector(qubits, bits, n) @ psi / math.sqrt(p[b])
        a = psi.copy()
        oracle.collapse(a, qubits, outcome=b, norm=p[b])
        np.testing.assert_allclose(a, ref, atol=1e-14)
        assert abs(np.vdot(a, a).real - 1.0) < 1e-13
    # parity collapse = (I + (-1)^par Z.Z.Z)/2 psi / sqrt(p_par)
    pe, po = oracle.zbasis_probs(psi, qubits)
    zzz = pauli_operator([(q, "Z") for q in qubits], n)
    for par, pp in ((0, pe), (1, po)):
        ref = 0.5 * (np.eye(1 << n) + (-1) ** par * zzz) @ psi / math.sqrt(pp)
        a = psi.copy()
        oracle.collapse(a, qubits, norm=pp, parity=par)
        np.testing.assert_allclose(a, ref, atol=1e-14)


def test_measurement_outcome_rules():
    # Z parity on GHZ is always even; on |+> the split is at randnum = 1/2
    ghz = oracle.run(4, W.ghz(4))
    for r in (0.0, 0.5, 0.999):
        assert oracle.measure_zbasis(ghz.copy(), [1, 3], r) == 0
    plus = oracle.run(1, [W.Gate("h", (0,), ())])
    assert oracle.measure_zbasis(plus.copy(), [0], 0.49) == 0
    assert oracle.measure_zbasis(plus.copy(), [0], 0.51) == 1
    # batched: probabilities (0.1, 0, 0.2, 0.7) -> upper-bound rule, never
    # the zero-probability outcome
    amp = np.sqrt(np.array([0.1, 0.0, 0.2, 0.7])).astype(np.complex128)
    for r, want in ((0.05, 0), (0.1, 2), (0.29, 2), (0.3, 3), (0.999, 3)):
        a = amp.copy()
        assert oracle.batch_measure(a, [0, 1], r) == want
        np.testing.assert_allclose(np.abs(a) ** 2, np.eye(4)[want], atol=1e-15)


# ----------------------------------------------- dense observable expectation

@pytest.mark.parametrize("seed", range(4))
def test_expect_matrix_matches_kronecker(seed):
    rng = np.random.default_rng(seed)
    n = 5
    k = int(rng.integers(1, 4))
    targets = tuple(int(q) for q in rng.permutation(n)[:k])
    m = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    psi = _rand_state(n, rng) * 0.8
    ref = np.vdot(psi, embed(m, targets, n) @ psi) / np.vdot(psi, psi)
    got = oracle.expect_matrix(psi, m, targets)
    assert abs(got - ref) < 1e-13
    # a Pauli product as a matrix equals the Pauli expectation
    term = [(targets[0], "Y")]
    assert abs(oracle.expect_matrix(psi, PAULI["Y"], targets[:1]) - oracle.expect_pauli(psi, term)) < 1e-14


# ---------------------------------------------- index bit swap and accessor

@pytest.mark.parametrize("seed", range(5))
def test_swap_index_bits_equals_swap_gates(seed):
    # exchanging bit pairs is a product of SWAP gates; with mask bits, of
    # SWAPs controlled on the mask values (Kronecker operators)
    rng = np.random.default_rng(seed)
    n = 6
    qs = [int(q) for q in rng.permutation(n)]
    npairs = int(rng.integers(1, 3))
    pairs = [(qs[2 * p], qs[2 * p + 1]) for p in range(npairs)]
    nm = int(rng.integers(0, n - 2 * npairs + 1))
    nm = min(nm, 2)
    mbits = qs[2 * npairs:2 * npairs + nm]
    mvals = [int(v) for v in rng.integers(0, 2, nm)]
    psi = _rand_state(n, rng)
    ref = psi.copy()
    swap = np.eye(4)[[0, 2, 1, 3]]
    for a, b in pairs:
        ref = embed(swap, (a, b), n, tuple(mbits), mvals if nm else None) @ ref
    oracle.swap_index_bits(psi, pairs, mbits, mvals)
    np.testing.assert_allclose(psi, ref, atol=1e-15)


def test_accessor_reorders_like_a_tensor_transpose():
    # with every bit listed, the reordered copy equals numpy's axis
    # permutation of the state viewed as a 2 x ... x 2 tensor; with mask
    # bits, a slice of it; set inverts get
    rng = np.random.default_rng(8)
    n = 5
    psi = _rand_state(n, rng)
    order = [3, 0, 4, 1, 2]
    # tensor axis t corresponds to qubit n - 1 - t (C order, qubit 0 last)
    t = psi.reshape([2] * n)
    # output bit a = state bit order[a]; output axis n-1-a <- state axis n-1-order[a]
    perm = [n - 1 - order[n - 1 - ax] for ax in range(n)]
    want = np.transpose(t, perm).reshape(-1)
    np.testing.assert_array_equal(oracle.accessor_get(psi, order), want)
    np.testing.assert_array_equal(oracle.accessor_get(psi, order, begin=5, end=19), want[5:19])
    sl = oracle.accessor_get(psi, [4, 0, 2], mask_bits=[1, 3], mask_values=[1, 0])
    idx = [(1 << 1) | (((k >> 0) & 1) << 4) | (((k >> 1) & 1) << 0) | (((k >> 2) & 1) << 2) for k in range(8)]
    np.testing.assert_array_equal(sl, psi[idx])
    phi = np.zeros_like(psi)
    oracle.accessor_set(phi, want, order)
    np.testing.assert_array_equal(phi, psi)
    with pytest.raises(ValueError):
        oracle.accessor_get(psi, [0, 1, 2])          # bits missing
    with pytest.raises(ValueError):
        oracle.swap_index_bits(psi, [(0, 1), (1, 2)])  # bit 1 twice
