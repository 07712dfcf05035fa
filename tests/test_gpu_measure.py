"""GPU parity of the Pauli rotation, measurement (probabilities, collapse,
Z-basis and batched measurement) and dense-observable expectation, through
the C ABI, against the oracle on the same seeded inputs.

Tolerances: complex128 amplitudes <= 1e-12 (one or two products per
amplitude); complex64 amplitudes <= 1e-6 of the largest (FP32 products).
Probabilities and expectations are FP64 sums on both sides over the same
amplitudes (the complex64 state upcast exactly for the oracle), so they
agree to 1e-12 of the total, the summation order aside.  An outcome chosen
by comparing randnum * total with running sums is checked by the interval
rule: the oracle's running sums must bracket it within 1e-12 of the total."""
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


def _state(P, H, n, dt, rng, scale=1.0):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v *= scale / np.linalg.norm(v)
    st = P.State(H, n, dt)
    host = v.astype(np.complex64 if dt == "c64" else np.complex128)
    P.sv_copy_from_host(st.s, host, 0)
    return st, host.astype(np.complex128)


def _check_amps(dt, got, ref):
    if dt == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        assert np.max(np.abs(got.astype(np.complex128) - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [5, 13, 16])
@pytest.mark.parametrize("seed", range(5))
def test_pauli_rotation_matches_oracle(P, H, dt, n, seed):
    # strings of 1-5 factors over I/X/Y/Z (seed 0: Z only, a phase sweep),
    # up to 2 controls with values
    rng = np.random.default_rng(77 * n + seed)
    qs = [int(q) for q in rng.permutation(n)]
    k = int(rng.integers(1, 6))
    ops = "Z" * k if seed == 0 else "".join("IXYZ"[int(rng.integers(0, 4))] for _ in range(k))
    term = list(zip(qs[:k], ops))
    nc = int(rng.integers(0, 3))
    controls = qs[k:k + nc]
    cvals = [int(v) for v in rng.integers(0, 2, nc)]
    theta = float(rng.uniform(-4, 4))
    st, ref = _state(P, H, n, dt, rng)
    P.sv_apply_pauli_rotation(st.s, theta, term, controls, cvals)
    oracle.apply_pauli_rotation(ref, theta, term, controls, cvals)
    _check_amps(dt, st.to_numpy(), ref)
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n,m", [(1, 1), (2, 2), (3, 2), (4, 1), (9, 4), (11, 4), (14, 10), (20, 3)])
def test_measure_probabilities_match_oracle(P, H, dt, n, m):
    rng = np.random.default_rng(n * 10 + m)
    qubits = [int(q) for q in rng.permutation(n)[:m]]
    st, ref = _state(P, H, n, dt, rng, scale=1.3)
    got = P.sv_measure_probabilities(st.s, qubits)
    want = oracle.measure_probs(ref, qubits)
    tot = want.sum()
    assert np.max(np.abs(got - want)) <= 1e-12 * tot
    pe, po = P.sv_zbasis_probabilities(st.s, qubits)
    we, wo = oracle.zbasis_probs(ref, qubits)
    assert abs(pe - we) <= 1e-12 * tot and abs(po - wo) <= 1e-12 * tot
    # bitwise reproducible
    np.testing.assert_array_equal(got, P.sv_measure_probabilities(st.s, qubits))
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [6, 15])
def test_collapse_matches_oracle(P, H, dt, n):
    rng = np.random.default_rng(n)
    qubits = [int(q) for q in rng.permutation(n)[:3]]
    for outcome in (0, 5, 7):
        st, ref = _state(P, H, n, dt, rng)
        p = oracle.measure_probs(ref, qubits)
        P.sv_collapse(st.s, qubits, outcome, p[outcome])
        oracle.collapse(ref, qubits, outcome=outcome, norm=p[outcome])
        _check_amps(dt, st.to_numpy(), ref)
        st.close()
    for parity in (0, 1):
        st, ref = _state(P, H, n, dt, rng)
        pe, po = oracle.zbasis_probs(ref, qubits)
        norm = pe if parity == 0 else po
        P.sv_collapse_zbasis(st.s, qubits, parity, norm)
        oracle.collapse(ref, qubits, norm=norm, parity=parity)
        _check_amps(dt, st.to_numpy(), ref)
        st.close()


def _bracket(c, b, r, tot):
    lo = c[b - 1] if b > 0 else 0.0
    return lo - 1e-12 * tot <= r < c[b] + 1e-12 * tot


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("seed", range(4))
def test_measure_zbasis_and_batch_measure(P, H, dt, seed):
    rng = np.random.default_rng(500 + seed)
    n = 12
    qubits = [int(q) for q in rng.permutation(n)[:4]]
    for r in (0.0, 0.3, float(rng.uniform()), 0.999999):
        st, ref = _state(P, H, n, dt, rng)
        p = oracle.measure_probs(ref, qubits)
        c = np.cumsum(p)
        b = P.sv_batch_measure(st.s, qubits, r, collapse=True)
        assert p[b] > 0 and _bracket(c, b, r * c[-1], c[-1])
        oracle.collapse(ref, qubits, outcome=b, norm=p[b])
        _check_amps(dt, st.to_numpy(), ref)
        st.close()
        st, ref = _state(P, H, n, dt, rng)
        pe, po = oracle.zbasis_probs(ref, qubits)
        par = P.sv_measure_zbasis(st.s, qubits, r, collapse=True)
        assert _bracket(np.array([pe, pe + po]), par, r * (pe + po), pe + po)
        oracle.collapse(ref, qubits, norm=pe if par == 0 else po, parity=par)
        _check_amps(dt, st.to_numpy(), ref)
        st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_measurement_closed_forms(P, H, dt):
    # GHZ: qubits 0 and n-1 always agree (parity even), batched outcome 0 or 3
    # by randnum; the collapsed state is |0..0> or |1..1>
    n = 10
    st = P.State(H, n, dt)
    st.run(W.ghz(n))
    assert P.sv_measure_zbasis(st.s, [0, n - 1], 0.9, collapse=False) == 0
    assert P.sv_batch_measure(st.s, [0, n - 1], 0.49, collapse=False) == 0
    assert P.sv_batch_measure(st.s, [0, n - 1], 0.51, collapse=True) == 3
    v = st.to_numpy()
    assert abs(abs(v[-1]) - 1.0) < 1e-6 and np.sum(np.abs(v[:-1])) < 1e-6
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_expect_matrix_matches_oracle(P, H, dt, k):
    rng = np.random.default_rng(40 + k)
    for n in (k, 11, 17):
        if n < k:
            continue
        targets = [int(q) for q in rng.permutation(n)[:k]]
        m = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
        st, ref = _state(P, H, n, dt, rng, scale=0.7)
        got = P.sv_expect_matrix(st.s, m, targets)
        want = oracle.expect_matrix(ref, m, targets)
        assert abs(got - want) <= 1e-11 * max(1.0, abs(want))
        st.close()


def test_bad_arguments(P, H):
    rng = np.random.default_rng(3)
    st, ref = _state(P, H, 6, "c128", rng)
    for call in (lambda: P.sv_measure_probabilities(st.s, []),
                 lambda: P.sv_measure_probabilities(st.s, [1, 1]),
                 lambda: P.sv_measure_probabilities(st.s, [6]),
                 lambda: P.sv_collapse(st.s, [0, 1], 4, 1.0),
                 lambda: P.sv_collapse(st.s, [0], 0, 0.0),
                 lambda: P.sv_collapse_zbasis(st.s, [0], 2, 1.0),
                 lambda: P.sv_measure_zbasis(st.s, [0], 1.0),
                 lambda: P.sv_batch_measure(st.s, [0], -0.1),
                 lambda: P.sv_expect_matrix(st.s, np.eye(64), list(range(6))),
                 lambda: P.sv_apply_pauli_rotation(st.s, 0.1, [(0, "Q")]),
                 lambda: P.sv_apply_pauli_rotation(st.s, 0.1, [(0, "X")], [0]),
                 lambda: P.sv_apply_pauli_rotation(st.s, float("nan"), [(0, "X")])):
        with pytest.raises(P.SVError):
            call()
    np.testing.assert_array_equal(st.to_numpy(), ref)
    st.close()
