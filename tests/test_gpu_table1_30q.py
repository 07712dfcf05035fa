"""The Table I operations at the size the benchmark times them: 30 qubits,
complex64 and complex128, on a product state (one U3 on every qubit), whose
amplitudes have a closed form, amp(y) = prod_j f_j(bit j of y) with
f_j(0) = cos(theta_j/2), f_j(1) = e^{i phi_j} sin(theta_j/2).  A host oracle
of a 30-qubit state is too slow for a test, so each operation is checked on
sampled outputs against the closed form of its result:
  - diagonal (k = 10, with and without a control) and permutation gates:
    diag[r(y)] times the closed-form amplitude at y with the target bits
    replaced by perm[r(y)];
  - Pauli rotation: cos(t) amp(y) + i sin(t) (P amp)(y);
  - outcome and parity probabilities: products of single-qubit
    probabilities; collapse: the closed form restricted and rescaled;
  - dense observable: <phi_T|M|phi_T> of the 3-qubit factor on the targets;
  - index bit swap and reordering accessor: amplitudes at permuted indices.
Tolerances: complex128 1e-12 relative per amplitude; complex64 2e-6
relative per amplitude (the state is rounded to FP32, then one or two FP32
products); probabilities and expectations 1e-12 (c128) / 2e-6 (c64)."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N = 30


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < (20 << 30):
        pytest.skip("needs 20 GiB of free device memory")
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


class Product:
    def __init__(self, seed):
        rng = np.random.default_rng(seed)
        self.th = rng.uniform(0.2, 2.9, N)
        self.ph = rng.uniform(0, 2 * np.pi, N)
        self.gates = [W.Gate("u3", (q,), (float(self.th[q]), float(self.ph[q]), 0.3)) for q in range(N)]
        self.f0 = np.cos(self.th / 2)
        self.f1 = np.exp(1j * self.ph) * np.sin(self.th / 2)

    def amp(self, y):
        v = 1.0 + 0.0j
        for j in range(N):
            v *= self.f1[j] if (y >> j) & 1 else self.f0[j]
        return v

    def p(self, q, bit):
        return float(abs(self.f1[q]) ** 2 if bit else self.f0[q] ** 2)


def _state(P, H, dt, prod):
    st = P.State(H, N, dt)
    st.run(prod.gates, 5)
    return st


def _amps(P, st, idx):
    out = np.empty(len(idx), dtype=np.complex128)
    one = np.empty(1, dtype=P.NP_DTYPES[st.dt])
    for j, i in enumerate(idx):
        P.sv_copy_to_host(st.s, one, int(i), 1)
        out[j] = one[0]
    return out


def _samples(seed, count=1024):
    rng = np.random.default_rng(seed)
    idx = list(rng.integers(0, 1 << N, count, dtype=np.uint64)) + [0, (1 << N) - 1]
    return [int(i) for i in idx]


def _close(dt, got, want, scale=None):
    # |got - want| <= rel * scale, scale = |want| unless the result is a sum
    # of terms (then the sum of their magnitudes)
    rel = 1e-12 if dt == "c128" else 2e-6
    scale = np.abs(want) if scale is None else np.asarray(scale)
    err = np.abs(got - want)
    assert np.all(err <= rel * scale + 1e-300), float(np.max(err / np.maximum(scale, 1e-300)))


def _row(y, targets):
    return sum(((y >> t) & 1) << a for a, t in enumerate(targets))


def _with_row(y, targets, r):
    for a, t in enumerate(targets):
        y = (y & ~(1 << t)) | (((r >> a) & 1) << t)
    return y


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_diagonal_and_permutation_gates_30q(P, H, dt):
    prod = Product(1)
    rng = np.random.default_rng(2)
    st = _state(P, H, dt, prod)
    tg = [int(q) for q in rng.permutation(N)[:10]]
    dg = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << 10))
    st.apply_gen_permutation(None, dg, tg)
    idx = _samples(3)
    _close(dt, _amps(P, st, idx), np.array([dg[_row(y, tg)] * prod.amp(y) for y in idx]))
    st.close()
    _release()
    # a controlled permutation on 3 targets (control 29 = 1), through the tiles
    st = _state(P, H, dt, prod)
    tg3 = [2, 17, 9]
    perm = [int(x) for x in rng.permutation(8)]
    dg3 = np.exp(1j * rng.uniform(0, 2 * np.pi, 8))
    st.apply_gen_permutation(perm, dg3, tg3, [29], [1])
    want = []
    for y in idx:
        if (y >> 29) & 1:
            r = _row(y, tg3)
            want.append(dg3[r] * prod.amp(_with_row(y, tg3, perm[r])))
        else:
            want.append(prod.amp(y))
    _close(dt, _amps(P, st, idx), np.array(want))
    st.close()
    _release()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_pauli_rotation_30q(P, H, dt):
    prod = Product(4)
    st = _state(P, H, dt, prod)
    term = [(0, "X"), (13, "Y"), (21, "Z"), (29, "X")]
    t = 0.37
    P.sv_apply_pauli_rotation(st.s, t, term)
    x = (1 << 0) | (1 << 13) | (1 << 29)
    z = (1 << 13) | (1 << 21)
    idx = _samples(5)
    want, scale = [], []
    for y in idx:
        # (P amp)(y) = i^nY (-1)^popcount((y ^ x) & z) amp(y ^ x)
        pa = (1j) ** 1 * (-1) ** bin((y ^ x) & z).count("1") * prod.amp(y ^ x)
        want.append(math.cos(t) * prod.amp(y) + 1j * math.sin(t) * pa)
        scale.append(abs(math.cos(t) * prod.amp(y)) + abs(math.sin(t) * pa))
    _close(dt, _amps(P, st, idx), np.array(want), scale)
    st.close()
    _release()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_measurement_30q(P, H, dt):
    prod = Product(6)
    tol = 1e-12 if dt == "c128" else 2e-6
    st = _state(P, H, dt, prod)
    for qs in ([3, 28, 15], [0, 7, 19, 24, 29, 11]):
        got = P.sv_measure_probabilities(st.s, qs)
        want = [np.prod([prod.p(q, (b >> a) & 1) for a, q in enumerate(qs)]) for b in range(1 << len(qs))]
        assert np.max(np.abs(got - want)) <= tol
    qz = [1, 5, 9, 22, 27]
    pe, po = P.sv_zbasis_probabilities(st.s, qz)
    z = np.prod([prod.p(q, 0) - prod.p(q, 1) for q in qz])
    assert abs((pe - po) - z) <= tol and abs(pe + po - 1.0) <= tol
    # collapse qubit 12 onto 1
    p1 = prod.p(12, 1)
    P.sv_collapse(st.s, [12], 1, p1)
    idx = _samples(7)
    want = [prod.amp(y) / math.sqrt(p1) if (y >> 12) & 1 else 0.0 for y in idx]
    _close(dt, _amps(P, st, idx), np.array(want, dtype=np.complex128))
    st.close()
    _release()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_dense_observable_30q(P, H, dt):
    prod = Product(8)
    rng = np.random.default_rng(9)
    st = _state(P, H, dt, prod)
    tg = [4, 26, 11]
    m = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
    phi = np.array([np.prod([prod.f1[q] if (r >> a) & 1 else prod.f0[q] for a, q in enumerate(tg)]) for r in range(8)])
    want = np.vdot(phi, m @ phi)
    got = P.sv_expect_matrix(st.s, m, tg)
    assert abs(got - want) <= (1e-12 if dt == "c128" else 2e-6) * max(1.0, abs(want))
    st.close()
    _release()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_index_bit_swap_and_accessor_30q(P, H, dt):
    prod = Product(10)
    idx = _samples(11)
    for pairs in ([(1, 25), (4, 17), (0, 29)], [(1, 25), (4, 17), (0, 29), (8, 20)]):  # tiles / scattered moves
        st = _state(P, H, dt, prod)
        P.sv_swap_index_bits(st.s, pairs)

        def pi(y):
            for a, b in pairs:
                if ((y >> a) ^ (y >> b)) & 1:
                    y ^= (1 << a) | (1 << b)
            return y

        _close(dt, _amps(P, st, idx), np.array([prod.amp(pi(y)) for y in idx]))
        st.close()
        _release()
    st = _state(P, H, dt, prod)
    order = list(range(N))[::-1]
    svd = P.SV_C64 if dt == "c64" else P.SV_C128
    lo = (1 << N) - 4096
    got = P.sv_accessor_get(st.s, svd, order, begin=lo, end=1 << N).astype(np.complex128)
    want = [prod.amp(int(format(k, f"0{N}b")[::-1], 2)) for k in range(lo, 1 << N)]
    _close(dt, got, np.array(want))
    st.close()
    _release()
