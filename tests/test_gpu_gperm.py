"""GPU parity of the generalized permutation gate G = D P and of the diagonal
gate (no permutation), through the C ABI, against the oracle's plain
definition on the same seeded inputs.  Tolerances: complex128 max |d amp| <=
1e-12 (one complex product per amplitude); complex64 max |d amp| <= 1e-6 of
the largest amplitude (diag rounded to FP32 once, one FP32 complex product:
a few units in the last place of a 24-bit significand)."""
import numpy as np
import pytest

import oracle

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


def _state(P, H, n, dt, rng):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    st = P.State(H, n, dt)
    host = v.astype(np.complex64 if dt == "c64" else np.complex128)
    P.sv_copy_from_host(st.s, host, 0)
    return st, host.astype(np.complex128)


def _check(dt, got, ref):
    if dt == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        assert np.max(np.abs(got.astype(np.complex128) - ref)) <= 1e-6 * np.max(np.abs(ref))


def _case(rng, n, kmax, ncmax, perm):
    k = int(rng.integers(1, kmax + 1))
    nc = int(rng.integers(0, min(ncmax, n - k) + 1))
    qs = [int(q) for q in rng.permutation(n)]
    targets, controls = qs[:k], qs[k:k + nc]
    cvals = [int(v) for v in rng.integers(0, 2, nc)]
    p = [int(x) for x in rng.permutation(1 << k)] if perm else None
    diag = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k)) * rng.uniform(0.5, 1.5, 1 << k)
    return targets, controls, cvals, p, diag


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [5, 13, 17])
@pytest.mark.parametrize("seed", range(4))
def test_diagonal_matches_oracle(P, H, dt, n, seed):
    # k up to 10 targets, up to 3 controls with values, adjoint on odd seeds;
    # sizes from one partial workgroup (5 qubits) to 32 workgroups
    rng = np.random.default_rng(100 * n + seed)
    targets, controls, cvals, _, diag = _case(rng, n, min(10, n), 3, False)
    st, ref = _state(P, H, n, dt, rng)
    adj = seed % 2 == 1
    st.apply_gen_permutation(None, diag, targets, controls, cvals, adjoint=adj)
    oracle.apply_gperm(ref, None, diag, targets, controls, cvals, adjoint=adj)
    _check(dt, st.to_numpy(), ref)
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_diagonal_with_control_on_bit_zero(P, H, dt):
    # complex64 pairs amplitudes (i, i + 1) per 16-byte access unless bit 0
    # is a control; that case runs one amplitude per access
    rng = np.random.default_rng(7)
    n = 14
    diag = np.exp(1j * rng.uniform(0, 2 * np.pi, 8))
    for controls, cvals in (((0,), (1,)), ((0, 9), (0, 1)), ((13, 0, 5), (1, 0, 0))):
        st, ref = _state(P, H, n, dt, rng)
        st.apply_gen_permutation(None, diag, (3, 1, 12), controls, cvals)
        oracle.apply_gperm(ref, None, diag, (3, 1, 12), controls, cvals)
        _check(dt, st.to_numpy(), ref)
        st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [5, 12, 16])
@pytest.mark.parametrize("seed", range(4))
def test_permutation_matches_oracle(P, H, dt, n, seed):
    # k + controls <= 6; 5 qubits runs the dense sweep with G written out,
    # 12 and 16 the LDS tile kernel (several tiles)
    rng = np.random.default_rng(1000 * n + seed)
    targets, controls, cvals, perm, diag = _case(rng, n, 5, 1, True)
    while len(targets) + len(controls) > 6:
        targets, controls, cvals, perm, diag = _case(rng, n, 5, 1, True)
    st, ref = _state(P, H, n, dt, rng)
    adj = seed % 2 == 1
    st.apply_gen_permutation(perm, diag, targets, controls, cvals, adjoint=adj)
    oracle.apply_gperm(ref, perm, diag, targets, controls, cvals, adjoint=adj)
    _check(dt, st.to_numpy(), ref)
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_permutation_round_trip_and_named_gates(P, H, dt):
    # G then G^dagger restores the state (unit-modulus diag); CX and SWAP as
    # permutations move amplitudes exactly (no arithmetic: bitwise)
    rng = np.random.default_rng(11)
    n = 15
    st, ref = _state(P, H, n, dt, rng)
    perm = [int(x) for x in rng.permutation(16)]
    diag = np.exp(1j * rng.uniform(0, 2 * np.pi, 16))
    st.apply_gen_permutation(perm, diag, (14, 2, 7, 0))
    st.apply_gen_permutation(perm, diag, (14, 2, 7, 0), adjoint=True)
    _check(dt, st.to_numpy(), ref)
    before = st.to_numpy()
    st.apply_gen_permutation([0, 3, 2, 1], np.ones(4), (4, 11))       # CX, control 4 -> target 11
    st.apply_gen_permutation([0, 2, 1, 3], np.ones(4), (0, 13))       # SWAP 0 <-> 13
    idx = np.arange(1 << n)
    src = idx.copy()
    b0, b13 = (idx >> 0) & 1, (idx >> 13) & 1
    src = (src & ~((1 << 0) | (1 << 13))) | (b13 << 0) | (b0 << 13)   # undo the swap
    b4, b11 = (src >> 4) & 1, (src >> 11) & 1
    src = src ^ ((b4 & 1) << 11)                                        # undo the CX
    np.testing.assert_array_equal(st.to_numpy(), before[src])
    st.close()


def test_identity_permutation_is_the_diagonal_path(P, H):
    rng = np.random.default_rng(5)
    st, ref = _state(P, H, 13, "c128", rng)
    diag = np.exp(1j * rng.uniform(0, 2 * np.pi, 32))
    st.apply_gen_permutation(list(range(32)), diag, (0, 3, 6, 9, 12), (5,), (0,))
    oracle.apply_gperm(ref, None, diag, (0, 3, 6, 9, 12), (5,), (0,))
    _check("c128", st.to_numpy(), ref)
    st.close()


def test_bad_arguments_leave_the_state_alone(P, H):
    rng = np.random.default_rng(6)
    st, ref = _state(P, H, 8, "c128", rng)
    bad = [
        dict(perm=[0, 0, 1, 2], diag=np.ones(4), targets=(0, 1)),            # not a permutation
        dict(perm=[0, 1, 2, 4], diag=np.ones(4), targets=(0, 1)),            # out of range
        dict(perm=None, diag=np.ones(4), targets=(0, 0)),                     # repeated target
        dict(perm=None, diag=np.ones(2), targets=(8,)),                       # out of range qubit
        dict(perm=None, diag=np.array([np.nan, 1]), targets=(1,)),            # non-finite
        dict(perm=list(range(64))[::-1], diag=np.ones(64), targets=(0, 1, 2, 3, 4, 5), controls=(7,)),  # 7 qubits
    ]
    for b in bad:
        with pytest.raises(P.SVError):
            st.apply_gen_permutation(b["perm"], b["diag"], b["targets"], b.get("controls", ()))
    with pytest.raises(P.SVError):
        P.sv_apply_gen_permutation(st.s, None, np.ones(4), (0, 1), (2, 2))   # control repeats
    np.testing.assert_array_equal(st.to_numpy(), ref)
    st.close()


# ------------------------------------------------ diagonal blocks in fusion

import workloads as W  # noqa: E402


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("circuit", ["qft", "diagheavy"])
@pytest.mark.parametrize("n", [9, 14])
def test_fused_program_with_diagonal_blocks_matches_oracle(P, H, dt, circuit, n):
    # dense blocks (k <= 5) and diagonal blocks (k <= 10) applied by libsv,
    # eagerly and as a recorded graph, against the unfused circuit in the
    # oracle; complex64 by state fidelity
    gates = W.qft(n) if circuit == "qft" else W.diagonal_heavy(n, 150, n)
    x = W.random_basis_state(n, 3)
    ref = oracle.run(n, gates, basis=x)
    f = P.fuse(gates, 5, 10)
    assert any(m.ndim == 1 for _, m in f.blocks())
    st = P.State(H, n, dt)
    P.sv_set_basis_state(st.s, x)
    P.sv_apply_fused(st.s, f.f)
    eager = st.to_numpy().astype(np.complex128)
    g = P.Graph(st, gates, 5, 10)
    P.sv_set_basis_state(st.s, x)
    g.launch()
    replay = st.to_numpy().astype(np.complex128)
    g.close()
    f.free()
    st.close()
    if dt == "c128":
        assert np.max(np.abs(eager - ref)) <= 1e-10
    else:
        assert oracle.fidelity(ref, eager) >= 1.0 - 1e-5
    np.testing.assert_array_equal(eager, replay)
