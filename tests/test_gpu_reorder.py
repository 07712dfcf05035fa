"""GPU parity of the index bit swap and of the reordering accessor, through
the C ABI, against the oracle's plain definitions.  Both only move
amplitudes, so the comparison is bit for bit."""
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
    return st, host


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [4, 13, 18])
@pytest.mark.parametrize("seed", range(4))
def test_swap_index_bits_matches_oracle(P, H, dt, n, seed):
    rng = np.random.default_rng(31 * n + seed)
    qs = [int(q) for q in rng.permutation(n)]
    npairs = int(rng.integers(1, n // 2 + 1))
    pairs = [(qs[2 * p], qs[2 * p + 1]) for p in range(npairs)]
    nm = int(rng.integers(0, min(2, n - 2 * npairs) + 1))
    mbits = qs[2 * npairs:2 * npairs + nm]
    mvals = [int(v) for v in rng.integers(0, 2, nm)]
    st, host = _state(P, H, n, dt, rng)
    ref = host.astype(np.complex128)
    P.sv_swap_index_bits(st.s, pairs, mbits, mvals)
    oracle.swap_index_bits(ref, pairs, mbits, mvals)
    np.testing.assert_array_equal(st.to_numpy().astype(np.complex128), ref)
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [3, 12, 23])
def test_accessor_get_and_set_match_oracle(P, H, dt, n):
    # 23 qubits complex128 = 128 MiB: several 16 MiB staging chunks
    rng = np.random.default_rng(n)
    st, host = _state(P, H, n, dt, rng)
    ref = host.astype(np.complex128)
    SVD = P.SV_C64 if dt == "c64" else P.SV_C128
    order = [int(q) for q in rng.permutation(n)]
    got = P.sv_accessor_get(st.s, SVD, order)
    np.testing.assert_array_equal(got.astype(np.complex128), oracle.accessor_get(ref, order))
    # a slice with two mask bits and a sub-range
    if n >= 3:
        mb, mv, ob = order[:2], [1, 0], order[2:]
        lo, hi = (1 << (n - 2)) // 5, (1 << (n - 2)) - (3 if n > 4 else 0)
        got = P.sv_accessor_get(st.s, SVD, ob, mb, mv, lo, hi)
        np.testing.assert_array_equal(got.astype(np.complex128), oracle.accessor_get(ref, ob, mb, mv, lo, hi))
    # set writes the reordered values back: a round trip through a reversed
    # order restores the state
    rev = order[::-1]
    vals = P.sv_accessor_get(st.s, SVD, rev)
    st2 = P.State(H, n, dt)
    P.sv_accessor_set(st2.s, SVD, vals, rev)
    np.testing.assert_array_equal(st2.to_numpy(), host)
    st2.close()
    st.close()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_accessor_small_workspace_many_chunks(P, dt):
    # a 12 MiB workspace stages 4 MiB chunks: the double-buffered pipeline
    # runs over many chunks, with a range that starts and ends inside one
    n = 21
    rng = np.random.default_rng(5)
    h = P.Handle(workspace_bytes=12 << 20)
    st, host = _state(P, h, n, dt, rng)
    ref = host.astype(np.complex128)
    SVD = P.SV_C64 if dt == "c64" else P.SV_C128
    order = [int(q) for q in rng.permutation(n)]
    lo, hi = 12345, (1 << n) - 777
    got = P.sv_accessor_get(st.s, SVD, order, begin=lo, end=hi)
    np.testing.assert_array_equal(got.astype(np.complex128), oracle.accessor_get(ref, order, (), (), lo, hi))
    # write a permuted copy back through the same ordering into a zero state
    st2 = P.State(h, n, dt)
    P.sv_copy_from_host(st2.s, np.zeros(1 << n, dtype=host.dtype), 0)
    P.sv_accessor_set(st2.s, SVD, got, order, begin=lo)
    back = P.sv_accessor_get(st2.s, SVD, order, begin=lo, end=hi)
    np.testing.assert_array_equal(back, got)
    st.close()
    st2.close()
    h.close()


def test_reorder_bad_arguments(P, H):
    rng = np.random.default_rng(1)
    st, host = _state(P, H, 6, "c128", rng)
    for call in (lambda: P.sv_swap_index_bits(st.s, [(0, 1), (1, 2)]),
                 lambda: P.sv_swap_index_bits(st.s, [(0, 6)]),
                 lambda: P.sv_swap_index_bits(st.s, [(0, 1)], [1], [0]),
                 lambda: P.sv_accessor_get(st.s, P.SV_C128, [0, 1, 2]),
                 lambda: P.sv_accessor_get(st.s, P.SV_C128, [0, 1, 2, 3, 4, 4]),
                 lambda: P.sv_accessor_get(st.s, P.SV_C128, [0, 1, 2, 3, 4, 5], begin=10, end=70)):
        with pytest.raises(P.SVError):
            call()
    np.testing.assert_array_equal(st.to_numpy(), host)
    st.close()
