"""The 30-qubit brickwork workload in the launch configuration the benchmark
times (fused blocks of up to 5 qubits through the tiled kernels), complex64
and complex128.  A host oracle of the depth-20 state takes too long for a
test, so these check what holds at any size:
  - depth 1 (a U3 on every qubit, then one CZ brick) is a product state up to
    CZ signs: every amplitude, <Z_j>, <Z_j Z_j+1> and the CDF at any index
    have closed forms.  Checked on 4096 sampled amplitudes (plus the ends),
    all 30 <Z_j> and 29 <Z_j Z_j+1>, and 2^16 samples by the epsilon rule;
  - depth 20 followed by its mirror returns to |0..0> (amplitude, norm,
    every sample).
"""
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


def _amps(P, st, idx):
    dt = P.NP_DTYPES[st.dt]
    out = np.empty(len(idx), dtype=np.complex128)
    one = np.empty(1, dtype=dt)
    for j, i in enumerate(idx):
        P.sv_copy_to_host(st.s, one, int(i), 1)
        out[j] = one[0]
    return out


def _product_form(gates, n):
    """Single-qubit factors of a depth-1 brickwork state: U3(theta, phi, lam)
    maps |0> to cos(theta/2)|0> + e^{i phi} sin(theta/2)|1>; the CZ brick only
    flips signs.  Returns (a0, a1, cz_pairs)."""
    a0 = np.empty(n)
    a1 = np.empty(n, dtype=np.complex128)
    pairs = []
    for g in gates:
        if g.name == "u3":
            th, ph, _ = g.params
            a0[g.qubits[0]] = math.cos(th / 2)
            a1[g.qubits[0]] = np.exp(1j * ph) * math.sin(th / 2)
        else:
            assert g.name == "cz"
            pairs.append(g.qubits)
    return a0, a1, pairs


def _amp(y, a0, a1, pairs):
    v = 1.0 + 0.0j
    for j in range(len(a0)):
        v *= a1[j] if (y >> j) & 1 else a0[j]
    for a, b in pairs:
        if (y >> a) & 1 and (y >> b) & 1:
            v = -v
    return v


def _cdf_below(y, q0, q1):
    """P(X < y) for independent bits with P(bit j = 0) = q0[j]: sum over the
    bits k where y has a 1 of P(bits above k agree with y) * q0[k]."""
    below, above = 0.0, 1.0
    for k in range(len(q0) - 1, -1, -1):
        if (y >> k) & 1:
            below += above * q0[k]
            above *= q1[k]
        else:
            above *= q0[k]
    return below, above  # above == P(X == y) after the last bit


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_depth1_product_state_closed_form(P, H, dt):
    gates = W.brickwork(N, 1, 2024)
    a0, a1, pairs = _product_form(gates, N)
    st = P.State(H, N, dt)
    nb = st.run(gates, max_fused_qubits=5)
    assert nb > 0
    rng = np.random.default_rng(7)
    ys = rng.integers(0, 1 << N, size=4096, dtype=np.uint64).tolist() + [0, 1, (1 << N) - 1, 1 << (N - 1)]
    got = _amps(P, st, ys)
    ref = np.array([_amp(int(y), a0, a1, pairs) for y in ys])
    scaled = np.max(np.abs(got - ref)) * math.sqrt(1 << N)
    assert scaled <= (1e-9 if dt == "c128" else 2e-4), scaled
    # an estimate of ||psi_gpu - psi|| from the sample, and the rigorous
    # bound sum |dp| <= 2 ||dpsi|| + ||dpsi||^2, with a safety factor of 10
    dnorm = math.sqrt(float(np.mean(np.abs(got - ref) ** 2)) * (1 << N))
    assert dnorm ** 2 <= 1e-5
    eps = 10 * (2 * dnorm + dnorm ** 2) + 1e-12
    q0 = a0 ** 2
    q1 = np.abs(a1) ** 2
    zs = st.expect([[(j, "Z")] for j in range(N)] + [[(j, "Z"), (j + 1, "Z")] for j in range(N - 1)])
    zref = np.concatenate([q0 - q1, (q0 - q1)[:-1] * (q0 - q1)[1:]])
    np.testing.assert_allclose(zs, zref, atol=(1e-10 if dt == "c128" else 1e-5))
    u = W.uniforms(1 << 16, 31)
    smp = st.sample(u)
    for uu, y in zip(u.tolist(), smp.tolist()):
        lo, p = _cdf_below(int(y), q0, q1)
        assert p > 0
        assert lo - eps <= uu < lo + p + eps, (uu, y, lo, p, eps)
    st.close()
    _release()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_depth20_mirror_returns_to_zero(P, H, dt):
    gates = W.brickwork(N, 20, 0)
    st = P.State(H, N, dt)
    st.run(gates + W.inverse(gates), max_fused_qubits=5)
    a = _amps(P, st, [0, 1, 1 << (N - 1)])
    tol = 1e-10 if dt == "c128" else 2e-4
    assert abs(a[0] - 1.0) <= tol and abs(a[1]) <= tol and abs(a[2]) <= tol, a
    assert abs(st.norm() - 1.0) <= (1e-10 if dt == "c128" else 1e-4)
    assert (st.sample(W.uniforms(1 << 16, 4)) == 0).all()
    st.close()
    _release()
