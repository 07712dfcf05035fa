"""The sampler with device-resident uniforms and outcomes (sv_sample_device)
and the bucketed resolver behind both sampler entry points, through the C
ABI.  The device variant must return bit for bit what sv_sample returns for
the same uniforms (index work), also over several shot batches of the host
variant; samples obey the epsilon-interval rule on the oracle's CDF; states
whose shots all fall into one chunk, or into a handful of chunks, exercise
the per-wave grouping of the bucket counters; invalid uniforms, which only
the kernels can see, and pointers that are not device memory are errors."""
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
    assert np.all(lo - eps <= r) and np.all(r < cdf[got] + eps)
    assert np.all(p_g[got] > 0)


def _device_sample(P, H, st, u, bit_ordering=None):
    import torch
    with torch.cuda.stream(H.stream):
        du = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64)).to("cuda")
        out = torch.empty(len(u), dtype=torch.int64, device="cuda")
    H.stream.synchronize()
    P.sv_sample_device(st.s, du.data_ptr(), len(u), out.data_ptr(), bit_ordering)
    return out.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 6, 13, 17, 21])
def test_device_sampler_equals_host_sampler(P, H, dt, n):
    gates = W.brickwork(n, 8, 50 + n)
    ref = oracle.run(n, gates)
    st = P.State(H, n, dt)
    st.run(gates)
    gpu = st.to_numpy()
    u = W.uniforms(60000, 7 + n)
    host = st.sample(u)
    dev = _device_sample(P, H, st, u)
    np.testing.assert_array_equal(dev, host)
    _eps_rule(gpu, ref, u, dev)
    if n >= 3:
        bo = [n - 1, 0, n // 2]
        np.testing.assert_array_equal(_device_sample(P, H, st, u, bo), st.sample(u, bo))
    st.close()


def test_device_sampler_over_several_host_batches(P, H):
    # more shots than one batch of the host variant's workspace: the host
    # path resolves them in several batches, the device path in one
    n = 16
    st = P.State(H, n, "c64")
    st.run(W.brickwork(n, 6, 3))
    u = W.uniforms(2_600_000, 5)
    host = st.sample(u)
    dev = _device_sample(P, H, st, u)
    np.testing.assert_array_equal(dev, host)
    gpu = st.to_numpy()
    _eps_rule(gpu, gpu.astype(np.complex128), u[:200000], dev[:200000])
    st.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_all_shots_in_one_chunk(P, H, dt):
    # |0..0>: every one of 2^20 shots lands in chunk 0, block 0, index 0
    n = 22
    st = P.State(H, n, dt)
    u = W.uniforms(1 << 20, 11)
    np.testing.assert_array_equal(st.sample(u), np.zeros(1 << 20, dtype=np.uint64))
    np.testing.assert_array_equal(_device_sample(P, H, st, u), np.zeros(1 << 20, dtype=np.uint64))
    st.close()


def test_shots_in_a_few_chunks(P, H):
    # mass on five amplitudes in five chunks, unequal weights: each outcome
    # is one of them, with the interval rule on the exact CDF
    n = 24
    dim = 1 << n
    idx = [5, 70000, 1 << 20, (1 << 23) + 17, dim - 1]
    w = np.array([0.1, 0.3, 0.05, 0.35, 0.2])
    psi = np.zeros(dim, dtype=np.complex128)
    psi[idx] = np.sqrt(w)
    st = P.State(H, n, "c128", basis=None)
    P.sv_copy_from_host(st.s, psi)
    u = W.uniforms(1 << 20, 12)
    host = st.sample(u)
    dev = _device_sample(P, H, st, u)
    np.testing.assert_array_equal(dev, host)
    assert set(np.unique(dev).tolist()) <= set(idx)
    # the kernels' probabilities (re^2, im = 0) and their running sum, which
    # here is the plain sequential cumulative sum: one amplitude per chunk
    cw = np.cumsum(psi[idx].real ** 2)
    r = np.minimum(u * cw[-1], np.nextafter(cw[-1], 0.0))
    expect = np.array(idx)[np.searchsorted(cw, r, side="right")]
    np.testing.assert_array_equal(dev.astype(np.int64), expect)
    st.close()


def test_device_sampler_rejects_invalid_uniforms_and_host_pointers(P, H):
    import torch
    n = 10
    st = P.State(H, n, "c64")
    st.run(W.brickwork(n, 4, 1))
    good = W.uniforms(1000, 2)
    for bad in (1.0, -0.25, float("nan")):
        u = good.copy()
        u[517] = bad
        with pytest.raises(P.SVError) as e:
            _device_sample(P, H, st, u)
        assert e.value.status == P.SV_ERR_INVALID_VALUE
    # the next call with valid uniforms is unaffected by the failed ones
    np.testing.assert_array_equal(_device_sample(P, H, st, good), st.sample(good))
    hu = np.ascontiguousarray(good)
    out = torch.empty(len(good), dtype=torch.int64, device="cuda")
    with pytest.raises(P.SVError) as e:
        P.sv_sample_device(st.s, hu.ctypes.data, len(good), out.data_ptr())
    assert e.value.status == P.SV_ERR_INVALID_VALUE
    du = torch.from_numpy(hu).to("cuda")
    ho = np.zeros(len(good), dtype=np.uint64)
    with pytest.raises(P.SVError) as e:
        P.sv_sample_device(st.s, du.data_ptr(), len(good), ho.ctypes.data)
    assert e.value.status == P.SV_ERR_INVALID_VALUE
    st.close()


def test_zero_state_is_rejected_by_both_samplers(P, H):
    n = 12
    st = P.State(H, n, "c64", basis=None)
    P.sv_copy_from_host(st.s, np.zeros(1 << n, dtype=np.complex64))
    u = W.uniforms(5000, 3)
    for f in (lambda: st.sample(u), lambda: _device_sample(P, H, st, u)):
        with pytest.raises(P.SVError) as e:
            f()
        assert e.value.status == P.SV_ERR_INVALID_VALUE
    st.close()
