"""The 30-qubit, depth-20 brickwork circuit (seed 0, start |0..0>) against
values the CPU oracle computed for it (``tests/golden/config2_30q_d20_seed0.npz``,
written by ``tests/golden/make_config2_golden.py``, which calls only the
oracle): 65540 amplitudes at seeded indices, the norm, all <Z_i>,
<Z_i Z_i+1>, eight random Pauli strings, the CDF at the same indices, and the
outcomes of 32768 seeded uniforms.

The GPU runs the circuit unfused (one sweep per gate) and fused into blocks of
up to five qubits through the tiled kernels the benchmark times, with each
tile variant forced and with the handle's own choice after the tuner has
settled, in complex128 and complex64.  Bars (Sec. II-B gate application;
Table I expectation and sampler):
  - complex128: max |d amp| <= 1e-10 on the sampled amplitudes;
  - complex64: ||d psi||^2, estimated from the sampled amplitudes scaled to
    the whole state, <= 1e-5 (fidelity >= 1 - ||d psi||^2 for unit vectors);
  - expectations |d| <= 1e-9 (c128) / 1e-4 (c64); norm |d| <= 1e-12 / 1e-5;
  - CDF of the GPU state (FP64 prefix sums of its probabilities) at the
    sampled indices within 1e-10 (c128) / 1e-5 (c64) of the oracle's;
  - samples: every GPU outcome lies in its interval of the GPU state's own
    CDF; every oracle outcome lies in its interval of the GPU state's CDF
    widened by the CDF bound above; in complex128 the outcomes equal the
    oracle's except where u N is within 1e-10 of an interval's edge.
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N, DEPTH, SEED = 30, 20, 0
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config2_30q_d20_seed0.npz")
TOL = {"c128": dict(amp=1e-10, dpsi2=None, expect=1e-9, norm=1e-12, cdf=1e-10),
       "c64": dict(amp=None, dpsi2=1e-5, expect=1e-4, norm=1e-5, cdf=1e-5)}
MODES = {"auto": 0, "narrow": 1, "wide": 2, "spread": 3}


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < (48 << 30):
        pytest.skip("needs 48 GiB of free device memory")
    import paper_2308_01999_amd as P
    return P


@pytest.fixture(scope="module")
def G():
    with np.load(GOLD, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    assert int(g["n"]) == N and int(g["depth"]) == DEPTH and int(g["seed"]) == SEED
    return g


@pytest.fixture(scope="module")
def gates():
    return W.brickwork(N, DEPTH, SEED)


def _terms(G):
    ops = G["pauli_ops"]
    return [[(q, "IXYZ"[int(o)]) for q, o in enumerate(row) if o] for row in ops]


def _release():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _cdf_at(st, where):
    """FP64 prefix sums of the GPU state's probabilities at the indices
    `where` (int64 numpy), and the total; computed on the device."""
    import torch
    t = st.tensor
    p = t.real.double().square_()
    p.add_(t.imag.double().square_())
    torch.cumsum(p, 0, out=p)
    total = float(p[-1].item())
    w = torch.from_numpy(np.ascontiguousarray(where, dtype=np.int64)).to(t.device)
    out = p[w].cpu().numpy()
    del p, w
    _release()
    return out, total


def _check(P, st, dt, G, label):
    import torch
    tol = TOL[dt]
    idx = G["idx"].astype(np.int64)
    got = st.tensor[torch.from_numpy(idx).to(st.tensor.device)].cpu().numpy().astype(np.complex128)
    d = got - G["amp"]
    if tol["amp"] is not None:
        err = float(np.max(np.abs(d)))
        assert err <= tol["amp"], f"{label}: max |d amp| = {err:.3e}"
    if tol["dpsi2"] is not None:
        est = float(np.sum(np.abs(d) ** 2)) * (2.0 ** N) / idx.size
        assert est <= tol["dpsi2"], f"{label}: estimated ||d psi||^2 = {est:.3e}"
    nrm = P.sv_norm(st.s)
    assert abs(nrm - float(G["norm"])) <= tol["norm"], f"{label}: norm {nrm!r}"
    for key, terms in (("z", W.z_terms(N)), ("zz", W.zz_neighbour_terms(N)), ("pauli", _terms(G))):
        e = P.sv_expect_pauli(st.s, terms)
        err = float(np.max(np.abs(e - G[key])))
        assert err <= tol["expect"], f"{label}: {key} expectations differ by {err:.3e}"

    # CDF at the sampled indices, then the samples
    u = W.uniforms(int(G["shots"].size), int(G["shot_seed"]))
    o_g = P.sv_sample(st.s, u).astype(np.int64)
    o_o = G["shots"].astype(np.int64)
    where = np.concatenate([idx, o_g, np.maximum(o_g - 1, 0), o_o, np.maximum(o_o - 1, 0)])
    c, total = _cdf_at(st, where)
    m, s = idx.size, o_g.size
    c_idx = c[:m]
    g_hi, g_lo = c[m:m + s], np.where(o_g > 0, c[m + s:m + 2 * s], 0.0)
    o_hi, o_lo = c[m + 2 * s:m + 3 * s], np.where(o_o > 0, c[m + 3 * s:], 0.0)
    cerr = float(np.max(np.abs(c_idx - G["cdf"])))
    assert cerr <= tol["cdf"], f"{label}: CDF differs from the oracle's by {cerr:.3e}"
    r = u * total
    eta = 1e-11  # prefix sums in another order than the sampler's
    ok = (g_lo - eta <= r) & (r < g_hi + eta)
    assert ok.all(), f"{label}: {(~ok).sum()} GPU outcomes outside their own CDF interval"
    eps = tol["cdf"] + eta
    ok = (o_lo - eps <= r) & (r < o_hi + eps)
    assert ok.all(), f"{label}: {(~ok).sum()} oracle outcomes outside the GPU CDF interval"
    if dt == "c128":
        r_o = u * float(G["norm"])
        edge = np.minimum(r_o - G["shot_c_lo"], G["shot_c_hi"] - r_o) <= 1e-10
        diff = (o_g != o_o) & ~edge
        assert not diff.any(), f"{label}: {diff.sum()} outcomes differ from the oracle's away from ties"


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_config2_unfused_matches_oracle(P, G, gates, dt):
    h = P.Handle()
    st = P.State(h, N, dt)
    print(f"config2 unfused {dt}", flush=True)
    st.run(gates)
    _check(P, st, dt, G, f"unfused {dt}")
    st.close()
    h.close()
    _release()


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_config2_fused_matches_oracle(P, G, gates, dt, mode):
    h = P.Handle()
    h.set_tile_mode(MODES[mode])
    st = P.State(h, N, dt)
    f = P.fuse(gates, 5)
    try:
        if mode == "auto":
            # the tuner's warm-up and trials happen on the circuit's own sweeps
            for _ in range(8):
                P.sv_set_basis_state(st.s, 0)
                P.sv_apply_fused(st.s, f.f)
            P.sv_set_basis_state(st.s, 0)
        print(f"config2 fused k<=5 {dt} tile mode {mode}", flush=True)
        P.sv_apply_fused(st.s, f.f)
    finally:
        f.free()
    _check(P, st, dt, G, f"fused {dt} {mode}")
    st.close()
    h.close()
    _release()
