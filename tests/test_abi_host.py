"""CPU checks of libsv: the shared library loads and exports every entry
point that include/sv.h declares, and its host logic (the gate table and gate
fusion) is right.  No compute call touches a GPU here."""
import json
import math
import os
import re

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import workloads as W
from tests.kron_ref import PAULI

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2308_01999_amd as P
    return P


def _declared():
    src = open(os.path.join(ROOT, "include", "sv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(P):
    import ctypes
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the declared entry points
    assert sorted(P.EXPORTED) == names


def test_binding_constants_match_the_header(P):
    # the Python names of the header's enum values and defines carry the
    # header's numbers
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sv.h")).read(), flags=re.S)
    enums = dict((k, int(v)) for k, v in re.findall(r"\b(SV_TILE_[A-Z]+)\s*=\s*(\d+)", src))
    assert set(enums) == {"SV_TILE_AUTO", "SV_TILE_NARROW", "SV_TILE_WIDE", "SV_TILE_SPREAD"}
    for name, v in enums.items():
        assert getattr(P, name) == v, name
    warm = re.search(r"#define\s+SV_TILE_WARM_SWEEPS\s+(\d+)", src)
    assert warm and P.TILE_WARM_SWEEPS == int(warm.group(1))


def test_version_string(P):
    assert "gfx950" in P.sv_version()


def _u3_ref(th, ph, la):
    rz = lambda a: expm(-0.5j * a * PAULI["Z"])
    ry = lambda a: expm(-0.5j * a * PAULI["Y"])
    return np.exp(0.5j * (ph + la)) * rz(ph) @ ry(th) @ rz(la)


@pytest.mark.parametrize("seed", range(4))
def test_gate_table_u3(P, seed):
    th, ph, la = np.random.default_rng(seed).uniform(0, 2 * math.pi, 3)
    m, nt, nc = P.sv_gate_matrix("u3", (th, ph, la))
    assert (nt, nc) == (1, 0)
    np.testing.assert_allclose(m, _u3_ref(th, ph, la), atol=1e-14)
    md, _, _ = P.sv_gate_matrix("u3_dg", (th, ph, la))
    np.testing.assert_allclose(md @ m, np.eye(2), atol=1e-14)


def test_gate_table_named(P):
    for name, ref, nt, nc in [("h", (PAULI["X"] + PAULI["Z"]) / math.sqrt(2), 1, 0), ("x", PAULI["X"], 1, 0),
                              ("y", PAULI["Y"], 1, 0), ("z", PAULI["Z"], 1, 0), ("cx", PAULI["X"], 1, 1),
                              ("cz", PAULI["Z"], 1, 1), ("swap", np.eye(4)[[0, 2, 1, 3]], 2, 0)]:
        m, a, b = P.sv_gate_matrix(name)
        assert (a, b) == (nt, nc), name
        np.testing.assert_allclose(m, ref, atol=1e-15, err_msg=name)
    m, nt, nc = P.sv_gate_matrix("cp", (0.7,))
    np.testing.assert_allclose(m, np.diag([1, np.exp(0.7j)]), atol=1e-15)
    m, _, _ = P.sv_gate_matrix("cp_dg", (0.7,))
    np.testing.assert_allclose(m, np.diag([1, np.exp(-0.7j)]), atol=1e-15)


def test_gate_table_rejects_bad_input(P):
    for args in [("nope", ()), ("u3", (1.0,)), ("cp", ()), ("u3", (float("nan"), 0, 0))]:
        with pytest.raises(P.SVError) as e:
            P.sv_gate_matrix(*args)
        assert e.value.status == P.SV_ERR_INVALID_VALUE


def _apply_blocks_with_oracle(n, blocks, basis=0):
    psi = oracle.basis_state(n, basis)
    for targets, m in blocks:
        if m.ndim == 1:  # a diagonal block
            oracle.apply_gperm(psi, None, m, targets)
        else:
            oracle.apply(psi, m, targets)
    return psi


@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("circuit", ["brickwork", "cxcp", "qft", "dense"])
def test_fusion_equals_unfused(P, kmax, circuit):
    n = 8
    if circuit == "brickwork":
        gates = W.brickwork(n, 6, kmax)
    elif circuit == "cxcp":
        gates = W.random_cx_cp(n, 5, kmax)
    elif circuit == "qft":
        gates = W.qft(n)
    else:
        gates = [W.Gate("mat", t, m) for t, c, cv, m in W.random_dense_circuit(n, 12, 3, kmax, with_controls=False)]
    x = W.random_basis_state(n, kmax)
    ref = oracle.run(n, gates, basis=x)
    f = P.fuse(gates, kmax)
    blocks = f.blocks()
    f.free()
    for targets, m in blocks:
        assert list(targets) == sorted(targets)
        assert len(targets) <= max(kmax, 3 if circuit == "dense" else 2)
        np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-13)
    got = _apply_blocks_with_oracle(n, blocks, basis=x)
    np.testing.assert_allclose(got, ref, atol=1e-12)


@pytest.mark.parametrize("kmax", [2, 5])
def test_fusion_of_adjoint_gates(P, kmax):
    # "mat_dg" gates reach the fuser as their matrix with the adjoint flag
    # set; the fused program equals the unfused oracle run, and a dense
    # circuit followed by its inverse fuses to the identity
    n = 7
    dense = [W.Gate("mat", t, m) for t, c, cv, m in W.random_dense_circuit(n, 10, 3, 5 + kmax, with_controls=False)]
    gates = dense + W.inverse(dense)
    assert any(g.name == "mat_dg" for g in gates)
    entries = P.gate_entries(gates)
    assert all(e[1] is not None and (e[4] == (g.name == "mat_dg")) for e, g in zip(entries, gates))
    x = W.random_basis_state(n, kmax)
    f = P.fuse(gates, kmax)
    blocks = f.blocks()
    f.free()
    got = _apply_blocks_with_oracle(n, blocks, basis=x)
    np.testing.assert_allclose(got, oracle.run(n, gates, basis=x), atol=1e-12)
    np.testing.assert_allclose(got, oracle.basis_state(n, x), atol=1e-12)
    # the flag gives exactly the block of the conjugate-transposed matrix
    t, c, cv, m = W.random_dense_circuit(n, 1, 3, 11, with_controls=False)[0]
    fa = P.sv_fuse_gates([(t, m, (), None, True)], 5)
    fb = P.sv_fuse_gates([(t, np.conj(m).T.copy(), (), None, False)], 5)
    np.testing.assert_array_equal(P.sv_fused_block(fa, 0)[1], P.sv_fused_block(fb, 0)[1])
    P.sv_fused_free(fa)
    P.sv_fused_free(fb)


def test_fusion_with_controls_and_values(P):
    n = 7
    ops = W.random_dense_circuit(n, 30, 2, 77)
    ref = oracle.basis_state(n, 3)
    for t, c, cv, m in ops:
        oracle.apply(ref, m, t, c, cv)
    entries = [(t, m, c, cv if c else None) for t, c, cv, m in ops]
    f = P.sv_fuse_gates(entries, 5)
    blocks = [P.sv_fused_block(f, i) for i in range(P.sv_fused_count(f))]
    P.sv_fused_free(f)
    got = _apply_blocks_with_oracle(n, blocks, basis=3)
    np.testing.assert_allclose(got, ref, atol=1e-12)


@pytest.mark.parametrize("kmax,kdiag", [(2, 3), (3, 6), (5, 10), (4, 1), (5, 0)])
@pytest.mark.parametrize("circuit", ["qft", "diagheavy", "cxcp", "brickwork"])
def test_diagonal_fusion_equals_unfused(P, kmax, kdiag, circuit):
    # dense and diagonal blocks applied in order (diagonal ones by the
    # oracle's diagonal gate) equal the unfused circuit; dense blocks are
    # unitary and within kmax, diagonal ones unit-modulus and within kdiag
    n = 9
    gates = {"qft": lambda: W.qft(n), "diagheavy": lambda: W.diagonal_heavy(n, 80, kmax + 10 * kdiag),
             "cxcp": lambda: W.random_cx_cp(n, 5, kdiag), "brickwork": lambda: W.brickwork(n, 5, kmax)}[circuit]()
    x = W.random_basis_state(n, kdiag)
    ref = oracle.run(n, gates, basis=x)
    f = P.fuse(gates, kmax, kdiag)
    blocks = f.blocks()
    n_diag = sum(P.sv_fused_block_is_diagonal(f.f, i) for i in range(f.count))
    f.free()
    for targets, m in blocks:
        assert list(targets) == sorted(targets)
        if m.ndim == 1:
            assert len(targets) <= kdiag
            np.testing.assert_allclose(np.abs(m), 1.0, atol=1e-13)
        else:
            assert len(targets) <= max(kmax, 3 if circuit == "diagheavy" else 2)
            np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-13)
    assert n_diag == sum(1 for _, m in blocks if m.ndim == 1)
    if kdiag == 0:
        assert n_diag == 0
    got = _apply_blocks_with_oracle(n, blocks, basis=x)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_diagonal_fusion_off_is_the_plain_fuser(P):
    gates = W.qft(10)
    a, b = P.fuse(gates, 4), P.fuse(gates, 4, 0)
    assert a.count == b.count
    for (ta, ma), (tb, mb) in zip(a.blocks(), b.blocks()):
        assert ta == tb
        np.testing.assert_array_equal(ma, mb)


def test_diagonal_fusion_cuts_qft_sweeps(P):
    # the QFT's controlled phases are diagonal: with diagonal blocks the
    # 30-qubit QFT needs far fewer sweeps than with dense blocks alone
    gates = W.qft(30)
    dense, both = P.fuse(gates, 5).count, P.fuse(gates, 5, 10).count
    assert both < 0.6 * dense


def _apply_coupled_with_oracle(n, blocks, couplings, basis=0):
    # each block: its phase coupling (as two-qubit controlled phases between
    # a block qubit and a coupled qubit, applied by the oracle), then its
    # matrix
    psi = oracle.basis_state(n, basis)
    for (targets, m), (cq, ph) in zip(blocks, couplings):
        for a, t in enumerate(targets):
            for c, q in enumerate(cq):
                if ph[a, c] != 0.0:
                    oracle.apply(psi, np.diag([1.0, 1.0, 1.0, np.exp(1j * ph[a, c])]), (t, q))
        oracle.apply(psi, m, targets)
    return psi


@pytest.mark.parametrize("kmax", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("circuit", ["qft", "diagheavy", "cxcp", "brickwork", "mirror"])
def test_coupled_fusion_equals_unfused(P, kmax, circuit):
    # blocks of coupled fusion applied in order (phase coupling, then
    # matrix) equal the unfused circuit from a random basis state; every
    # block is unitary on at most kmax qubits and couples only qubits outside
    # it
    n = 10
    gates = {"qft": lambda: W.qft(n), "diagheavy": lambda: W.diagonal_heavy(n, 90, 7 * kmax),
             "cxcp": lambda: W.random_cx_cp(n, 6, kmax), "brickwork": lambda: W.brickwork(n, 6, kmax),
             "mirror": lambda: W.random_cx_cp(n, 4, 3) + W.inverse(W.random_cx_cp(n, 4, 3))}[circuit]()
    x = W.random_basis_state(n, kmax)
    ref = oracle.run(n, gates, basis=x)
    f = P.fuse(gates, kmax, coupled=True)
    blocks, couplings = f.blocks(), f.couplings()
    f.free()
    for (targets, m), (cq, ph) in zip(blocks, couplings):
        assert list(targets) == sorted(targets)
        assert len(targets) <= max(kmax, 3 if circuit == "diagheavy" else 2)
        assert m.ndim == 2
        np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-12)
        assert list(cq) == sorted(cq) and not set(cq) & set(targets)
        assert ph.shape == (len(targets), len(cq))
    got = _apply_coupled_with_oracle(n, blocks, couplings, basis=x)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_coupled_fusion_of_the_qft_is_as_tight_as_table_ii(P):
    # Table II fuses the 33-qubit QFT (577 gates) into 18 gates with a fused
    # size of 4 or 5; coupled fusion at 5 needs no more: seven dense blocks
    # of five H with their phases (the phases to earlier qubits as
    # couplings) and the final swaps two by two
    counts = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_gate_counts.json")))
    gates = W.qft(33)
    assert len(gates) == counts["qft"]["gates"]
    f = P.fuse(gates, 5, coupled=True)
    assert f.count <= counts["qft"]["fused_1gpu"]
    assert P.fuse(gates, 5).count > 2 * f.count
    f.free()


def test_coupled_fusion_keeps_non_phase_diagonals_in_blocks(P):
    # a diagonal gate whose entries are not all of modulus one is not a
    # phase and is never deferred: it stays a dense gate of its block
    d = np.diag([1.0, 0.5])
    gates = [("mat", (0,), np.diag(np.exp([0.3j, 1.1j]))), ("mat", (1,), d), ("h", (1,), ()),
             ("cz", (0, 1), ()), ("mat", (0, 1), np.diag([1.0, 1.0, 0.2, 1.0]))]
    ref = oracle.run(2, gates, basis=3)
    f = P.fuse(gates, 1, coupled=True)
    got = _apply_coupled_with_oracle(2, f.blocks(), f.couplings(), basis=3)
    f.free()
    np.testing.assert_allclose(got, ref, atol=1e-13)


def test_diagonal_fusion_rejects_bad_sizes(P):
    gates = W.qft(4)
    for kd in (-1, 11):
        with pytest.raises(P.SVError):
            P.fuse(gates, 4, kd)


def test_fusion_reduces_sweeps_on_brickwork(P):
    # the block count is reported, not pinned; it must beat one sweep per
    # two-qubit brick by a wide margin
    gates = W.brickwork(30, 20, 0)
    counts = {k: P.fuse(gates, k).count for k in (4, 5, 6)}
    assert counts[5] < 100 and counts[6] <= counts[5] <= counts[4]


def test_fusion_rejects_bad_input(P):
    with pytest.raises(P.SVError):
        P.sv_fuse_gates([((0,), np.eye(2), (), None)], 0)
    with pytest.raises(P.SVError):
        P.sv_fuse_gates([((0, 0), np.eye(4), (), None)], 5)
    with pytest.raises(P.SVError):
        P.sv_fuse_gates([((0,), np.eye(2), (0,), None)], 5)
    with pytest.raises(P.SVError):
        P.sv_fuse_gates([((0,), np.full((2, 2), np.inf), (), None)], 5)
    with pytest.raises(P.SVError):
        P.sv_fuse_gates([((1,), np.eye(2), (0,), (2,))], 5)
    assert P.sv_last_error()


def test_empty_fusion(P):
    f = P.sv_fuse_gates([], 5)
    assert P.sv_fused_count(f) == 0
    P.sv_fused_free(f)


def test_handle_create_without_gpu_reports_device_error(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.SVError) as e:
        P.sv_handle_create(0, 0)
    assert e.value.status == P.SV_ERR_DEVICE


def test_package_binds_one_hip_runtime():
    """Importing the package before torch must not load a second HIP/HSA
    runtime next to torch's (the second one enumerates no device)."""
    import subprocess
    import sys
    code = ("import paper_2308_01999_amd, torch\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in m if 'libamdhip64' in l or 'libhsa-runtime64' in l}\n"
            "print(len([x for x in libs if 'amdhip' in x]), len([x for x in libs if 'hsa-runtime' in x]))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, check=True)
    assert out.stdout.split() == ["1", "1"], out.stdout


def test_hbm_budget_caps_allocations_before_device_work():
    """SV_HBM_BUDGET_BYTES caps what libsv allocates; a handle whose
    workspace does not fit fails with SV_ERR_OUT_OF_MEMORY before any HIP
    call (so the same status comes back with or without a GPU), and an
    unparsable value means no cap.  Run in a child process: the cap is read
    once per process."""
    import subprocess
    import sys
    code = ("import paper_2308_01999_amd as P\n"
            "print(P.sv_hbm_usage())\n"
            "try:\n"
            "    P.sv_handle_create(0, 32 << 20)\n"
            "    print('created')\n"
            "except P.SVError as e:\n"
            "    print(e.status, 'budget' in str(e))\n"
            "P.sv_set_hbm_budget(0)\n"
            "print(P.sv_hbm_usage())\n")
    env = dict(os.environ, SV_HBM_BUDGET_BYTES=str(16 << 20))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True,
                         env=env)
    lines = out.stdout.split("\n")
    assert lines[0] == f"(0, {16 << 20})"
    assert lines[1] == "2 True"            # SV_ERR_OUT_OF_MEMORY, message names the budget
    assert lines[2] == "(0, 0)"
    env["SV_HBM_BUDGET_BYTES"] = "lots"
    out = subprocess.run([sys.executable, "-c", "import paper_2308_01999_amd as P; print(P.sv_hbm_usage())"],
                         cwd=ROOT, capture_output=True, text=True, check=True, env=env)
    assert out.stdout.strip() == "(0, 0)"


def test_hbm_budget_setter(P):
    used, cap = P.sv_hbm_usage()
    try:
        P.sv_set_hbm_budget(1 << 20)
        assert P.sv_hbm_usage()[1] == 1 << 20
        with pytest.raises(P.SVError) as e:
            P.sv_handle_create(0, 12 << 20)
        assert e.value.status == P.SV_ERR_OUT_OF_MEMORY
    finally:
        P.sv_set_hbm_budget(cap)
