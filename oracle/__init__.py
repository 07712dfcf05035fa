"""CPU oracle for state-vector circuit simulation (complex128, FP64 sums).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the benchmark's ``cpu_baseline`` leg may import this package; the GPU
library never does, and this package imports nothing from it.

The arithmetic lives in ``sv_oracle.c`` (plain C, OpenMP over independent
amplitude groups only); this module marshals numpy arrays into it and builds
whole-circuit runs out of single-gate applications.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sv_oracle.c")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fcx-limited-range", "-fPIC", "-shared",
          "-std=c11"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc.  Building the checker is not using it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        L.orc_gate_matrix.argtypes = [ctypes.c_char_p, dp, ctypes.c_int, dp, ip, ip]
        L.orc_gate_matrix.restype = ctypes.c_int
        L.orc_apply.argtypes = [vp, ctypes.c_int, vp, ip, ctypes.c_int, ip, ip, ctypes.c_int]
        L.orc_apply.restype = ctypes.c_int
        L.orc_apply_gperm.argtypes = [vp, ctypes.c_int, vp, vp, ip, ctypes.c_int, ip, ip, ctypes.c_int]
        L.orc_apply_gperm.restype = ctypes.c_int
        L.orc_apply_pauli_rotation.argtypes = [vp, ctypes.c_int, ctypes.c_double, ip, ctypes.c_char_p, ctypes.c_int,
                                               ip, ip, ctypes.c_int]
        L.orc_apply_pauli_rotation.restype = ctypes.c_int
        L.orc_measure_probs.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, dp]
        L.orc_measure_probs.restype = ctypes.c_int
        L.orc_collapse.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_double]
        L.orc_collapse.restype = ctypes.c_int
        L.orc_expect_matrix.argtypes = [vp, ctypes.c_int, vp, ip, ctypes.c_int, dp]
        L.orc_expect_matrix.restype = ctypes.c_int
        L.orc_swap_index_bits.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, ip, ip, ctypes.c_int]
        L.orc_swap_index_bits.restype = ctypes.c_int
        L.orc_accessor.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, ip, ip, ctypes.c_int, vp, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int]
        L.orc_accessor.restype = ctypes.c_int
        L.orc_norm.argtypes = [vp, ctypes.c_int]
        L.orc_norm.restype = ctypes.c_double
        L.orc_expect_pauli.argtypes = [vp, ctypes.c_int, ip, ctypes.c_char_p, ctypes.c_int, dp]
        L.orc_expect_pauli.restype = ctypes.c_int
        L.orc_sample.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int64, ip, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_uint64), dp]
        L.orc_sample.restype = ctypes.c_int
        L.orc_set_basis.argtypes = [vp, ctypes.c_int, ctypes.c_uint64]
        L.orc_set_basis.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _ints(seq):
    seq = list(seq)
    return (ctypes.c_int * max(1, len(seq)))(*seq)


def _nqubits(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.dtype != np.complex128 or psi.ndim != 1 or (1 << n) != psi.size or not psi.flags.c_contiguous:
        raise ValueError("state must be a contiguous 1-D complex128 array of length 2^n")
    return n


def gate_matrix(name: str, params=()) -> tuple:
    """(matrix complex128 [2^k, 2^k], k, n_controls) from the oracle's own gate table."""
    p = (ctypes.c_double * 3)(*[float(v) for v in params])
    out = np.zeros((4, 4), dtype=np.complex128)
    k = ctypes.c_int()
    nc = ctypes.c_int()
    rc = lib().orc_gate_matrix(name.encode(), p, len(params), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(k), ctypes.byref(nc))
    if rc != 0:
        raise ValueError(f"unknown gate {name!r} or bad params {params!r}")
    d = 1 << k.value
    return out.reshape(-1)[: d * d].reshape(d, d).copy(), k.value, nc.value


def apply(psi: np.ndarray, matrix, targets, controls=(), cvals=None) -> None:
    """In-place dense gate application (targets[0] is the matrix LSB)."""
    n = _nqubits(psi)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    k = len(targets)
    if m.shape != (1 << k, 1 << k):
        raise ValueError("matrix shape does not match the number of targets")
    cv = None if cvals is None else _ints(cvals)
    rc = lib().orc_apply(psi.ctypes.data, n, m.ctypes.data, _ints(targets), k, _ints(controls), cv,
                         len(controls))
    if rc != 0:
        raise ValueError("invalid gate arguments")


def gperm_matrix(perm, diag) -> np.ndarray:
    """The dense 2^k x 2^k form of the generalized permutation matrix G = D P:
    row r has diag[r] in column perm[r] (perm None: the diagonal matrix)."""
    dg = np.asarray(diag, dtype=np.complex128)
    d = dg.shape[0]
    g = np.zeros((d, d), dtype=np.complex128)
    for r in range(d):
        g[r, r if perm is None else int(perm[r])] = dg[r]
    return g


def gperm_adjoint(perm, diag) -> tuple:
    """(perm', diag') with G' = D' P' equal to G^dagger: G^dagger maps the
    amplitude at row r of G's input column perm[r] back, so output q reads
    input r = perm^-1[q] with factor conj(diag[r])."""
    dg = np.asarray(diag, dtype=np.complex128)
    d = dg.shape[0]
    if perm is None:
        return None, np.conj(dg)
    inv = np.empty(d, dtype=np.int64)
    for r in range(d):
        inv[int(perm[r])] = r
    return inv, np.conj(dg[inv])


def apply_gperm(psi: np.ndarray, perm, diag, targets, controls=(), cvals=None, adjoint: bool = False) -> None:
    """In-place generalized permutation gate G = D P on `targets` (perm None:
    the diagonal gate diag): the amplitude at group offset r becomes
    diag[r] times the one at offset perm[r]."""
    n = _nqubits(psi)
    if adjoint:
        perm, diag = gperm_adjoint(perm, diag)
    dg = np.ascontiguousarray(diag, dtype=np.complex128)
    k = len(targets)
    if dg.shape != (1 << k,):
        raise ValueError("diagonal length does not match the number of targets")
    pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    if pm is not None and pm.shape != (1 << k,):
        raise ValueError("permutation length does not match the number of targets")
    cv = None if cvals is None else _ints(cvals)
    rc = lib().orc_apply_gperm(psi.ctypes.data, n, None if pm is None else pm.ctypes.data, dg.ctypes.data,
                               _ints(targets), k, _ints(controls), cv, len(controls))
    if rc != 0:
        raise ValueError("invalid generalized permutation gate arguments")


def apply_pauli_rotation(psi: np.ndarray, theta: float, term, controls=(), cvals=None) -> None:
    """psi <- exp(i theta P) psi for the Pauli string term = [(qubit, op)],
    on the indices whose controls hold their values (default 1)."""
    n = _nqubits(psi)
    qs = [q for q, _ in term]
    ops = "".join(o for _, o in term).encode()
    cv = None if cvals is None else _ints(cvals)
    rc = lib().orc_apply_pauli_rotation(psi.ctypes.data, n, float(theta), _ints(qs), ops, len(qs), _ints(controls), cv,
                                        len(controls))
    if rc != 0:
        raise ValueError("invalid Pauli rotation arguments")


def measure_probs(psi: np.ndarray, qubits) -> np.ndarray:
    """Unnormalised probabilities of the 2^m outcomes of measuring qubits
    (bit a of an outcome = the value of qubits[a])."""
    n = _nqubits(psi)
    out = np.zeros(1 << len(qubits), dtype=np.float64)
    rc = lib().orc_measure_probs(psi.ctypes.data, n, _ints(qubits), len(qubits),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("invalid measurement arguments")
    return out


def zbasis_probs(psi: np.ndarray, qubits) -> tuple:
    """(even, odd): unnormalised probabilities of the two eigenvalues +1
    (even parity of the measured bits) and -1 of the Z-product on qubits."""
    p = measure_probs(psi, qubits)
    par = np.array([bin(b).count("1") & 1 for b in range(p.size)])
    return float(p[par == 0].sum()), float(p[par == 1].sum())


def collapse(psi: np.ndarray, qubits, outcome: int = 0, norm: float = 1.0, parity: int | None = None) -> None:
    """Keep the amplitudes whose bits at qubits spell outcome (or, with
    parity 0/1, whose bits at qubits have that parity), divided by
    sqrt(norm); zero all others."""
    n = _nqubits(psi)
    rc = lib().orc_collapse(psi.ctypes.data, n, _ints(qubits), len(qubits), int(outcome),
                            -1 if parity is None else int(parity), float(norm))
    if rc != 0:
        raise ValueError("invalid collapse arguments")


def measure_zbasis(psi: np.ndarray, qubits, randnum: float, collapse_state: bool = True) -> int:
    """Parity outcome of measuring the Z-product on qubits with the uniform
    randnum in [0, 1): 0 (eigenvalue +1) if randnum * N < P_even, else 1;
    with collapse_state the state is projected and renormalised."""
    pe, po = zbasis_probs(psi, qubits)
    parity = 0 if randnum * (pe + po) < pe else 1
    if collapse_state:
        collapse(psi, qubits, norm=pe if parity == 0 else po, parity=parity)
    return parity


def batch_measure(psi: np.ndarray, qubits, randnum: float, collapse_state: bool = True) -> int:
    """Joint outcome of measuring qubits with the uniform randnum in [0, 1):
    the smallest b with randnum * N < C_b, C_b the running sum of the
    outcome probabilities in outcome order; with collapse_state the state is
    projected onto b and renormalised."""
    p = measure_probs(psi, qubits)
    c = np.cumsum(p)
    r = randnum * c[-1]
    b = int(np.searchsorted(c, r, side="right"))
    if collapse_state:
        collapse(psi, qubits, outcome=b, norm=float(p[b]))
    return b


def expect_matrix(psi: np.ndarray, matrix, targets) -> complex:
    """<psi| M |psi> / <psi|psi> for the dense observable M on targets."""
    n = _nqubits(psi)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    out = (ctypes.c_double * 3)()
    rc = lib().orc_expect_matrix(psi.ctypes.data, n, m.ctypes.data, _ints(targets), len(targets), out)
    if rc != 0:
        raise ValueError("invalid expectation arguments")
    return complex(out[0], out[1])


def swap_index_bits(psi: np.ndarray, pairs, mask_bits=(), mask_values=()) -> None:
    """Exchange index bits a and b for every pair (a, b) (all distinct), on
    the indices whose mask bits hold the mask values."""
    n = _nqubits(psi)
    flat = [q for p in pairs for q in p]
    rc = lib().orc_swap_index_bits(psi.ctypes.data, n, _ints(flat), len(pairs), _ints(mask_bits), _ints(mask_values),
                                   len(mask_bits))
    if rc != 0:
        raise ValueError("invalid index bit swap arguments")


def accessor_get(psi: np.ndarray, ordering, mask_bits=(), mask_values=(), begin: int = 0, end: int | None = None):
    """Amplitudes in the qubit order `ordering` (bit a of the output index is
    state bit ordering[a]) on the slice whose mask bits hold mask_values,
    output indices [begin, end)."""
    n = _nqubits(psi)
    if end is None:
        end = 1 << len(ordering)
    buf = np.zeros(max(0, end - begin), dtype=np.complex128)
    rc = lib().orc_accessor(psi.ctypes.data, n, _ints(ordering), len(ordering), _ints(mask_bits), _ints(mask_values),
                            len(mask_bits), buf.ctypes.data, begin, end, 0)
    if rc != 0:
        raise ValueError("invalid accessor arguments")
    return buf


def accessor_set(psi: np.ndarray, values, ordering, mask_bits=(), mask_values=(), begin: int = 0) -> None:
    """The inverse of accessor_get: writes values into those amplitudes."""
    n = _nqubits(psi)
    buf = np.ascontiguousarray(values, dtype=np.complex128)
    rc = lib().orc_accessor(psi.ctypes.data, n, _ints(ordering), len(ordering), _ints(mask_bits), _ints(mask_values),
                            len(mask_bits), buf.ctypes.data, begin, begin + buf.size, 1)
    if rc != 0:
        raise ValueError("invalid accessor arguments")


def apply_gate(psi: np.ndarray, gate) -> None:
    """Apply one workload gate (name, qubits, params)."""
    name, qubits, params = gate
    if name in ("mat", "mat_dg"):
        m = np.asarray(params, dtype=np.complex128)
        if name == "mat_dg":
            m = np.conj(m).T
        apply(psi, m, qubits)
        return
    m, k, nc = gate_matrix(name, params)
    if len(qubits) != k + nc:
        raise ValueError(f"gate {name} takes {k + nc} qubits")
    apply(psi, m, qubits[nc:], qubits[:nc])


def basis_state(n: int, x: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def run(n: int, gates, basis: int = 0, psi: np.ndarray | None = None) -> np.ndarray:
    """The ordered product of the gates applied to |basis> (or to a copy of psi)."""
    psi = basis_state(n, basis) if psi is None else np.array(psi, dtype=np.complex128, copy=True)
    for g in gates:
        apply_gate(psi, g)
    return psi


def norm(psi: np.ndarray) -> float:
    """sum_i |psi_i|^2 (compensated, FP64)."""
    return float(lib().orc_norm(psi.ctypes.data, _nqubits(psi)))


def expect_pauli(psi: np.ndarray, term) -> float:
    """<psi|P|psi>/<psi|psi> for a Pauli string given as [(qubit, 'X'|'Y'|'Z'), ...]."""
    n = _nqubits(psi)
    qs = [int(q) for q, _ in term]
    ops = "".join(o for _, o in term)
    out = (ctypes.c_double * 3)()
    rc = lib().orc_expect_pauli(psi.ctypes.data, n, _ints(qs), ops.encode(), len(qs), out)
    if rc != 0:
        raise ValueError("invalid Pauli term")
    return float(out[0])


def expect_pauli_full(psi: np.ndarray, term) -> tuple:
    """(real part, imaginary part, norm) of the expectation."""
    n = _nqubits(psi)
    qs = [int(q) for q, _ in term]
    ops = "".join(o for _, o in term)
    out = (ctypes.c_double * 3)()
    rc = lib().orc_expect_pauli(psi.ctypes.data, n, _ints(qs), ops.encode(), len(qs), out)
    if rc != 0:
        raise ValueError("invalid Pauli term")
    return float(out[0]), float(out[1]), float(out[2])


def sample(psi: np.ndarray, u, bit_ordering=None, return_cdf: bool = False):
    """Outcomes for the uniforms ``u`` (upper-bound inverse CDF, input order)."""
    n = _nqubits(psi)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(u.size, dtype=np.uint64)
    cdf = np.zeros(psi.size, dtype=np.float64) if return_cdf else None
    bo = None if bit_ordering is None else _ints(bit_ordering)
    nb = 0 if bit_ordering is None else len(bit_ordering)
    rc = lib().orc_sample(psi.ctypes.data, n, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), u.size,
                          bo, nb, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                          None if cdf is None else cdf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("invalid sampling arguments (uniforms must lie in [0, 1))")
    return (out, cdf) if return_cdf else out


def threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads for the oracle's parallel loops (n >= 1)."""
    lib().orc_set_threads(int(n))


def fidelity(a: np.ndarray, b: np.ndarray) -> float:
    """|<a|b>|^2 / (<a|a><b|b>) in FP64."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ov = np.vdot(a, b)
    return float(abs(ov) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
