"""Python binding of libsv, the MI355X state-vector simulation core.

A thin ctypes layer over the C ABI declared in ``include/sv.h``: the
``sv_*`` functions below have the names of the C entry points and only
marshal arguments; every step of the computation runs in libsv's HIP kernels
(or, for gate fusion and the gate table, in its host C++).  PyTorch provides
device memory and streams: states are ``torch`` tensors on ``cuda:0`` whose
storage libsv borrows, and handles run on torch streams.

Importing the package loads ``libsv.so`` and raises ``ImportError`` if it has
not been built (``python paper_2308_01999_amd/build.py``): there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsv.so is not built at {LIB_PATH}; run paper_2308_01999_amd/build.py")

# torch ships its own HIP and HSA runtimes (soname libamdhip64.so.7, like
# ROCm's).  Loading torch first makes libsv bind to that same runtime; loading
# libsv first would bring in a second HIP/HSA runtime whose device enumeration
# fails once torch's has opened the GPU.
import torch  # noqa: E402,F401

_L = ctypes.CDLL(LIB_PATH)

SV_OK, SV_ERR_INVALID_VALUE, SV_ERR_OUT_OF_MEMORY, SV_ERR_NOT_SUPPORTED, SV_ERR_DEVICE, SV_ERR_INTERNAL = range(6)
SV_C64, SV_C128 = 0, 1
SV_MAX_QUBITS = 36
SV_MAX_TARGETS = 10
SV_SAMPLE_NOALLOC_MAX_QUBITS = 28

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pd = ctypes.POINTER(ctypes.c_double)
_pu64 = ctypes.POINTER(ctypes.c_uint64)


class sv_gate_t(ctypes.Structure):
    _fields_ = [("n_targets", _i32), ("targets", _pi32), ("matrix", _pd), ("n_controls", _i32),
                ("controls", _pi32), ("control_values", _pi32), ("adjoint", _i32)]


class sv_pauli_term_t(ctypes.Structure):
    _fields_ = [("n_ops", _i32), ("qubits", _pi32), ("ops", ctypes.c_char_p)]


class sv_batch_size_plan_t(ctypes.Structure):
    _fields_ = [("max_fused_qubits", _i32), ("level_path", _i32), ("tiles_per_wg", _i32), ("spread", _i32),
                ("tuned", _i32)]


# name -> (argtypes); every entry point returns sv_status_t except the two
# string getters
_SIGS = {
    "sv_handle_create": [ctypes.POINTER(_vp), _vp, ctypes.c_size_t],
    "sv_handle_destroy": [_vp],
    "sv_handle_set_stream": [_vp, _vp],
    "sv_handle_set_tile_mode": [_vp, _i32],
    "sv_handle_set_batch_level_qubits": [_vp, _i32],
    "sv_graph_create": [_vp, _vp, ctypes.POINTER(_vp)],
    "sv_graph_launch": [_vp],
    "sv_graph_destroy": [_vp],
    "sv_sync": [_vp],
    "sv_create": [_vp, _i32, ctypes.c_int, _vp, ctypes.POINTER(_vp)],
    "sv_destroy": [_vp],
    "sv_state_device_ptr": [_vp, ctypes.POINTER(_vp)],
    "sv_set_basis_state": [_vp, _u64],
    "sv_apply_matrix": [_vp, _pd, _pi32, _i32, _pi32, _pi32, _i32, _i32],
    "sv_apply_gen_permutation": [_vp, ctypes.POINTER(ctypes.c_int64), _pd, _pi32, _i32, _pi32, _pi32, _i32, _i32],
    "sv_gate_matrix": [ctypes.c_char_p, _pd, _i32, _pd, _pi32, _pi32],
    "sv_fuse_gates": [ctypes.POINTER(sv_gate_t), _i32, _i32, ctypes.POINTER(_vp)],
    "sv_fuse_gate_list": [_pi32, _pi32, _pd, _i32, _i32, ctypes.POINTER(_vp)],
    "sv_fuse_gates_diag": [ctypes.POINTER(sv_gate_t), _i32, _i32, _i32, ctypes.POINTER(_vp)],
    "sv_fuse_gate_list_diag": [_pi32, _pi32, _pd, _i32, _i32, _i32, ctypes.POINTER(_vp)],
    "sv_fused_block_is_diagonal": [_vp, _i32, _pi32],
    "sv_fuse_gates_coupled": [ctypes.POINTER(sv_gate_t), _i32, _i32, ctypes.POINTER(_vp)],
    "sv_fuse_gate_list_coupled": [_pi32, _pi32, _pd, _i32, _i32, ctypes.POINTER(_vp)],
    "sv_fused_block_coupling": [_vp, _i32, _pi32, _pi32, _pd],
    "sv_fused_count": [_vp, _pi32],
    "sv_fused_block": [_vp, _i32, _pi32, _pi32, _pd],
    "sv_fused_free": [_vp],
    "sv_apply_fused": [_vp, _vp],
    "sv_apply_fused_range": [_vp, _vp, _i32, _i32],
    "sv_norm": [_vp, _pd],
    "sv_renormalize": [_vp, _pd],
    "sv_expect_pauli": [_vp, ctypes.POINTER(sv_pauli_term_t), _i32, _pd],
    "sv_sample": [_vp, _pd, _i64, _pi32, _i32, _pu64],
    "sv_sample_noalloc": [_vp, _pd, _i64, _pi32, _i32, _pu64],
    "sv_sample_device": [_vp, _vp, _i64, _pi32, _i32, _vp],
    "sv_apply_pauli_rotation": [_vp, ctypes.c_double, ctypes.POINTER(sv_pauli_term_t), _pi32, _pi32, _i32],
    "sv_measure_probabilities": [_vp, _pi32, _i32, _pd],
    "sv_zbasis_probabilities": [_vp, _pi32, _i32, _pd, _pd],
    "sv_collapse": [_vp, _pi32, _i32, _u64, ctypes.c_double],
    "sv_collapse_zbasis": [_vp, _pi32, _i32, _i32, ctypes.c_double],
    "sv_measure_zbasis": [_vp, _pi32, _i32, ctypes.c_double, _i32, _pi32],
    "sv_batch_measure": [_vp, _pi32, _i32, ctypes.c_double, _i32, _pu64],
    "sv_expect_matrix": [_vp, _pd, _pi32, _i32, _pd],
    "sv_swap_index_bits": [_vp, _pi32, _i32, _pi32, _pi32, _i32],
    "sv_accessor_get": [_vp, _pi32, _i32, _pi32, _pi32, _i32, _vp, _i64, _i64],
    "sv_accessor_set": [_vp, _pi32, _i32, _pi32, _pi32, _i32, _vp, _i64, _i64],
    "sv_copy_to_host": [_vp, _vp, _u64, _u64],
    "sv_copy_from_host": [_vp, _vp, _u64, _u64],
    "sv_batch_create": [_vp, _i32, _pi32, _pi32, _pi32, _pi32, _pd, _pi32, _pu64, _i32, ctypes.POINTER(_vp)],
    "sv_batch_state_layout": [_vp, _pu64, _pu64],
    "sv_batch_info": [_vp, _i32, _pi32, _pi32],
    "sv_batch_plan": [_vp, _i32, ctypes.POINTER(sv_batch_size_plan_t)],
    "sv_batch_host_times": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "sv_batch_run": [_vp, _vp, _pd, _pd, _pd],
    "sv_batch_destroy": [_vp],
    "sv_set_hbm_budget": [_u64],
    "sv_hbm_usage": [_pu64, _pu64],
}
for _name, _args in _SIGS.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_L.sv_last_error.argtypes = []
_L.sv_last_error.restype = ctypes.c_char_p
_L.sv_version.argtypes = []
_L.sv_version.restype = ctypes.c_char_p

EXPORTED = sorted(list(_SIGS) + ["sv_last_error", "sv_version"])


class SVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsv status {status}: {msg}")
        self.status = status


def _check(status: int) -> None:
    if status != SV_OK:
        raise SVError(status, _L.sv_last_error().decode(errors="replace"))


def _i32arr(seq):
    seq = [int(v) for v in seq]
    return (ctypes.c_int32 * max(1, len(seq)))(*seq)


def _mat(m) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_pd)


# --------------------------------------------------------------------------
# 1:1 entry points
# --------------------------------------------------------------------------

def sv_version() -> str:
    return _L.sv_version().decode()


def sv_last_error() -> str:
    return _L.sv_last_error().decode(errors="replace")


def sv_set_hbm_budget(budget_bytes: int) -> None:
    """Cap on the device memory libsv allocates itself (0: no cap)."""
    _check(_L.sv_set_hbm_budget(int(budget_bytes)))


def sv_hbm_usage() -> tuple:
    """(bytes libsv has allocated, cap or 0)."""
    used = ctypes.c_uint64()
    cap = ctypes.c_uint64()
    _check(_L.sv_hbm_usage(ctypes.byref(used), ctypes.byref(cap)))
    return used.value, cap.value


def sv_handle_create(stream_ptr: int = 0, workspace_bytes: int = 0) -> int:
    h = _vp()
    _check(_L.sv_handle_create(ctypes.byref(h), _vp(stream_ptr or None), workspace_bytes))
    return h.value


def sv_handle_destroy(h: int) -> None:
    _check(_L.sv_handle_destroy(_vp(h)))


def sv_handle_set_stream(h: int, stream_ptr: int) -> None:
    _check(_L.sv_handle_set_stream(_vp(h), _vp(stream_ptr or None)))


SV_TILE_AUTO, SV_TILE_NARROW, SV_TILE_WIDE, SV_TILE_SPREAD = 0, 1, 2, 3
TILE_WARM_SWEEPS = 64  # SV_TILE_WARM_SWEEPS


def sv_handle_set_tile_mode(h: int, mode: int) -> None:
    _check(_L.sv_handle_set_tile_mode(_vp(h), _i32(mode)))


SV_BATCH_LEVEL_MIN_QUBITS, SV_BATCH_LEVEL_DEFAULT, SV_BATCH_LEVEL_NONE = 13, 15, 31


def sv_handle_set_batch_level_qubits(h: int, n_qubits: int) -> None:
    _check(_L.sv_handle_set_batch_level_qubits(_vp(h), _i32(n_qubits)))


def sv_graph_create(s: int, f: int) -> int:
    out = _vp()
    _check(_L.sv_graph_create(_vp(s), _vp(f), ctypes.byref(out)))
    return out.value


def sv_graph_launch(g: int) -> None:
    _check(_L.sv_graph_launch(_vp(g)))


def sv_graph_destroy(g: int) -> None:
    _check(_L.sv_graph_destroy(_vp(g)))


def sv_sync(h: int) -> None:
    _check(_L.sv_sync(_vp(h)))


def sv_create(h: int, n_qubits: int, dtype: int, device_ptr: int = 0) -> int:
    s = _vp()
    _check(_L.sv_create(_vp(h), n_qubits, dtype, _vp(device_ptr or None), ctypes.byref(s)))
    return s.value


def sv_destroy(s: int) -> None:
    _check(_L.sv_destroy(_vp(s)))


def sv_state_device_ptr(s: int) -> int:
    p = _vp()
    _check(_L.sv_state_device_ptr(_vp(s), ctypes.byref(p)))
    return p.value


def sv_set_basis_state(s: int, x: int) -> None:
    _check(_L.sv_set_basis_state(_vp(s), x))


def sv_apply_matrix(s: int, matrix, targets, controls=(), control_values=None, adjoint: bool = False) -> None:
    m = _mat(matrix)
    cv = None if control_values is None else _i32arr(control_values)
    _check(_L.sv_apply_matrix(_vp(s), m.ctypes.data_as(_pd), _i32arr(targets), len(targets),
                              _i32arr(controls), cv, len(controls), int(bool(adjoint))))


def sv_apply_gen_permutation(s: int, perm, diag, targets, controls=(), control_values=None,
                             adjoint: bool = False) -> None:
    """G = D P on targets: the amplitude at group offset r becomes diag[r]
    times the one at offset perm[r] (perm None: the diagonal gate diag)."""
    dg = np.ascontiguousarray(diag, dtype=np.complex128)
    pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    cv = None if control_values is None else _i32arr(control_values)
    _check(_L.sv_apply_gen_permutation(_vp(s), None if pm is None else pm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       dg.ctypes.data_as(_pd), _i32arr(targets), len(targets), _i32arr(controls), cv,
                                       len(controls), int(bool(adjoint))))


def sv_gate_matrix(name: str, params=()) -> tuple:
    """(matrix [2^k, 2^k] complex128, n_targets, n_controls) of a named gate."""
    p = (ctypes.c_double * 3)(*[float(v) for v in params])
    out = np.zeros(16, dtype=np.complex128)
    nt = _i32()
    nc = _i32()
    _check(_L.sv_gate_matrix(name.encode(), p, len(params), _dptr(out), ctypes.byref(nt), ctypes.byref(nc)))
    d = 1 << nt.value
    return out[: d * d].reshape(d, d).copy(), nt.value, nc.value


def _gate_struct(targets, matrix, controls=(), control_values=None, adjoint=False, keep=None):
    m = _mat(matrix)
    t = _i32arr(targets)
    c = _i32arr(controls)
    cv = None if control_values is None else _i32arr(control_values)
    keep.extend([m, t, c, cv])
    return sv_gate_t(len(targets), t, m.ctypes.data_as(_pd), len(controls), c, cv, int(bool(adjoint)))


def _gate_array(gates, keep):
    """Entries (targets, matrix, controls, control_values[, adjoint]) as a
    sv_gate_t array."""
    arr = (sv_gate_t * max(1, len(gates)))()
    for i, e in enumerate(gates):
        t, m, c, cv = e[:4]
        arr[i] = _gate_struct(t, m, c, cv, e[4] if len(e) > 4 else False, keep)
    return arr


def sv_fuse_gates(gates, max_fused_qubits: int) -> int:
    """gates: list of (targets, matrix, controls, control_values[, adjoint])."""
    keep = []
    arr = _gate_array(gates, keep)
    f = _vp()
    _check(_L.sv_fuse_gates(arr, len(gates), max_fused_qubits, ctypes.byref(f)))
    return f.value


def sv_fuse_gates_diag(gates, max_fused_qubits: int, max_fused_diagonal_qubits: int) -> int:
    """As sv_fuse_gates, with diagonal blocks of up to max_fused_diagonal_qubits."""
    keep = []
    arr = _gate_array(gates, keep)
    f = _vp()
    _check(_L.sv_fuse_gates_diag(arr, len(gates), max_fused_qubits, max_fused_diagonal_qubits, ctypes.byref(f)))
    return f.value


def sv_fuse_gates_coupled(gates, max_fused_qubits: int) -> int:
    """Coupled fusion of sv_gate_t-style gates (see sv.h)."""
    keep = []
    arr = _gate_array(gates, keep)
    f = _vp()
    _check(_L.sv_fuse_gates_coupled(arr, len(gates), max_fused_qubits, ctypes.byref(f)))
    return f.value


GATE_CODES = {"u3": 0, "h": 1, "x": 2, "y": 3, "z": 4, "cx": 5, "cz": 6, "cp": 7, "swap": 8}
SV_GATE_ADJOINT = 256
_GATE_CODE_OF = {**GATE_CODES, **{k + "_dg": v | SV_GATE_ADJOINT for k, v in GATE_CODES.items()}}


def sv_fuse_gate_list(codes, qubits, params, max_fused_qubits: int) -> int:
    """codes int32[G], qubits int32[G, 2], params float64[G, 3] (see sv.h)."""
    c = np.ascontiguousarray(codes, dtype=np.int32)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.float64)
    if q.shape != (c.size, 2) or p.shape != (c.size, 3):
        raise ValueError("qubits must be [G, 2] and params [G, 3]")
    f = _vp()
    _check(_L.sv_fuse_gate_list(c.ctypes.data_as(_pi32), q.ctypes.data_as(_pi32), _dptr(p), c.size,
                                max_fused_qubits, ctypes.byref(f)))
    return f.value


def sv_fuse_gate_list_diag(codes, qubits, params, max_fused_qubits: int, max_fused_diagonal_qubits: int) -> int:
    c = np.ascontiguousarray(codes, dtype=np.int32)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.float64)
    if q.shape != (c.size, 2) or p.shape != (c.size, 3):
        raise ValueError("qubits must be [G, 2] and params [G, 3]")
    f = _vp()
    _check(_L.sv_fuse_gate_list_diag(c.ctypes.data_as(_pi32), q.ctypes.data_as(_pi32), _dptr(p), c.size,
                                     max_fused_qubits, max_fused_diagonal_qubits, ctypes.byref(f)))
    return f.value


def sv_fuse_gate_list_coupled(codes, qubits, params, max_fused_qubits: int) -> int:
    c = np.ascontiguousarray(codes, dtype=np.int32)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.float64)
    if q.shape != (c.size, 2) or p.shape != (c.size, 3):
        raise ValueError("qubits must be [G, 2] and params [G, 3]")
    f = _vp()
    _check(_L.sv_fuse_gate_list_coupled(c.ctypes.data_as(_pi32), q.ctypes.data_as(_pi32), _dptr(p), c.size,
                                        max_fused_qubits, ctypes.byref(f)))
    return f.value


def sv_fused_block_coupling(f: int, i: int, k: int):
    """(coupled qubits, phases [k, n_coupled]) of block i (k its qubit count)."""
    nc = _i32()
    q = (ctypes.c_int32 * SV_MAX_QUBITS)()
    _check(_L.sv_fused_block_coupling(_vp(f), i, ctypes.byref(nc), q, None))
    ph = np.zeros((k, nc.value), dtype=np.float64)
    if nc.value:
        _check(_L.sv_fused_block_coupling(_vp(f), i, ctypes.byref(nc), q, _dptr(ph)))
    return [int(q[c]) for c in range(nc.value)], ph


def gate_list_arrays(gates):
    """Workload gates (named gates only) -> (codes, qubits, params) arrays."""
    G = len(gates)
    try:
        codes = np.fromiter((_GATE_CODE_OF[g[0]] for g in gates), dtype=np.int32, count=G)
    except KeyError as e:
        raise KeyError(f"unknown gate {e.args[0]!r}") from None
    qubits = np.fromiter((x for g in gates for x in (g[1][0], g[1][1] if len(g[1]) > 1 else 0)),
                         dtype=np.int32, count=2 * G).reshape(G, 2)
    pad = (0.0, 0.0, 0.0)
    params = np.fromiter((x for g in gates for x in (tuple(g[2]) + pad)[:3]),
                         dtype=np.float64, count=3 * G).reshape(G, 3)
    return codes, qubits, params


def sv_fused_count(f: int) -> int:
    n = _i32()
    _check(_L.sv_fused_count(_vp(f), ctypes.byref(n)))
    return n.value


def sv_fused_block_is_diagonal(f: int, i: int) -> bool:
    d = _i32()
    _check(_L.sv_fused_block_is_diagonal(_vp(f), i, ctypes.byref(d)))
    return bool(d.value)


def sv_fused_block(f: int, i: int) -> tuple:
    """(targets, matrix [2^k, 2^k]) of a dense block, (targets, diagonal
    [2^k]) of a diagonal one."""
    k = _i32()
    t = (ctypes.c_int32 * SV_MAX_TARGETS)()
    _check(_L.sv_fused_block(_vp(f), i, ctypes.byref(k), t, None))
    d = 1 << k.value
    if sv_fused_block_is_diagonal(f, i):
        v = np.zeros(d, dtype=np.complex128)
        _check(_L.sv_fused_block(_vp(f), i, ctypes.byref(k), t, _dptr(v)))
        return tuple(t[: k.value]), v
    m = np.zeros(d * d, dtype=np.complex128)
    _check(_L.sv_fused_block(_vp(f), i, ctypes.byref(k), t, _dptr(m)))
    return tuple(t[: k.value]), m.reshape(d, d)


def sv_fused_free(f: int) -> None:
    _check(_L.sv_fused_free(_vp(f)))


def sv_apply_fused(s: int, f: int) -> None:
    _check(_L.sv_apply_fused(_vp(s), _vp(f)))


def sv_apply_fused_range(s: int, f: int, first: int, count: int) -> None:
    _check(_L.sv_apply_fused_range(_vp(s), _vp(f), first, count))


def sv_norm(s: int) -> float:
    out = ctypes.c_double()
    _check(_L.sv_norm(_vp(s), ctypes.byref(out)))
    return out.value


def sv_renormalize(s: int) -> float:
    out = ctypes.c_double()
    _check(_L.sv_renormalize(_vp(s), ctypes.byref(out)))
    return out.value


def sv_expect_pauli(s: int, terms) -> np.ndarray:
    """terms: list of [(qubit, 'X'|'Y'|'Z'|'I'), ...]."""
    keep = []
    arr = (sv_pauli_term_t * max(1, len(terms)))()
    for i, term in enumerate(terms):
        q = _i32arr([qq for qq, _ in term])
        ops = "".join(o for _, o in term).encode()
        keep.extend([q, ops])
        arr[i] = sv_pauli_term_t(len(term), q, ops)
    out = np.zeros(max(1, len(terms)), dtype=np.float64)
    _check(_L.sv_expect_pauli(_vp(s), arr, len(terms), _dptr(out)))
    return out[: len(terms)]


def sv_apply_pauli_rotation(s: int, theta: float, term, controls=(), control_values=None) -> None:
    """psi <- exp(i theta P) psi, term = [(qubit, 'I'|'X'|'Y'|'Z'), ...]."""
    q = _i32arr([qq for qq, _ in term])
    ops = "".join(o for _, o in term).encode()
    t = sv_pauli_term_t(len(term), q, ops)
    cv = None if control_values is None else _i32arr(control_values)
    _check(_L.sv_apply_pauli_rotation(_vp(s), float(theta), ctypes.byref(t), _i32arr(controls), cv, len(controls)))


def sv_measure_probabilities(s: int, qubits) -> np.ndarray:
    out = np.zeros(1 << len(qubits), dtype=np.float64)
    _check(_L.sv_measure_probabilities(_vp(s), _i32arr(qubits), len(qubits), _dptr(out)))
    return out


def sv_zbasis_probabilities(s: int, qubits) -> tuple:
    e, o = ctypes.c_double(), ctypes.c_double()
    _check(_L.sv_zbasis_probabilities(_vp(s), _i32arr(qubits), len(qubits), ctypes.byref(e), ctypes.byref(o)))
    return e.value, o.value


def sv_collapse(s: int, qubits, outcome: int, norm: float) -> None:
    _check(_L.sv_collapse(_vp(s), _i32arr(qubits), len(qubits), int(outcome), float(norm)))


def sv_collapse_zbasis(s: int, qubits, parity: int, norm: float) -> None:
    _check(_L.sv_collapse_zbasis(_vp(s), _i32arr(qubits), len(qubits), int(parity), float(norm)))


def sv_measure_zbasis(s: int, qubits, randnum: float, collapse: bool = True) -> int:
    p = _i32()
    _check(_L.sv_measure_zbasis(_vp(s), _i32arr(qubits), len(qubits), float(randnum), int(bool(collapse)),
                                ctypes.byref(p)))
    return p.value


def sv_batch_measure(s: int, qubits, randnum: float, collapse: bool = True) -> int:
    o = _u64()
    _check(_L.sv_batch_measure(_vp(s), _i32arr(qubits), len(qubits), float(randnum), int(bool(collapse)),
                               ctypes.byref(o)))
    return o.value


def sv_expect_matrix(s: int, matrix, targets) -> complex:
    m = _mat(matrix)
    out = np.zeros(2, dtype=np.float64)
    _check(_L.sv_expect_matrix(_vp(s), m.ctypes.data_as(_pd), _i32arr(targets), len(targets), _dptr(out)))
    return complex(out[0], out[1])


def sv_swap_index_bits(s: int, pairs, mask_bits=(), mask_values=()) -> None:
    flat = [int(q) for p in pairs for q in p]
    _check(_L.sv_swap_index_bits(_vp(s), _i32arr(flat), len(pairs), _i32arr(mask_bits), _i32arr(mask_values),
                                 len(mask_bits)))


def sv_accessor_get(s: int, dtype: int, ordering, mask_bits=(), mask_values=(), begin: int = 0,
                    end: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """out (optional): a C-contiguous array of end - begin elements of the
    state's dtype to fill (reusing it spares the host the page faults of a
    fresh array)."""
    if end is None:
        end = 1 << len(ordering)
    want = np.complex64 if dtype == SV_C64 else np.complex128
    if out is None:
        out = np.zeros(max(0, end - begin), dtype=want)
    elif out.dtype != want or out.size != max(0, end - begin) or not out.flags["C_CONTIGUOUS"]:
        raise ValueError("out must be a C-contiguous array of end - begin elements of the state's dtype")
    _check(_L.sv_accessor_get(_vp(s), _i32arr(ordering), len(ordering), _i32arr(mask_bits), _i32arr(mask_values),
                              len(mask_bits), out.ctypes.data, begin, end))
    return out


def sv_accessor_set(s: int, dtype: int, values, ordering, mask_bits=(), mask_values=(), begin: int = 0) -> None:
    v = np.ascontiguousarray(values, dtype=np.complex64 if dtype == SV_C64 else np.complex128)
    _check(_L.sv_accessor_set(_vp(s), _i32arr(ordering), len(ordering), _i32arr(mask_bits), _i32arr(mask_values),
                              len(mask_bits), v.ctypes.data, begin, begin + v.size))


def sv_sample(s: int, uniforms, bit_ordering=None) -> np.ndarray:
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.zeros(max(1, u.size), dtype=np.uint64)
    bo = None if bit_ordering is None else _i32arr(bit_ordering)
    nb = 0 if bit_ordering is None else len(bit_ordering)
    _check(_L.sv_sample(_vp(s), _dptr(u), u.size, bo, nb, out.ctypes.data_as(_pu64)))
    return out[: u.size]


def sv_sample_noalloc(s: int, uniforms, bit_ordering=None) -> np.ndarray:
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.zeros(max(1, u.size), dtype=np.uint64)
    bo = None if bit_ordering is None else _i32arr(bit_ordering)
    nb = 0 if bit_ordering is None else len(bit_ordering)
    _check(_L.sv_sample_noalloc(_vp(s), _dptr(u), u.size, bo, nb, out.ctypes.data_as(_pu64)))
    return out[: u.size]


def sv_sample_device(s: int, uniforms_ptr: int, n_shots: int, out_ptr: int, bit_ordering=None) -> None:
    """sv_sample_device: uniforms_ptr and out_ptr are device addresses (for
    example torch CUDA tensors' data_ptr(): float64 and 64-bit integers)."""
    bo = None if bit_ordering is None else _i32arr(bit_ordering)
    nb = 0 if bit_ordering is None else len(bit_ordering)
    _check(_L.sv_sample_device(_vp(s), _vp(uniforms_ptr), n_shots, bo, nb, _vp(out_ptr)))


def sv_copy_to_host(s: int, dst: np.ndarray, first: int = 0, count: int | None = None) -> None:
    count = dst.size if count is None else count
    _check(_L.sv_copy_to_host(_vp(s), dst.ctypes.data, first, count))


def sv_copy_from_host(s: int, src: np.ndarray, first: int = 0) -> None:
    src = np.ascontiguousarray(src)
    _check(_L.sv_copy_from_host(_vp(s), src.ctypes.data, first, src.size))


# --------------------------------------------------------------------------
# small conveniences over the entry points (no arithmetic of the method)
# --------------------------------------------------------------------------

DTYPES = {"c64": SV_C64, "c128": SV_C128}
NP_DTYPES = {SV_C64: np.complex64, SV_C128: np.complex128}


class Handle:
    """A libsv handle on a torch stream (default: torch's current stream)."""

    def __init__(self, stream=None, workspace_bytes: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libsv needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = sv_handle_create(self.stream.cuda_stream, workspace_bytes)

    def sync(self):
        sv_sync(self.h)

    def set_tile_mode(self, mode: int) -> None:
        sv_handle_set_tile_mode(self.h, mode)

    def set_batch_level_qubits(self, n_qubits: int) -> None:
        sv_handle_set_batch_level_qubits(self.h, n_qubits)

    def close(self):
        if self.h:
            sv_handle_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """A state of n qubits in a torch tensor that libsv borrows."""

    def __init__(self, handle: Handle, n: int, dtype: str = "c64", basis: int = 0, tensor=None):
        import torch
        self.handle = handle
        self.n = n
        self.dt = DTYPES[dtype]
        tdt = torch.complex64 if self.dt == SV_C64 else torch.complex128
        if tensor is None:
            with torch.cuda.stream(handle.stream):
                tensor = torch.empty(1 << n, dtype=tdt, device="cuda")
        if tensor.dtype != tdt or tensor.numel() != (1 << n) or not tensor.is_contiguous():
            raise ValueError("tensor must be contiguous with 2^n elements of the state's dtype")
        self.tensor = tensor
        self.s = sv_create(handle.h, n, self.dt, tensor.data_ptr())
        if basis is not None:
            sv_set_basis_state(self.s, basis)

    def apply_matrix(self, matrix, targets, controls=(), control_values=None, adjoint=False):
        sv_apply_matrix(self.s, matrix, targets, controls, control_values, adjoint)

    def apply_gen_permutation(self, perm, diag, targets, controls=(), control_values=None, adjoint=False):
        sv_apply_gen_permutation(self.s, perm, diag, targets, controls, control_values, adjoint)

    def apply_gate(self, gate):
        """One workload gate (name, qubits, params) via the library's gate table."""
        name, qubits, params = gate
        if name in ("mat", "mat_dg"):
            sv_apply_matrix(self.s, params, qubits, adjoint=(name == "mat_dg"))
            return
        m, nt, nc = sv_gate_matrix(name, params)
        sv_apply_matrix(self.s, m, qubits[nc:], qubits[:nc])

    def run(self, gates, max_fused_qubits: int | None = None, coupled: bool = False):
        if not max_fused_qubits:
            for g in gates:
                self.apply_gate(g)
            return None
        f = fuse(gates, max_fused_qubits, coupled=coupled)
        try:
            sv_apply_fused(self.s, f.f)
            return f.count
        finally:
            f.free()

    def norm(self):
        return sv_norm(self.s)

    def expect(self, terms):
        return sv_expect_pauli(self.s, terms)

    def sample(self, uniforms, bit_ordering=None):
        return sv_sample(self.s, uniforms, bit_ordering)

    def to_numpy(self):
        out = np.empty(1 << self.n, dtype=NP_DTYPES[self.dt])
        sv_copy_to_host(self.s, out)
        return out

    def close(self):
        if self.s:
            sv_destroy(self.s)
            self.s = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gate_entries(gates):
    """Workload gates -> (targets, matrix, controls, control_values, adjoint)
    via the library's gate table; a "mat_dg" gate passes its matrix with the
    adjoint flag set."""
    out = []
    for name, qubits, params in gates:
        if name in ("mat", "mat_dg"):
            out.append((tuple(qubits), _mat(params), (), None, name == "mat_dg"))
        else:
            m, nt, nc = sv_gate_matrix(name, params)
            out.append((tuple(qubits[nc:]), m, tuple(qubits[:nc]), None, False))
    return out


class Fused:
    def __init__(self, f: int):
        self.f = f
        self.count = sv_fused_count(f)

    def blocks(self):
        return [sv_fused_block(self.f, i) for i in range(self.count)]

    def couplings(self):
        """Per block: (coupled qubits, phases [k, n_coupled])."""
        out = []
        for i in range(self.count):
            t, _ = sv_fused_block(self.f, i)
            out.append(sv_fused_block_coupling(self.f, i, len(t)))
        return out

    def free(self):
        if self.f:
            sv_fused_free(self.f)
            self.f = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Graph:
    """A fused program recorded into a HIP graph for one state; launch()
    replays it on the state (async, on the handle's stream)."""

    def __init__(self, state, gates, max_fused_qubits: int = 5, max_fused_diagonal_qubits: int = 0,
                 coupled: bool = False):
        f = fuse(gates, max_fused_qubits, max_fused_diagonal_qubits, coupled)
        try:
            self.blocks = f.count
            self.g = sv_graph_create(state.s, f.f)
        finally:
            f.free()

    def launch(self) -> None:
        sv_graph_launch(self.g)

    def close(self) -> None:
        if self.g:
            sv_graph_destroy(self.g)
            self.g = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fuse(gates, max_fused_qubits: int, max_fused_diagonal_qubits: int = 0, coupled: bool = False) -> Fused:
    """Fused blocks of a workload circuit; with max_fused_diagonal_qubits > 0
    diagonal gates also form diagonal blocks of up to that many qubits; with
    coupled, phase gates are deferred into the phase couplings of later
    blocks (sv_fuse_gate_list_coupled)."""
    named = not any(g[0] in ("mat", "mat_dg") for g in gates)
    if coupled:
        if named:
            return Fused(sv_fuse_gate_list_coupled(*gate_list_arrays(gates), max_fused_qubits))
        return Fused(sv_fuse_gates_coupled(gate_entries(gates), max_fused_qubits))
    if not named:
        if max_fused_diagonal_qubits:
            return Fused(sv_fuse_gates_diag(gate_entries(gates), max_fused_qubits, max_fused_diagonal_qubits))
        return Fused(sv_fuse_gates(gate_entries(gates), max_fused_qubits))
    if max_fused_diagonal_qubits:
        return Fused(sv_fuse_gate_list_diag(*gate_list_arrays(gates), max_fused_qubits, max_fused_diagonal_qubits))
    return Fused(sv_fuse_gate_list(*gate_list_arrays(gates), max_fused_qubits))


# --------------------------------------------------------------------------
# batched circuits
# --------------------------------------------------------------------------

def z_mask(qubits) -> int:
    """Bit mask of a Z-type Pauli string acting on `qubits`."""
    m = 0
    for q in qubits:
        m |= 1 << int(q)
    return m


def sv_batch_create(h: int, n_qubits, circuits, z_masks, max_fused_qubits: int = 0) -> int:
    """n_qubits[i], circuits[i] (workload gate list of named gates),
    z_masks[i] (list of Z-type term masks)."""
    nc = len(n_qubits)
    arrays = [gate_list_arrays(g) for g in circuits]
    goff = np.zeros(nc + 1, dtype=np.int32)
    goff[1:] = np.cumsum([a[0].size for a in arrays])
    codes = np.concatenate([a[0] for a in arrays]) if nc else np.zeros(0, np.int32)
    qubits = np.concatenate([a[1] for a in arrays]) if nc else np.zeros((0, 2), np.int32)
    params = np.concatenate([a[2] for a in arrays]) if nc else np.zeros((0, 3), np.float64)
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    toff = np.zeros(nc + 1, dtype=np.int32)
    toff[1:] = np.cumsum([len(z) for z in z_masks])
    zm = np.ascontiguousarray(np.array([int(m) for z in z_masks for m in z], dtype=np.uint64))
    if zm.size == 0:
        zm = np.zeros(1, dtype=np.uint64)
    nq = np.ascontiguousarray(n_qubits, dtype=np.int32)
    b = _vp()
    _check(_L.sv_batch_create(_vp(h), nc, nq.ctypes.data_as(_pi32), goff.ctypes.data_as(_pi32),
                              codes.ctypes.data_as(_pi32), qubits.ctypes.data_as(_pi32), _dptr(params),
                              toff.ctypes.data_as(_pi32), zm.ctypes.data_as(_pu64), max_fused_qubits,
                              ctypes.byref(b)))
    return b.value


def sv_batch_state_layout(b: int, n_circuits: int):
    total = ctypes.c_uint64()
    offs = np.zeros(max(1, n_circuits), dtype=np.uint64)
    _check(_L.sv_batch_state_layout(_vp(b), ctypes.byref(total), offs.ctypes.data_as(_pu64)))
    return total.value, offs[:n_circuits]


def sv_batch_info(b: int, n_qubits: int, n_circuits: int):
    k = _i32()
    blocks = np.zeros(max(1, n_circuits), dtype=np.int32)
    _check(_L.sv_batch_info(_vp(b), n_qubits, ctypes.byref(k), blocks.ctypes.data_as(_pi32)))
    return k.value, blocks[:n_circuits]


def sv_batch_plan(b: int, n_qubits: int) -> dict:
    p = sv_batch_size_plan_t()
    _check(_L.sv_batch_plan(_vp(b), n_qubits, ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in sv_batch_size_plan_t._fields_}


def sv_batch_host_times(b: int):
    """(seconds in the autotuner, seconds fusing, packing and uploading)"""
    t, u = ctypes.c_double(), ctypes.c_double()
    _check(_L.sv_batch_host_times(_vp(b), ctypes.byref(t), ctypes.byref(u)))
    return t.value, u.value


def sv_batch_run(b: int, states_ptr: int, n_terms_total: int, n_circuits: int):
    exp = np.zeros(max(1, n_terms_total), dtype=np.float64)
    lat = np.zeros(max(1, n_circuits), dtype=np.float64)
    ks = ctypes.c_double()
    _check(_L.sv_batch_run(_vp(b), _vp(states_ptr), _dptr(exp), _dptr(lat), ctypes.byref(ks)))
    return exp[:n_terms_total], lat[:n_circuits], ks.value


def sv_batch_destroy(b: int) -> None:
    _check(_L.sv_batch_destroy(_vp(b)))


class Batch:
    """A batch of complex64 circuits run by one persistent launch; the states
    live in one torch buffer that libsv borrows."""

    def __init__(self, handle: Handle, n_qubits, circuits, z_masks, max_fused_qubits: int = 0):
        import torch
        self.handle = handle
        self.n_qubits = [int(v) for v in n_qubits]
        self.z_masks = [list(z) for z in z_masks]
        self.n_terms = sum(len(z) for z in self.z_masks)
        self.b = sv_batch_create(handle.h, self.n_qubits, circuits, self.z_masks, max_fused_qubits)
        total, self.offsets = sv_batch_state_layout(self.b, len(self.n_qubits))
        with torch.cuda.stream(handle.stream):
            self.buffer = torch.empty(int(total) // 8 + 32, dtype=torch.complex64, device="cuda")
        self.base = self.buffer.data_ptr()
        pad = (-self.base) % 256
        self.base += pad

    def run(self):
        """(expectations split per circuit, latencies in s, kernel time in s)"""
        exp, lat, ks = sv_batch_run(self.b, self.base, self.n_terms, len(self.n_qubits))
        out, at = [], 0
        for z in self.z_masks:
            out.append(exp[at: at + len(z)])
            at += len(z)
        return out, lat, ks

    def fusion_width(self, n: int) -> int:
        return sv_batch_info(self.b, n, len(self.n_qubits))[0]

    def blocks(self):
        return sv_batch_info(self.b, 0, len(self.n_qubits))[1]

    def plan(self, n: int) -> dict:
        return sv_batch_plan(self.b, n)

    def host_times(self):
        return sv_batch_host_times(self.b)

    def state(self, i: int) -> np.ndarray:
        import torch
        n = self.n_qubits[i]
        off = int(self.offsets[i]) // 8 + (self.base - self.buffer.data_ptr()) // 8
        torch.cuda.synchronize()
        return self.buffer[off: off + (1 << n)].cpu().numpy()

    def close(self):
        if self.b:
            sv_batch_destroy(self.b)
            self.b = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
