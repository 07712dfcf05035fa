"""Seeded synthetic inputs for state-vector circuit simulation.

This module only draws random numbers and lays out gate lists; it holds none
of the simulation arithmetic (no gate matrices of named gates, no state
updates, no reductions).  Both the CPU oracle and the GPU library consume the
same gate lists, and each side turns a named gate into its matrix with its own
gate table.

A gate is ``Gate(name, qubits, params)``:

* ``name`` is one of ``"u3" "h" "x" "y" "z" "cz" "cx" "cp" "swap" "mat"``,
  optionally with the suffix ``"_dg"`` that asks for the adjoint.
* ``qubits`` lists the qubits the gate touches.  For ``cx`` and ``cp`` the
  first qubit is the control and the second the target (``cz`` and ``cp`` are
  symmetric anyway).  For ``mat`` every listed qubit is a target and
  ``qubits[0]`` is the least-significant bit of the matrix row/column index.
* ``params`` is a tuple of angles for ``u3`` (theta, phi, lambda) and ``cp``
  (phi), empty for the fixed gates, and the 2^k x 2^k complex128 row-major
  matrix (a numpy array) for ``mat``.

Qubit j is bit j of the amplitude index (qubit 0 is the least-significant
bit), the convention of the paper's index-bit description (Sec. II-C).
"""
from __future__ import annotations

import math
from collections import namedtuple

import numpy as np

Gate = namedtuple("Gate", "name qubits params")

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# circuits of the benchmark configurations
# --------------------------------------------------------------------------

def brickwork(n: int, depth: int, seed: int) -> list:
    """Brickwork random circuit: ``depth`` layers, each a U3 on every qubit
    followed by CZ on neighbouring pairs (i, i+1), with the brick offset
    alternating between even (layer 0) and odd layers.

    Angles are drawn all at once as ``rng.uniform(0, 2*pi, size=(depth, n, 3))``
    in (layer, qubit, (theta, phi, lambda)) order.
    """
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, TWO_PI, size=(depth, n, 3))
    gates = []
    for layer in range(depth):
        for q in range(n):
            gates.append(Gate("u3", (q,), tuple(float(a) for a in ang[layer, q])))
        for i in range(layer % 2, n - 1, 2):
            gates.append(Gate("cz", (i, i + 1), ()))
    return gates


def _random_far_pairs(n: int, rng) -> list:
    """A random matching of the qubits into floor(n/2) disjoint pairs whose
    members are at least two apart; redrawn until that holds.  For odd n the
    idle qubit is never one of the two top qubits, so the top index bits are
    always inside a pair."""
    while True:
        perm = [int(v) for v in rng.permutation(n)]
        pairs = [(perm[2 * j], perm[2 * j + 1]) for j in range(n // 2)]
        if any(abs(a - b) < 2 for a, b in pairs):
            continue
        if n % 2 == 1 and perm[-1] >= n - 2:
            continue
        return pairs


def random_cx_cp(n: int, depth: int, seed: int) -> list:
    """Random circuit of CNOT and controlled-phase gates on random
    non-adjacent pairs: each layer is a U3 on every qubit, then a random
    far-pair matching; each pair gets CNOT (first member controls) or
    CP(phi ~ U[0, 2pi)) by a fair coin."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(depth):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 3))
        for q in range(n):
            gates.append(Gate("u3", (q,), tuple(float(a) for a in ang[q])))
        for a, b in _random_far_pairs(n, rng):
            if rng.random() < 0.5:
                gates.append(Gate("cx", (a, b), ()))
            else:
                gates.append(Gate("cp", (a, b), (float(rng.uniform(0.0, TWO_PI)),)))
    return gates


def qft(n: int) -> list:
    """Textbook QFT gate list: for j = n-1 down to 0, H(j) then CP(pi/2^(j-m))
    on (m, j) for m = j-1 down to 0; then SWAP(j, n-1-j) for j < n//2.
    Gate count n + n(n-1)/2 + n//2 (577 at n = 33)."""
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("h", (j,), ()))
        for m in range(j - 1, -1, -1):
            gates.append(Gate("cp", (m, j), (math.pi / float(2 ** (j - m)),)))
    for j in range(n // 2):
        gates.append(Gate("swap", (j, n - 1 - j), ()))
    return gates


def ghz(n: int, order=None) -> list:
    """H on the first qubit of ``order`` then a CNOT chain along ``order``
    (default 0, 1, ..., n-1)."""
    order = list(range(n)) if order is None else list(order)
    gates = [Gate("h", (order[0],), ())]
    for a, b in zip(order[:-1], order[1:]):
        gates.append(Gate("cx", (a, b), ()))
    return gates


def cluster_1d(n: int) -> list:
    """H on every qubit, then CZ on every neighbouring pair."""
    gates = [Gate("h", (q,), ()) for q in range(n)]
    gates += [Gate("cz", (i, i + 1), ()) for i in range(n - 1)]
    return gates


def inverse(gates: list) -> list:
    """The mirror of a gate list: reversed order, each gate marked as its
    adjoint by toggling the ``_dg`` suffix of its name.  Each consumer turns
    ``<name>_dg`` into the conjugate transpose of its own ``<name>`` matrix."""
    out = []
    for g in reversed(gates):
        name = g.name[:-3] if g.name.endswith("_dg") else g.name + "_dg"
        out.append(Gate(name, g.qubits, g.params))
    return out


# --------------------------------------------------------------------------
# random inputs
# --------------------------------------------------------------------------

def haar_unitary(k: int, rng) -> np.ndarray:
    """A 2^k x 2^k Haar-random unitary (QR of a complex Gaussian with the
    phases of R's diagonal folded back), complex128 row-major."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return np.ascontiguousarray(q * ph[None, :])


def random_targets(n: int, k: int, rng) -> tuple:
    """k distinct qubits in [0, n), in random order."""
    return tuple(int(v) for v in rng.choice(n, size=k, replace=False))


def random_dense_circuit(n: int, n_gates: int, kmax: int, seed: int, with_controls=True) -> list:
    """Random ``mat`` gates on random targets (k in 1..kmax), some with random
    controls encoded as ``Gate("mat", targets, M)`` plus a controls list; used
    for gate-level parity.  Returns a list of (targets, controls, cvals, M)."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(n_gates):
        k = int(rng.integers(1, min(kmax, n) + 1))
        qs = [int(v) for v in rng.choice(n, size=min(n, k + 2), replace=False)]
        t = tuple(qs[:k])
        c, cv = (), ()
        if with_controls and len(qs) > k and rng.random() < 0.5:
            nc = int(rng.integers(1, len(qs) - k + 1))
            c = tuple(qs[k:k + nc])
            cv = tuple(int(v) for v in rng.integers(0, 2, size=nc))
        ops.append((t, c, cv, haar_unitary(k, rng)))
    return ops


def diagonal_heavy(n: int, count: int, seed: int) -> list:
    """`count` random gates, two thirds of them diagonal: U3, CZ, CP, Z, CX
    and random diagonal unitaries on 1-3 qubits (as "mat" gates), each kind
    equally likely, on random qubits."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(count):
        kind = rng.integers(0, 6)
        qs = [int(q) for q in rng.permutation(n)]
        if kind == 0:
            gates.append(Gate("u3", (qs[0],), tuple(float(a) for a in rng.uniform(0, 2 * np.pi, 3))))
        elif kind == 1:
            gates.append(Gate("cz", (qs[0], qs[1]), ()))
        elif kind == 2:
            gates.append(Gate("cp", (qs[0], qs[1]), (float(rng.uniform(0, 2 * np.pi)),)))
        elif kind == 3:
            gates.append(Gate("z", (qs[0],), ()))
        elif kind == 4:
            gates.append(Gate("cx", (qs[0], qs[1]), ()))
        else:
            k = int(rng.integers(1, 4))
            gates.append(Gate("mat", tuple(qs[:k]), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k)))))
    return gates


def random_basis_state(n: int, seed: int) -> int:
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 1 << n, dtype=np.uint64)) if n < 64 else 0


def uniforms(count: int, seed: int) -> np.ndarray:
    """``count`` uniforms in [0, 1) (float64)."""
    return np.random.default_rng(seed).random(count)


def random_pauli_terms(n: int, count: int, rng) -> list:
    """``count`` Pauli strings, each qubit i.i.d. uniform over {I, X, Y, Z},
    redrawn when all identity.  A term is a list of (qubit, 'X'|'Y'|'Z')."""
    terms = []
    while len(terms) < count:
        ops = rng.integers(0, 4, size=n)
        if not ops.any():
            continue
        terms.append([(q, "IXYZ"[int(o)]) for q, o in enumerate(ops) if o != 0])
    return terms


def z_terms(n: int) -> list:
    return [[(q, "Z")] for q in range(n)]


def zz_neighbour_terms(n: int) -> list:
    return [[(q, "Z"), (q + 1, "Z")] for q in range(n - 1)]


# --------------------------------------------------------------------------
# batched and serving workloads
# --------------------------------------------------------------------------

BatchItem = namedtuple("BatchItem", "n depth seed gates")


def batched(count: int = 4096, seed: int = 0, n_lo: int = 8, n_hi: int = 20,
            d_lo: int = 10, d_hi: int = 40) -> list:
    """``count`` independent brickwork circuits with qubit counts uniform in
    [n_lo, n_hi] and depths uniform in [d_lo, d_hi]; circuit i uses seed
    10**6 + i."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    return [BatchItem(int(ns[i]), int(ds[i]), 10 ** 6 + i,
                      brickwork(int(ns[i]), int(ds[i]), 10 ** 6 + i)) for i in range(count)]


Request = namedtuple("Request", "rid arrival n depth gates terms uniforms")


def serving_circuit(n: int, depth: int, rng) -> list:
    """Each layer: U3 on all qubits, then floor(n/2) random disjoint pairs,
    each CZ or CNOT by a fair coin."""
    gates = []
    for _ in range(depth):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 3))
        for q in range(n):
            gates.append(Gate("u3", (q,), tuple(float(a) for a in ang[q])))
        perm = [int(v) for v in rng.permutation(n)]
        for j in range(n // 2):
            a, b = perm[2 * j], perm[2 * j + 1]
            gates.append(Gate("cz" if rng.random() < 0.5 else "cx", (a, b), ()))
    return gates


def serving_requests(count: int, rate_per_s: float, seed: int = 0, n_lo: int = 10,
                     n_hi: int = 28, d_lo: int = 10, d_hi: int = 100,
                     n_terms: int = 16, n_shots: int = 1024) -> list:
    """A Poisson stream: exponential inter-arrival times at ``rate_per_s``;
    qubit count floor(n_lo * ((n_hi+1)/n_lo)^u), u ~ U[0,1) (log-uniform over
    [n_lo, n_hi]); depth uniform in [d_lo, d_hi]; ``n_terms`` random Pauli
    strings and ``n_shots`` uniforms per request.  Request r draws from its
    own generator seeded (seed, r)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    reqs = []
    for r in range(count):
        rr = np.random.default_rng([seed, r])
        n = int(math.floor(n_lo * ((n_hi + 1) / n_lo) ** rr.random()))
        n = min(max(n, n_lo), n_hi)
        depth = int(rr.integers(d_lo, d_hi + 1))
        gates = serving_circuit(n, depth, rr)
        terms = random_pauli_terms(n, n_terms, rr)
        reqs.append(Request(r, float(t[r]), n, depth, gates, terms, rr.random(n_shots)))
    return reqs
