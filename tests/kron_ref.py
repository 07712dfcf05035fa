"""Brute-force reference operators for tiny qubit counts (n <= 8).

Builds the full 2^n x 2^n operator of a gate from ``numpy.kron`` and an
explicit index permutation, with no loop over amplitude groups, so that it
shares nothing with the oracle's gate application.  Used only to pin the
oracle.
"""
import numpy as np


def embed(matrix, targets, n, controls=(), cvals=None):
    """Full operator of ``matrix`` acting on ``targets`` (targets[0] = matrix
    LSB), controlled on ``controls`` having values ``cvals`` (default all 1)."""
    k = len(targets)
    rest = [q for q in range(n) if q not in targets]
    big = np.kron(np.asarray(matrix, dtype=np.complex128), np.eye(1 << (n - k)))
    dim = 1 << n
    # position of each standard basis index inside big's ordering:
    # bits of the matrix index (targets) on top, the other qubits below in order
    perm = np.zeros(dim, dtype=np.int64)
    for i in range(dim):
        hi = sum(((i >> t) & 1) << a for a, t in enumerate(targets))
        lo = sum(((i >> q) & 1) << b for b, q in enumerate(rest))
        perm[i] = (hi << (n - k)) | lo
    full = big[np.ix_(perm, perm)]
    if controls:
        cvals = [1] * len(controls) if cvals is None else list(cvals)
        sel = np.array([all(((i >> c) & 1) == v for c, v in zip(controls, cvals)) for i in range(dim)])
        d = np.diag(sel.astype(np.complex128))
        full = d @ full + (np.eye(dim) - d)
    return full


PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def pauli_operator(term, n):
    """Kronecker product of single-qubit Paulis; qubit n-1 is the leftmost factor."""
    ops = ["I"] * n
    for q, o in term:
        ops[q] = o
    full = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        full = np.kron(full, PAULI[ops[q]])
    return full
