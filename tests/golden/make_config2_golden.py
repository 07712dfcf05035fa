"""Writes ``config2_30q_d20_seed0.npz``: values of the 30-qubit, depth-20
brickwork circuit (seed 0, start |0..0>) computed by the CPU oracle alone.

The oracle applies the 890 unfused gates in circuit order to a complex128
state (16 GiB) and then evaluates, on that state:
  - ``idx``/``amp``: 65536 amplitudes at seeded random indices plus the
    indices 0, 1, 2^29 and 2^30 - 1;
  - ``cdf``: the cumulative probability C_i = sum_{j <= i} |psi_j|^2 at the
    same indices, and ``norm`` = C_{2^30 - 1};
  - ``z`` (<Z_i>, i = 0..29), ``zz`` (<Z_i Z_i+1>, i = 0..28) and
    ``pauli`` (eight random X/Y/Z strings, ``pauli_ops``[t, q] in 0..3 for
    I, X, Y, Z on qubit q), each normalised by the norm;
  - ``shots``: the outcomes for 32768 uniforms (``shot_seed``), with the
    cumulative probabilities just below (``shot_c_lo`` = C_{o-1}, 0 for
    o = 0) and at (``shot_c_hi`` = C_o) each outcome o.
Nothing here reads the GPU library.  Run from the repository root:
    python tests/golden/make_config2_golden.py   (about an hour on 8 cores,
    32 GiB of host memory)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N = 30
DEPTH = 20
SEED = 0
IDX_SEED = 20260
N_IDX = 65536
PAULI_SEED = 20261
N_PAULI = 8
SHOT_SEED = 20262
N_SHOTS = 32768
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_30q_d20_seed0.npz")


def main():
    t0 = time.time()
    gates = W.brickwork(N, DEPTH, SEED)
    psi = oracle.basis_state(N, 0)
    for g, gate in enumerate(gates):
        oracle.apply_gate(psi, gate)
        if g % 50 == 0:
            print(f"gate {g}/{len(gates)} {time.time() - t0:.0f}s", flush=True)
    idx = np.random.default_rng(IDX_SEED).integers(0, 1 << N, size=N_IDX, dtype=np.uint64)
    idx = np.concatenate([idx, np.array([0, 1, 1 << (N - 1), (1 << N) - 1], dtype=np.uint64)])
    amp = psi[idx.astype(np.int64)].copy()
    norm = oracle.norm(psi)
    print(f"norm {norm!r} {time.time() - t0:.0f}s", flush=True)
    z = np.array([oracle.expect_pauli(psi, t) for t in W.z_terms(N)])
    print(f"z done {time.time() - t0:.0f}s", flush=True)
    zz = np.array([oracle.expect_pauli(psi, t) for t in W.zz_neighbour_terms(N)])
    print(f"zz done {time.time() - t0:.0f}s", flush=True)
    terms = W.random_pauli_terms(N, N_PAULI, np.random.default_rng(PAULI_SEED))
    ops = np.zeros((N_PAULI, N), dtype=np.int8)
    for t, term in enumerate(terms):
        for q, o in term:
            ops[t, q] = "IXYZ".index(o)
    pauli = np.array([oracle.expect_pauli(psi, t) for t in terms])
    print(f"pauli done {time.time() - t0:.0f}s", flush=True)
    u = W.uniforms(N_SHOTS, SHOT_SEED)
    shots, cdf_all = oracle.sample(psi, u, return_cdf=True)
    cdf = cdf_all[idx.astype(np.int64)].copy()
    o = shots.astype(np.int64)
    c_hi = cdf_all[o].copy()
    c_lo = np.where(o > 0, cdf_all[np.maximum(o - 1, 0)], 0.0)
    del cdf_all, psi
    np.savez(OUT, n=N, depth=DEPTH, seed=SEED, idx_seed=IDX_SEED, idx=idx, amp=amp, cdf=cdf, norm=norm,
             z=z, zz=zz, pauli_seed=PAULI_SEED, pauli_ops=ops, pauli=pauli, shot_seed=SHOT_SEED,
             shots=shots, shot_c_lo=c_lo, shot_c_hi=c_hi, oracle_threads=oracle.threads())
    print(f"wrote {OUT} {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
