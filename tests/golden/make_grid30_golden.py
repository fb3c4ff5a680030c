"""Writes tests/golden/grid30_d20_s2.npz: reference values of the 30-qubit,
depth-20 supremacy-style grid circuit (5 x 6 grid, seed 2), computed by the
CPU oracle alone.

The circuit's output is the ordered product of its gate matrices applied to
|0...0> (paper, Sec. I.A; Sec. II: the simulator is a chain of matrix-vector
products).  The oracle evaluates that chain in complex128, gate by gate, with
no fusion and no reordering; its threaded build gives the same bits as the
single-thread one.  The full 16 GiB state cannot be stored, so the file keeps
statistics that a state compared element by element would also pass:

  amps      amplitudes at 65 536 seeded indices (workloads.sample_indices,
            seed 7; the indices are re-drawn by the reader)
  lo_block  psi[0 : 4096]                (every value of qubits 0..11)
  hi_block  psi[j << 18], j < 4096        (every value of qubits 18..29)
  marg_lo   P(qubits 0..9 = v), v < 1024  (sums over all 2^30 amplitudes)
  marg_hi   P(qubits 20..29 = v), v < 1024
  energy    <psi| sum_i Z_i Z_{i+1} + 0.5 sum_i X_i |psi>, open chain
  norm2     <psi|psi>
  digest    SHA-256 of the generated op list (the reader checks it)

Run from the repository root: python tests/golden/make_grid30_golden.py
It needs about 17 GiB of host memory; on 8 threads it takes about 40 minutes.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid30_d20_s2.npz")
N_QUBITS, SAMPLE_COUNT, SAMPLE_SEED = 30, 1 << 16, 7


def marginals(psi: np.ndarray, lo_bits: int, hi_bits: int, n: int):
    """Probabilities of the low `lo_bits` qubits and of the high `hi_bits`
    qubits, accumulated in double over chunks of the state."""
    marg_lo = np.zeros(1 << lo_bits)
    marg_hi = np.zeros(1 << hi_bits)
    chunk = max(1 << 24, 1 << (n - hi_bits))
    for start in range(0, 1 << n, chunk):
        p = np.abs(psi[start:start + chunk]) ** 2
        marg_lo += p.reshape(-1, 1 << lo_bits).sum(axis=0)
        hi_first, hi_count = start >> (n - hi_bits), p.size >> (n - hi_bits)
        marg_hi[hi_first:hi_first + hi_count] += p.reshape(hi_count, -1).sum(axis=1)
    return marg_lo, marg_hi


def main() -> None:
    circ = W.random_grid_circuit(5, 6, depth=20, seed=2)
    assert circ.n == N_QUBITS
    oracle.build(force=False)
    t0 = time.time()
    psi = oracle.apply_circuit(circ, threaded=True)
    t_apply = time.time() - t0
    print(f"circuit applied in {t_apply:.0f} s", flush=True)
    idx = W.sample_indices(N_QUBITS, SAMPLE_COUNT, SAMPLE_SEED)
    amps = psi[idx.astype(np.int64)]
    lo_block = psi[:4096].copy()
    hi_block = psi[np.arange(4096, dtype=np.int64) << 18].copy()
    marg_lo, marg_hi = marginals(psi, 10, 10, N_QUBITS)
    norm2 = float(np.vdot(psi, psi).real)
    print("statistics done", flush=True)
    t0 = time.time()
    energy = oracle.expectation(psi, W.chain_observable(N_QUBITS))
    print(f"energy {energy!r} in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(
        OUT, amps=amps, lo_block=lo_block, hi_block=hi_block, marg_lo=marg_lo,
        marg_hi=marg_hi, energy=np.float64(energy), norm2=np.float64(norm2),
        sample_seed=np.int64(SAMPLE_SEED), sample_count=np.int64(SAMPLE_COUNT),
        digest=np.array(W.circuit_digest(circ)), gates=np.int64(len(circ.ops)))
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
