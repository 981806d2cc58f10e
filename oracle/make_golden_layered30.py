"""Write the 30-qubit layered-circuit golden file from the CPU oracle.

    python oracle/make_golden_layered30.py            # about 15-30 min on 8 cores, 16 GiB

Test infrastructure: calls only the oracle (and the seeded input generators).
The workload is the layered ansatz of the paper's evaluation (Section 9.1)
at 30 qubits and 20 layers, seed 0: per layer RY then RZ on every qubit, then
the CNOT ladder.  The oracle applies the 1780 gates one by one in FP64 from
|0...0>, then writes to tests/golden/layered30_seed0.npz:

  idx      65536-odd sorted basis indices drawn from numpy's default_rng(2030)
           plus 0 and 2^30 - 1
  amp      the oracle's complex128 amplitudes at idx
  zexp     <Z_q> for q = 0..29 (the Pauli reduction of Section 4.4)
  norm     <psi|psi> summed by the oracle's Pauli pass with the identity term
  samples  1000 terminal samples of all 30 qubits with seed 0 under the
           sampling specification (bit q of a sample = qubit q)
  meta     n, layers, seed, oracle threads, seconds

Nothing here reads the GPU library.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2608_09733_amd import inputs as I  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "layered30_seed0.npz")
N_QUBITS, LAYERS, SEED = 30, 20, 0
IDX_SEED, N_IDX, SHOT_SEED, SHOTS = 2030, 1 << 16, 0, 1000


def golden_indices() -> np.ndarray:
    rng = np.random.default_rng(IDX_SEED)
    idx = rng.integers(0, 1 << N_QUBITS, size=N_IDX, dtype=np.int64)
    idx = np.unique(np.concatenate([idx, [0, (1 << N_QUBITS) - 1]]))
    return idx


def main() -> None:
    if not os.path.exists(O.LIB_PATH):
        from oracle import build
        build.build()
    circ = I.layered(N_QUBITS, LAYERS, seed=SEED)
    t0 = time.time()
    psi = O.run_circuit(circ)
    t_run = time.time() - t0
    print(f"oracle run: {t_run:.1f} s on {O.threads()} threads", flush=True)
    idx = golden_indices()
    amp = psi[idx].copy()
    zham = I.hamiltonian(N_QUBITS, [("Z", [q], 1.0) for q in range(N_QUBITS)] + [("I", [0], 1.0)])
    vals, _, _ = O.expect(N_QUBITS, psi, zham)
    smp = O.sample(N_QUBITS, psi, SHOT_SEED, SHOTS, list(range(N_QUBITS)))
    meta = np.array([N_QUBITS, LAYERS, SEED, O.threads(), int(round(t_run))], dtype=np.int64)
    np.savez(OUT, idx=idx, amp=amp, zexp=vals[:N_QUBITS], norm=np.array([vals[N_QUBITS]]),
             samples=smp, meta=meta)
    print(f"wrote {OUT}: {len(idx)} amplitudes, norm-1 = {vals[N_QUBITS] - 1:.3e}, "
          f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
