"""Write the oracle's results for the 21-qubit benchmark circuit.

Runs only the CPU oracle (``oracle/``) on the seeded workload: 50,000 Pauli
exponentials exp(-i theta P / 2) on 21 qubits (seed 2, 450,728 gates,
Section 3.2 update equations applied gate by gate), and stores what a GPU
result is checked against:

* ``energy`` and ``term``: <H> of the 100-term Pauli sum (seed 3) and each
  term's <P_k> (normalised by <psi|psi>);
* ``z``: <Z_i> for every qubit;
* ``probs_lo`` / ``probs_hi``: marginal probabilities of qubits 0..9 and
  11..20;
* ``sample_idx`` / ``sample_amp``: 4,096 amplitudes at seeded indices;
* ``probe``: overlaps <r_k|psi> with the seeded complex Gaussian vectors of
  ``workloads.probe_vectors`` (E|<r|d>|^2 = 2||d||^2 for a difference d),
  from which a test estimates ||psi_gpu - psi_oracle||^2, an upper bound of
  the infidelity of two unit states, without the 32 MiB oracle state;
* ``gates_sha256``: hash of the gate records, so a changed generator is
  caught.

Usage: python tests/golden/make_cfg2_fixture.py [--n-exp N] [--out PATH]
(about 20 minutes on 8 host cores).
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_QUBITS = 21
N_PROBES = 48


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-exp", type=int, default=50_000)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    out = a.out or os.path.join(HERE, f"cfg2_21q_{a.n_exp // 1000}k_oracle.npz")
    n = N_QUBITS
    g, thetas, _ = W.pauli_exponential_circuit(n, a.n_exp, seed=2)
    H = W.pauli_sum(n, 100, seed=3)
    oracle.set_threads(a.threads)
    t0 = time.time()
    psi, _, _ = oracle.run(n, g)
    t_run = time.time() - t0
    print(f"{len(g)} gates in {t_run:.0f} s", flush=True)
    term = np.array([oracle.expval(n, psi, H[k:k + 1]) for k in range(len(H))])
    z = np.array([oracle.expval(n, psi, W.z_terms(n)[i:i + 1]) for i in range(n)])
    rng = np.random.default_rng(np.random.SeedSequence([2024, n]))
    idx = np.sort(rng.choice(1 << n, size=4096, replace=False)).astype(np.int64)
    probe = np.array([np.vdot(r, psi) for r in W.probe_vectors(n, N_PROBES)])
    np.savez(out,
             n=np.int64(n), n_exp=np.int64(a.n_exp), n_gates=np.int64(len(g)),
             gates_sha256=np.frombuffer(hashlib.sha256(g.tobytes()).digest(), dtype=np.uint8),
             energy=np.float64(oracle.expval(n, psi, H)), term=term, z=z,
             norm=np.float64(oracle.norm(n, psi)),
             probs_lo=oracle.probs(n, psi, list(range(10))),
             probs_hi=oracle.probs(n, psi, list(range(11, 21))),
             sample_idx=idx, sample_amp=psi[idx], probe=probe,
             oracle_seconds=np.float64(t_run))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
