#!/usr/bin/env python3
"""Write the stored expected values of the full-size parity tests.

Everything here comes from the CPU oracle (`oracle/`, complex128, one gate at
a time, no fusion, no slicing) and the seeded input generator
(`paper_1910_09534_amd.workload`, which holds no simulation arithmetic).
Nothing is read from the GPU path.

    python tests/golden/make_golden.py headline   # 30 qubits: 16 GiB of RAM, ~30 min on 8 cores
    python tests/golden/make_golden.py batch      # one batch circuit per qubit count 20..28

headline -> tests/golden/headline_30q_d14.npz
    the 30-qubit 5x6-grid ABCDCDAB circuit of depth 14 (circuit seed 1002):
    amplitudes of its 2^16 seeded bitstrings (seed 2002), the norm, and the
    cross-entropy sums over those bitstrings.
batch    -> tests/golden/batch_samples.npz
    for each qubit count 20..28, the first circuit of the 256-circuit batch
    specification with that count: its index j, n, depth, and the amplitudes
    of its 1024 seeded bitstrings (seed 20000 + j).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc                    # noqa: E402
from paper_1910_09534_amd import workload as W     # noqa: E402

HEADLINE = os.path.join(HERE, "headline_30q_d14.npz")
BATCH = os.path.join(HERE, "batch_samples.npz")


def run_circuit(circ, label: str, chunk: int = 40) -> np.ndarray:
    """psi = U_L ... U_1 |0...0>, applied in chunks of gates for progress lines."""
    psi = orc.zero_state(circ.n)
    t0 = time.time()
    for g0 in range(0, len(circ.gates), chunk):
        orc.apply_gates(psi, circ.gates[g0:g0 + chunk])
        print(f"{label}: {min(g0 + chunk, len(circ.gates))}/{len(circ.gates)} gates, "
              f"{time.time() - t0:.0f} s", flush=True)
    return psi


def headline() -> None:
    circ = W.config_circuit(2)
    bits = W.config_bitstrings(2)
    psi = run_circuit(circ, "headline 30q d14")
    amps = orc.gather(psi, bits)
    nrm = orc.norm(psi)
    s1, s2 = orc.xeb_sums(circ.n, amps)
    del psi
    np.savez(HEADLINE, amps=amps, bitstrings=bits, norm=np.float64(nrm), xeb=np.array([s1, s2]),
             n=np.int64(circ.n), depth=np.int64(circ.depth), seed=np.int64(circ.seed))
    print(f"wrote {HEADLINE}: norm={nrm:.15f} sum Np={s1:.6f} sum ln Np={s2:.6f}", flush=True)


def batch() -> None:
    specs = W.batch_specs()
    pick = {}
    for s in specs:
        pick.setdefault(s["n"], s)
    js, ns, ds, amps = [], [], [], []
    for n in sorted(pick):
        s = pick[n]
        circ = W.sycamore_circuit(s["n"], s["depth"], seed=s["seed"])
        bits = W.bitstrings(s["n"], 1024, seed=s["bit_seed"])
        psi = run_circuit(circ, f"batch circuit {s['j']} ({n}q d{s['depth']})", chunk=200)
        amps.append(orc.gather(psi, bits))
        del psi
        js.append(s["j"]); ns.append(n); ds.append(s["depth"])
    np.savez(BATCH, j=np.array(js), n=np.array(ns), depth=np.array(ds), amps=np.stack(amps))
    print(f"wrote {BATCH}: circuits {js}", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["batch", "headline"]
    for w in which:
        {"headline": headline, "batch": batch}[w]()
