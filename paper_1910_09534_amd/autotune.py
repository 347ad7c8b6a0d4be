"""Autotuner for the fusion width and the kernel form (host driver).

For every qubit count n it times, on the GPU through the C-ABI, one dense
sweep of a random k-qubit block (k = 1..6) with the VALU kernel and, for
k >= 4, with the matrix-core kernel, then:
  * mfma_min_k[n] = the smallest k from which the matrix-core form wins;
  * kmax[n] = the fusion width whose plan of a representative ABCDCDAB
    circuit on n qubits has the lowest modelled time (sum over the planned
    blocks of the measured time of a block of that width).
Results can be written to / read from a JSON file.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable

import numpy as np

from . import planner, sv
from . import workload as W


def time_sweep(n: int, k: int, mfma: int, reps: int = 5) -> float:
    """Milliseconds per sweep of a random k-block on an n-qubit complex64 state
    (targets at positions 6.., HIP events on the state's stream)."""
    st = sv.State(n, 0, "c64")
    try:
        sv.set_option(st.h, sv.SV_OPT_MFMA, mfma)
        qs = list(range(min(6, n - k), min(6, n - k) + k))
        u = W.random_unitary(1 << k, np.random.default_rng(k)).astype(np.complex64)
        st.fused(qs, u)
        st.sync()
        sv.sweep_time(st.h)
        sv.set_option(st.h, sv.SV_OPT_TIMING, 1)
        for _ in range(reps):
            st.fused(qs, u)
        st.sync()
        ms, cnt = sv.sweep_time(st.h)
        return ms / max(cnt, 1)
    finally:
        st.close()


def tune(ns: Iterable[int] = range(20, 29), ks=(3, 4, 5, 6), depth: int = 15) -> Dict[str, Dict]:
    table: Dict[int, Dict[int, float]] = {}
    mfma_min: Dict[int, int] = {}
    kmax: Dict[int, int] = {}
    for n in ns:
        t = {}
        best_from = 0
        for k in range(1, 7):
            valu = time_sweep(n, k, 0)
            t[k] = valu
            if k >= 4 and n >= k + 4:
                mf = time_sweep(n, k, 4)
                if mf < valu:
                    t[k] = mf
                    if not best_from:
                        best_from = k
        table[n] = t
        mfma_min[n] = best_from if best_from else 0
        circ = W.sycamore_circuit(n, depth, seed=777)
        costs = {}
        for kk in ks:
            ops = planner.plan(circ.gates, kk, staged=False)
            costs[kk] = sum(t[len(o.qubits)] for o in ops if o.kind == "dense")
        kmax[n] = min(costs, key=costs.get)
    return {"kmax": kmax, "mfma_min_k": mfma_min, "sweep_ms": table}


def save(result, path: str) -> None:
    with open(path, "w") as f:
        json.dump({k: {str(n): v for n, v in d.items()} for k, d in result.items()}, f, indent=1)


def load(path: str):
    with open(path) as f:
        d = json.load(f)
    out = {}
    for k, v in d.items():
        out[k] = {int(n): (x if not isinstance(x, dict) else {int(a): b for a, b in x.items()})
                  for n, x in v.items()}
    return out
