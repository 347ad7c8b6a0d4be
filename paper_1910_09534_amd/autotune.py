"""Autotuner for the fusion width, the staged tile limit and the kernel
form (host driver; every timing runs on the GPU through the C-ABI).

tune_staged (the batch's staged path): for every qubit count n, a
representative ABCDCDAB circuit is planned for each fusion width kmax in
{3..6} and staged tile limit in {12, 13, 14}, run from a reset, and the
fastest (kmax, tile limit) is kept.

tune (single sweeps, no staging): one dense sweep of a random k-qubit block
(k = 1..6) is timed with the VALU kernel and, for k >= 4, with the
matrix-core kernel, then:
  * mfma_min_k[n] = the smallest k from which the matrix-core form wins;
  * kmax[n] = the fusion width whose plan of a representative ABCDCDAB
    circuit on n qubits has the lowest modelled time (sum over the planned
    blocks of the measured time of a block of that width).
Results can be written to / read from a JSON file.
"""
from __future__ import annotations

import json
import os
import time
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


def time_staged_plan(n: int, ops, stage_t: int, reps: int = 3) -> float:
    """Device milliseconds per run of a planned op list on an n-qubit
    complex64 state from a reset (sparse start, staged passes on tiles of at
    most stage_t positions): the sum of the run's launch times, HIP events
    on the state's stream (SV_OPT_TIMING); the best of `reps` runs."""
    st = sv.State(n, 0, "c64")
    try:
        sv.set_option(st.h, sv.SV_OPT_STAGE, stage_t)
        packed = planner.pack(ops, st.dtype)
        best = float("inf")
        for r in range(reps + 1):
            sv.reset(st.h)
            sv.sweep_profile(st.h)
            sv.set_option(st.h, sv.SV_OPT_TIMING, 1 if r else 0)
            planner.enqueue(st.h, packed, st.dtype)
            st.sync()
            p = sv.sweep_profile(st.h)
            if r:
                best = min(best, p["sweep"]["ms"] + p["staged"]["ms"])
        return best
    finally:
        st.close()


def tune_staged(ns: Iterable[int] = range(20, 29), kmaxes=(3, 4, 5, 6), tiles=(12, 13, 14),
                depth: int = 15, reps: int = 3) -> Dict[str, Dict]:
    """Fusion width and staged tile limit per qubit count for the batch's
    staged path (Sec. 5: the width of the aggregated gates is the tuned
    parameter): for every n, a representative ABCDCDAB circuit is planned
    with plan_fast for each (kmax, tile limit) and run on the GPU from a
    reset; the fastest pair is kept.  kmax 3 blocks are widened to 4 qubits
    and staged like the rest; kmax 6 adds 6-qubit blocks, which run as
    single matrix-core sweeps between staged passes."""
    kmax: Dict[int, int] = {}
    tile: Dict[int, int] = {}
    table: Dict[int, Dict[str, float]] = {}
    for n in ns:
        circ = W.sycamore_circuit(n, depth, seed=777)
        t = {}
        # tile limits above n - 9 leave fewer than 512 tiles per pass: the
        # candidates are capped there
        cand = sorted({min(tl, n - 9) for tl in tiles if min(tl, n - 9) >= 9})
        for kk in kmaxes:
            for tl in cand:
                ops = planner.plan_fast(circ.gates, kk, nloc=n, sparse_start=True, tmax=tl)
                for o in ops:
                    o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
                t[f"{kk}/{tl}"] = time_staged_plan(n, ops, tl, reps)
        best = min(t, key=t.get)
        kmax[n], tile[n] = (int(x) for x in best.split("/"))
        table[n] = {k: round(v, 4) for k, v in t.items()}
    return {"kmax": kmax, "stage_t": tile, "ms": table}


def save(result, path: str) -> None:
    with open(path, "w") as f:
        json.dump({k: {str(n): v for n, v in d.items()} for k, d in result.items()}, f, indent=1)


def load(path: str):
    with open(path) as f:
        d = json.load(f)
    out = {}
    for k, v in d.items():
        out[k] = {int(n): (x if not isinstance(x, dict) else
                           {(int(a) if a.isdigit() else a): b for a, b in x.items()})
                  for n, x in v.items()}
    return out
