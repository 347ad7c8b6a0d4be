"""Product-level entry points: plan a circuit on the host, run it through the
C-ABI, and return amplitudes plus FP64 statistics.

`simulate` is the unsliced path (one resident state).  `simulate_sliced`
is the sliced path of Sec. 4: phases alternate between slice sets, each
phase switch is a `permute_qubits` (the all-to-all reorganisation), slices
live in HBM or in the pinned host tier, and the last gates on sliced qubits
are applied by the cross-slice reduction.
"""
from __future__ import annotations

import time
from typing import Dict, Optional, Sequence

import numpy as np

from . import planner, sv


def simulate(circuit, bits: np.ndarray, dtype="c64", kmax: int = 5, fold_diag: bool = False,
             timing: bool = False, mfma: int = 4, stream=None) -> Dict[str, object]:
    t0 = time.perf_counter()
    ops = planner.plan(circuit.gates, kmax, fold_diag=fold_diag)
    t_plan = time.perf_counter() - t0
    st = sv.State(circuit.n, 0, dtype, stream)
    try:
        if timing:
            sv.set_option(st.h, sv.SV_OPT_TIMING, 1)
        sv.set_option(st.h, sv.SV_OPT_MFMA, int(mfma))
        t1 = time.perf_counter()
        planner.enqueue(st.h, ops, st.dtype)
        amps, stats = st.reduce(bits)
        t_run = time.perf_counter() - t1
        out = {"amps": amps, "norm": stats[0], "xeb_sum": stats[1], "xeb_log_sum": stats[2],
               "t_plan": t_plan, "t_run": t_run, "plan": planner.stats(ops),
               "counters": sv.counters(st.h)}
        if timing:
            out["sweep_ms"], out["sweeps_timed"] = sv.sweep_time(st.h)
        return out
    finally:
        st.close()
