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
             timing: bool = False, mfma: int = 4, stream=None, stage: Optional[int] = None) -> Dict[str, object]:
    """stage: widest staged tile (SV_OPT_STAGE); None = planner.stage_tmax(n,
    dtype), 0 = no staged passes."""
    t0 = time.perf_counter()
    if stage is None:
        stage = planner.stage_tmax(circuit.n, dtype)
    ops = planner.plan(circuit.gates, kmax, fold_diag=fold_diag, staged=stage > 0,
                       nloc=max(circuit.n, stage + 9) if stage else None, sparse_start=stage > 0,
                       tmax=stage or None)
    t_plan = time.perf_counter() - t0
    st = sv.State(circuit.n, 0, dtype, stream)
    try:
        if timing:
            sv.set_option(st.h, sv.SV_OPT_TIMING, 1)
        sv.set_option(st.h, sv.SV_OPT_MFMA, int(mfma))
        sv.set_option(st.h, sv.SV_OPT_STAGE, int(stage))
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


def grid_slice_sets(n: int):
    """Two disjoint 4-qubit slice sets on the near-square grid of n qubits:
    the four corner sites and the 2 x 2 block at the centre."""
    from .workload import grid_shape
    rows, cols = grid_shape(n)
    last_row_len = n - (rows - 1) * cols
    corners = sorted({0, cols - 1, (rows - 1) * cols, (rows - 1) * cols + last_row_len - 1})
    r0, c0 = (rows - 1) // 2, (cols - 1) // 2
    centre = sorted({r0 * cols + c0, r0 * cols + c0 + 1, (r0 + 1) * cols + c0, (r0 + 1) * cols + c0 + 1})
    assert not set(corners) & set(centre) and all(q < n for q in centre)
    return tuple(corners), tuple(centre)


def simulate_sliced(circuit, bits: np.ndarray, set_a, set_b, dtype="c64", kmax: int = 5,
                    tier: bool = False, timing: bool = False, sched=None,
                    pageable: bool = False, tier_dir: Optional[str] = None,
                    checkpoint: bool = False, resume: bool = False,
                    stop_after: Optional[int] = None) -> Dict[str, object]:
    """Sliced evolution (Sec. 4): phases alternate the sliced set; each switch
    is one permute_qubits; the trailing gates on the last sliced set are
    applied by the FP64 cross-slice reduction.

    With the tier in files (tier_dir): checkpoint makes the start of every
    phase a restart point (sv_checkpoint, tagged with the phase index: all
    earlier phases applied, the layout of this phase); resume continues
    from the last checkpoint in tier_dir instead of starting from |0...0>.
    stop_after=i ends the run right after phase i's checkpoint, leaving the
    files and the checkpoint in place (as a run that dies there would);
    the result then holds only "stopped"."""
    t0 = time.perf_counter()
    if sched is None:
        sched = planner.phase_schedule(circuit, set_a, set_b, kmax)
    t_plan = time.perf_counter() - t0
    n = circuit.n
    mask = sum(1 << q for q in sched.phases[0].sliced)
    if resume:
        st = sv.State.open(tier_dir, n, mask, dtype)
        start = int(st.tag)
    else:
        st = sv.State(n, mask, dtype, tier=tier, pageable=pageable, tier_dir=tier_dir)
        start = 0
    if dtype == "c64":   # the phases were planned for this tile limit
        sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(n - len(sched.phases[0].sliced)))
    try:
        if timing:
            sv.set_option(st.h, sv.SV_OPT_TIMING, 1)
        t1 = time.perf_counter()
        for i, ph in enumerate(sched.phases):
            if i < start:
                continue
            sv.permute_qubits(st.h, ph.order)
            if checkpoint:
                sv.checkpoint(st.h, i)
            if stop_after is not None and i >= stop_after:
                sv.set_option(st.h, sv.SV_OPT_KEEP_FILES, 1)
                return {"stopped": i}
            planner.enqueue(st.h, ph.ops, st.dtype)
        amps, stats = sv.reduce_slices(st.h, bits, sched.trailing)
        t_run = time.perf_counter() - t1
        out = {"amps": amps, "norm": stats[0], "xeb_sum": stats[1], "xeb_log_sum": stats[2],
               "t_plan": t_plan, "t_run": t_run, "phases": len(sched.phases), "resumed_at": start,
               "trailing_gates": len(sched.trailing_gate_ids),
               "sweeps": sum(len(p.ops) for p in sched.phases), "counters": sv.counters(st.h)}
        if timing:
            out["sweep_ms"], out["sweeps_timed"] = sv.sweep_time(st.h)
        return out
    finally:
        st.close()


# host threads issuing the per-state reductions after a batch
REDUCE_THREADS = 8


def run_batch(circuits, bits_list, dtype="c64", kmax=5, mfma_min_k=4, graph: bool = True,
              repeats: int = 1, plans=None, staged: bool = False, stage_t=None) -> Dict[str, object]:
    """Many independent circuits as one batched execution (one graph launch
    per run).  kmax / mfma_min_k / stage_t: an int, or a dict n -> value
    (autotuned).  staged (complex64): each state's runs of 4/5-qubit blocks
    go through staged passes (tile limit stage_t, default
    planner.stage_tmax(n)), planned for them.  Each repeat resets every
    state and replays the batch; the returned amplitudes are those of the
    last repeat."""
    kof = (lambda n: kmax[n]) if isinstance(kmax, dict) else (lambda n: kmax)
    mof = (lambda n: mfma_min_k[n]) if isinstance(mfma_min_k, dict) else (lambda n: mfma_min_k)
    staged = staged and dtype == "c64"
    if not staged:
        tmax = lambda n: 0                                            # noqa: E731
    elif isinstance(stage_t, dict):
        tmax = lambda n: stage_t[n]                                   # noqa: E731
    elif stage_t is not None:
        tmax = lambda n: min(int(stage_t), n - 9)                     # noqa: E731
    else:
        tmax = planner.stage_tmax
    t0 = time.perf_counter()
    if plans is None:
        plans = [planner.plan_fast(c.gates, kof(c.n), nloc=c.n, sparse_start=True, tmax=tmax(c.n))
                 if tmax(c.n) > 0
                 else planner.plan(c.gates, kof(c.n), staged=False) for c in circuits]
    t_plan = time.perf_counter() - t0
    states = []
    b = None
    try:
        for c in circuits:
            st = sv.State(c.n, 0, dtype)
            sv.set_option(st.h, sv.SV_OPT_MFMA, int(mof(c.n)))
            sv.set_option(st.h, sv.SV_OPT_STAGE, int(tmax(c.n)))
            states.append(st)
        for st, ops in zip(states, plans):
            planner.enqueue(st.h, ops, st.dtype)
        b = sv.batch_prepare([st.h for st in states], graph=graph)
        times = []
        outs = None
        import torch
        from concurrent.futures import ThreadPoolExecutor
        # the per-state reductions run from a few host threads: each call
        # waits for its own results, and the library takes calls on
        # different states concurrently (their streams are independent)
        with ThreadPoolExecutor(max_workers=REDUCE_THREADS) as pool:
            list(pool.map(lambda _: None, range(REDUCE_THREADS)))      # start the threads
            for rep in range(repeats):
                # from a reset every state starts as |0...0> unwritten: the batch
                # then runs its reset variant (no fill ahead, sparse first passes)
                for st in states:
                    sv.reset(st.h)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sv.batch_launch(b)
                outs = list(pool.map(lambda sb: sv.reduce_slices(sb[0].h, sb[1]), zip(states, bits_list)))
                times.append(time.perf_counter() - t1)
        info = sv.batch_info(b)
        return {"amps": [o[0] for o in outs], "stats": [o[1] for o in outs], "times": times,
                "t_plan": t_plan, "info": info,
                "sweeps": [sum(1 for o in p if o.kind == "dense") for p in plans]}
    finally:
        if b is not None:
            sv.batch_destroy(b)
        for st in states:
            st.close()


def simulate_deferred(circuit, bits: np.ndarray, part1: Sequence[int], ncycles: int, kmax: int = 5,
                      timing: bool = False) -> Dict[str, object]:
    """Contraction deferral (Sec. 2; App. A): the first `ncycles` cycles run
    as two tensors (part1 and the other qubits) with EI / E2Q for every
    bridging gate, each a complex64 state of its part plus the entanglement
    indices; both are permuted so the entanglement indices sit at the top
    in the same order, `sv_contract` forms the joint state, and the rest of
    the circuit runs on it.  Returns amplitudes of `bits` (over the circuit
    qubits), the norm and the cross-entropy sums, and the stage times."""
    import torch
    from . import deferral
    t0 = time.perf_counter()
    sp = deferral.split(circuit, part1, ncycles)
    nt1, nt2 = sp.n1 + sp.e, sp.n2 + sp.e
    plans = []
    for ops, nq in ((sp.ops1, nt1), (sp.ops2, nt2)):
        p = planner.plan(ops, kmax, nloc=nq, sparse_start=True) if ops else []
        for o in p:
            o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
        plans.append(p)
    rest = planner.plan(sp.rest, kmax, nloc=circuit.n) if sp.rest else []
    for o in rest:
        o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    jbits = sp.joint_bits(bits)
    t_plan = time.perf_counter() - t0
    # a stream of its own: the contraction and the joint state's work are
    # ordered on it (a NULL stream would give the joint state a stream of
    # the library's own, unordered with the contraction)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        out = torch.empty(1 << circuit.n, dtype=torch.complex64, device="cuda")
    s1 = sv.State(nt1, 0, "c64")
    s2 = sv.State(nt2, 0, "c64")
    h3 = None
    try:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for st, p, nq, order in ((s1, plans[0], nt1, sp.order1), (s2, plans[1], nt2, sp.order2)):
            sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(nq))
            planner.enqueue(st.h, p, st.dtype)
            sv.permute_qubits(st.h, order)
        p1, _ = sv.device_buffer(s1.h)
        p2, _ = sv.device_buffer(s2.h)
        sv.sync_state(s1.h)
        sv.sync_state(s2.h)
        t2 = time.perf_counter()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        sv.contract(p1, p2, out.data_ptr(), sp.n1, sp.n2, sp.e, "c64", stream.cuda_stream)
        ev[1].record(stream)
        h3 = sv.create_state_ext(circuit.n, 0, "c64", stream.cuda_stream, out.data_ptr(),
                                 out.numel() * 8, keep=True)
        if timing:
            sv.set_option(h3, sv.SV_OPT_TIMING, 1)
        sv.set_option(h3, sv.SV_OPT_STAGE, planner.stage_tmax(circuit.n))
        planner.enqueue(h3, rest, sv.SV_C64)
        amps, stats = sv.reduce_slices(h3, jbits)
        stream.synchronize()
        t3 = time.perf_counter()
        return {"amps": amps, "norm": stats[0], "xeb_sum": stats[1], "xeb_log_sum": stats[2],
                "split": sp, "t_plan": t_plan, "t_tensors": t2 - t1,
                "contract_ms": ev[0].elapsed_time(ev[1]), "t_run": t3 - t1,
                "plans": [planner.stats(p) for p in plans] + [planner.stats(rest)]}
    finally:
        if h3 is not None:
            sv.destroy_state(h3)
        s1.close()
        s2.close()
        del out
