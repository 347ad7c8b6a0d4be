"""Request server: simulate-and-return-amplitudes requests with continuous
batching on one GPU.

Each request carries a circuit and the bitstrings whose amplitudes it wants.
The admission loop keeps requests in arrival order and admits the head of
the queue as soon as a slot is free and its complex64 state (2^n x 8 bytes)
gets a block of the HBM budget (one device allocation, made up front and
carved by a buddy allocator); admitted requests run concurrently, each
on its own slot stream, so requests that arrive while others are on the GPU
start as soon as memory and a slot free up and their kernels overlap on the
device.  Each request is planned on the host, in a pool of planning
processes from the moment it arrives (or by its slot worker when there is
no pool); the slot worker creates a resident state in its block of the
arena (no device allocation while requests run), queues the whole plan with
one C-ABI call, and reduces the requested amplitudes and the norm in FP64.
Latency = completion - arrival.

PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import dataclasses
import heapq
import threading
import time
from typing import Dict, List, Optional

import numpy as np

from . import planner, sv


@dataclasses.dataclass
class Request:
    rid: int
    t_arrival: float           # seconds from the start of the trace
    circuit: object
    bits: np.ndarray


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    amps: np.ndarray
    norm: float
    t_arrival: float
    t_admit: float
    t_done: float
    sweeps: int
    t_planned: float = 0.0      # plan ready (seconds from the start of the trace)
    t_queued: float = 0.0       # state allocated and the plan queued to the library
    device_ms: float = 0.0      # sum of the request's sweep / staged-pass launch times

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def state_bytes(n: int) -> int:
    return (1 << n) * 8


def plan_request(circuit, kmax: int):
    """Single-heuristic staged plan (fast enough to sit inside the request
    path): blocks ordered and widened for staged passes, ranked for a run
    from |0...0> (the request's state starts there: sparse start)."""
    ops = planner.plan_fast(circuit.gates, kmax, sparse_start=True)
    for o in ops:
        o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    return ops


def planning_pool(workers: int = 8):
    """Processes that plan requests outside this interpreter (planning is
    host Python and would otherwise hold the interpreter lock that the slot
    workers need).  Create it before this process touches the GPU: the
    workers are started here, by spawning fresh interpreters."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn"))
    # return once every worker runs (each has taken a task), so that none is
    # still starting up while the caller goes on
    seen = set()
    for _ in range(20):
        seen |= set(pool.map(_warm, range(4 * workers)))
        if len(seen) >= workers:
            break
    return pool


def _warm(_):
    import os
    import time
    time.sleep(0.02)
    return os.getpid()


class BuddyArena:
    """Device memory for the states of admitted requests: one allocation
    made up front, carved into power-of-two blocks by a buddy allocator on
    the host.  A request's state (2^n x 8 bytes) takes one block; freeing a
    block merges it with its free buddy.  No device allocation or release
    happens while requests run (a release would wait for the whole device,
    and a caching allocator under memory pressure does exactly that)."""

    def __init__(self, torch, budget_bytes: int, max_block: int = 1 << 35, min_block: int = 1 << 19):
        top = 1 << (int(min(budget_bytes, max_block)).bit_length() - 1)
        self.top = top
        self.min_block = min(min_block, top)
        self.count = max(1, int(budget_bytes) // top)
        self.size = self.count * top
        # torch=None: bookkeeping only (no device memory; offsets from 0)
        self.buf = None if torch is None else torch.empty(self.size, dtype=torch.uint8, device="cuda")
        self.base = 0 if self.buf is None else self.buf.data_ptr()
        # free offsets per block size
        self.free: Dict[int, set] = {top: {i * top for i in range(self.count)}}

    def block_size(self, nbytes: int) -> int:
        b = self.min_block
        while b < nbytes:
            b <<= 1
        return b

    def alloc(self, nbytes: int) -> Optional[int]:
        """Offset of a free block of at least nbytes, or None."""
        want = self.block_size(nbytes)
        b = want
        while b <= self.top and not self.free.get(b):
            b <<= 1
        if b > self.top:
            return None
        off = min(self.free[b])                 # lowest address first: deterministic
        self.free[b].discard(off)
        while b > want:                         # split, keeping the low half
            b >>= 1
            self.free.setdefault(b, set()).add(off + b)
        return off

    def release(self, off: int, nbytes: int) -> None:
        b = self.block_size(nbytes)
        while b < self.top:
            buddy = off ^ b
            if buddy in self.free.get(b, ()):
                self.free[b].discard(buddy)
                off = min(off, buddy)
                b <<= 1
            else:
                break
        self.free.setdefault(b, set()).add(off)


def run_one(torch, stream, req: Request, kmax: int, mfma_min_k: int = 4, ops=None, marks=None,
            dev_ptr: Optional[int] = None):
    """Plan (unless `ops` is given) and simulate one request on `stream`;
    returns (amps, norm, sweeps).  dev_ptr: device memory for the state
    (2^n x 8 bytes, e.g. a BuddyArena block); None: a buffer from torch's
    caching allocator.  marks: optional list that receives the
    perf_counter time at which the plan was queued to the library and the
    request's launch time in milliseconds."""
    n = req.circuit.n
    if ops is None:
        ops = plan_request(req.circuit, kmax)
    buf = None
    if dev_ptr is None:
        with torch.cuda.stream(stream):
            buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
        dev_ptr = buf.data_ptr()
    # the buffer's old contents are kept and the reset deferred: the first
    # pass builds |0...0> itself, so no fill kernel writes the whole buffer
    h = sv.create_state_ext(n, 0, "c64", stream.cuda_stream, dev_ptr, (1 << n) * 8, keep=True)
    try:
        sv.reset(h)
        sv.set_option(h, sv.SV_OPT_MFMA, mfma_min_k)
        sv.set_option(h, sv.SV_OPT_STAGE, planner.stage_tmax(n))
        if marks is not None:
            sv.set_option(h, sv.SV_OPT_TIMING, 1)
        planner.enqueue(h, ops, sv.SV_C64)          # one library call for the whole plan
        if marks is not None:
            marks.append(time.perf_counter())
        amps, stats = sv.reduce_slices(h, req.bits)
        if marks is not None:
            p = sv.sweep_profile(h)
            marks.append(p["sweep"]["ms"] + p["staged"]["ms"])
    finally:
        sv.destroy_state(h)
    del buf
    return amps, stats[0], sum(1 for o in ops if o.kind == "dense")


class Server:
    def __init__(self, budget_bytes: float = 250e9, slots: int = 8, kmax: int = 5,
                 mfma_min_k: int = 4, planner_pool=None, arena: Optional[BuddyArena] = None):
        import torch
        self.torch = torch
        # with a planning pool every request is planned from its arrival on,
        # in another process, while earlier requests run
        self.pool = planner_pool
        self.plans: Dict[int, object] = {}
        # states live in one arena of the budget (pass one to reuse it)
        self.arena = arena if arena is not None else BuddyArena(torch, int(budget_bytes))
        self.budget = self.arena.size
        self.kmax = kmax
        self.mfma_min_k = mfma_min_k
        self.streams = [torch.cuda.Stream() for _ in range(slots)]   # default priority
        self.free_slots = list(range(slots))
        self.mem_used = 0
        self.cv = threading.Condition()
        self.results: Dict[int, Result] = {}
        self.errors: List[str] = []
        self.finished: set = set()
        self.max_inflight = 0
        self.inflight = 0

    def _run_worker(self, slot: int, req: Request, off: int, t_admit: float, t0: float):
        """Thread body: the worker; if it fails without recording an outcome,
        the failure is recorded and the slot and memory are released, so the
        admission loop never waits for a request that will not finish."""
        try:
            self._worker(slot, req, off, t_admit, t0)
        except BaseException as e:          # recorded, never swallowed
            with self.cv:
                if req.rid not in self.finished:
                    self._finish(req, None, f"request {req.rid}: {e!r}", slot, off)

    def _finish(self, req: Request, res, err, slot: int, off: int) -> None:
        """Record a request's outcome and release its slot and memory (with
        self.cv held)."""
        self.finished.add(req.rid)
        if res is not None:
            self.results[req.rid] = res
        else:
            self.errors.append(err)
        self.arena.release(off, state_bytes(req.circuit.n))
        self.mem_used -= self.arena.block_size(state_bytes(req.circuit.n))
        self.free_slots.append(slot)
        self.inflight -= 1
        self.cv.notify_all()

    def _worker(self, slot: int, req: Request, off: int, t_admit: float, t0: float):
        try:
            fut = self.plans.pop(req.rid, None)
            ops = fut.result() if fut is not None else None
            t_planned = time.perf_counter() - t0
            marks: List[float] = []
            amps, norm, sweeps = run_one(self.torch, self.streams[slot], req, self.kmax,
                                         self.mfma_min_k, ops=ops, marks=marks,
                                         dev_ptr=self.arena.base + off)
            t_done = time.perf_counter() - t0
            res = Result(req.rid, req.circuit.n, amps, norm, req.t_arrival, t_admit, t_done, sweeps,
                         t_planned, (marks[0] - t0) if marks else t_planned, marks[1] if len(marks) > 1 else 0.0)
        except Exception as e:            # reported, never swallowed
            res = None
            err = f"request {req.rid}: {e}"
        with self.cv:
            self._finish(req, res, None if res is not None else err, slot, off)

    def serve(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Run the trace; with realtime=False every request is available at t=0."""
        for r in requests:
            if state_bytes(r.circuit.n) > self.arena.top:
                raise ValueError(f"request {r.rid} needs more than the HBM budget")
        arrivals = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
        queue: List[Request] = []
        nxt = 0
        threads = []
        t0 = time.perf_counter()
        with self.cv:
            while len(self.results) + len(self.errors) < len(requests):
                now = time.perf_counter() - t0
                while nxt < len(arrivals) and (not realtime or arrivals[nxt].t_arrival <= now):
                    queue.append(arrivals[nxt])
                    if self.pool is not None:
                        self.plans[arrivals[nxt].rid] = self.pool.submit(plan_request, arrivals[nxt].circuit,
                                                                         self.kmax)
                    nxt += 1
                # admit in arrival order while a slot is free and the state
                # gets a block of the arena
                while queue and self.free_slots:
                    off = self.arena.alloc(state_bytes(queue[0].circuit.n))
                    if off is None:
                        break
                    req = queue.pop(0)
                    slot = self.free_slots.pop()
                    self.mem_used += self.arena.block_size(state_bytes(req.circuit.n))
                    self.inflight += 1
                    self.max_inflight = max(self.max_inflight, self.inflight)
                    th = threading.Thread(target=self._run_worker,
                                          args=(slot, req, off, time.perf_counter() - t0, t0), daemon=True)
                    th.start()
                    threads.append(th)
                timeout = None
                if realtime and nxt < len(arrivals):
                    timeout = max(0.0, arrivals[nxt].t_arrival - (time.perf_counter() - t0))
                self.cv.wait(timeout=timeout if timeout is not None else 1.0)
        for th in threads:
            th.join()
        if self.errors:
            raise RuntimeError("; ".join(self.errors[:5]))
        return [self.results[r.rid] for r in requests]


def summarize(results: List[Result]) -> Dict[str, float]:
    lat = np.array([r.latency for r in results])
    first = min(r.t_arrival for r in results)
    last = max(r.t_done for r in results)
    return {"completed": len(results), "circuits_per_s": len(results) / (last - first),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "makespan_s": last - first,
            # where a request's time goes: queued for admission, waiting for
            # its plan after admission, allocation + queueing, device work
            "mean_wait_admit_s": float(np.mean([r.t_admit - r.t_arrival for r in results])),
            "mean_wait_plan_s": float(np.mean([max(0.0, r.t_planned - r.t_admit) for r in results])),
            "mean_queue_s": float(np.mean([max(0.0, r.t_queued - r.t_planned) for r in results])),
            "mean_run_s": float(np.mean([r.t_done - r.t_queued for r in results])),
            # the requests' sweep and staged-pass launch times summed, over the
            # makespan: not a busy fraction, since requests on different slot
            # streams share the device and each counts its whole launch time
            # (above 1 where they overlap)
            "launch_time_over_makespan": float(sum(r.device_ms for r in results) * 1e-3 / (last - first))}
