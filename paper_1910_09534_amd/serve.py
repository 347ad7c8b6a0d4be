"""Request server: simulate-and-return-amplitudes requests with continuous
batching on one GPU.

Each request carries a circuit and the bitstrings whose amplitudes it wants.
The admission loop keeps requests in arrival order and admits the head of
the queue as soon as a slot is free and its complex64 state (2^n x 8 bytes)
fits in the remaining HBM budget; admitted requests run concurrently, each
on its own slot stream, so requests that arrive while others are on the GPU
start as soon as memory and a slot free up and their kernels overlap on the
device.  A slot worker plans the circuit (host), creates a resident state
in a buffer from torch's caching allocator (no device-wide allocation
stalls), enqueues the fused sweeps through the C-ABI, and reduces the
requested amplitudes and the norm in FP64.  Latency = completion - arrival.

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

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def state_bytes(n: int) -> int:
    return (1 << n) * 8


def plan_request(circuit, kmax: int):
    """Single-heuristic staged plan (fast enough to sit inside the request
    path): blocks ordered and widened for staged passes."""
    ops = planner.plan_fast(circuit.gates, kmax)
    for o in ops:
        o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    return ops


def run_one(torch, stream, req: Request, kmax: int, mfma_min_k: int = 4):
    """Plan and simulate one request on `stream`; returns (amps, norm, sweeps)."""
    n = req.circuit.n
    ops = plan_request(req.circuit, kmax)
    with torch.cuda.stream(stream):
        buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    # the buffer's old contents are kept and the reset deferred: the first
    # pass builds |0...0> itself, so no fill kernel writes the whole buffer
    h = sv.create_state_ext(n, 0, "c64", stream.cuda_stream, buf.data_ptr(), buf.numel() * 8, keep=True)
    try:
        sv.reset(h)
        sv.set_option(h, sv.SV_OPT_MFMA, mfma_min_k)
        sv.set_option(h, sv.SV_OPT_STAGE, planner.stage_tmax(n))
        planner.enqueue(h, ops, sv.SV_C64)
        amps, stats = sv.reduce_slices(h, req.bits)
    finally:
        sv.destroy_state(h)
    del buf
    return amps, stats[0], sum(1 for o in ops if o.kind == "dense")


class Server:
    def __init__(self, budget_bytes: float = 250e9, slots: int = 8, kmax: int = 5,
                 mfma_min_k: int = 4):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.kmax = kmax
        self.mfma_min_k = mfma_min_k
        self.streams = [torch.cuda.Stream() for _ in range(slots)]   # default priority
        self.free_slots = list(range(slots))
        self.mem_used = 0
        self.cv = threading.Condition()
        self.results: Dict[int, Result] = {}
        self.errors: List[str] = []
        self.max_inflight = 0
        self.inflight = 0

    def _worker(self, slot: int, req: Request, t_admit: float, t0: float):
        try:
            amps, norm, sweeps = run_one(self.torch, self.streams[slot], req, self.kmax,
                                         self.mfma_min_k)
            t_done = time.perf_counter() - t0
            res = Result(req.rid, req.circuit.n, amps, norm, req.t_arrival, t_admit, t_done, sweeps)
        except Exception as e:            # reported, never swallowed
            res = None
            err = f"request {req.rid}: {e}"
        with self.cv:
            if res is not None:
                self.results[req.rid] = res
            else:
                self.errors.append(err)
            self.mem_used -= state_bytes(req.circuit.n)
            self.free_slots.append(slot)
            self.inflight -= 1
            self.cv.notify_all()

    def serve(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Run the trace; with realtime=False every request is available at t=0."""
        for r in requests:
            if state_bytes(r.circuit.n) > self.budget:
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
                    nxt += 1
                # admit in arrival order while a slot is free and the state fits
                while queue and self.free_slots and \
                        self.mem_used + state_bytes(queue[0].circuit.n) <= self.budget:
                    req = queue.pop(0)
                    slot = self.free_slots.pop()
                    self.mem_used += state_bytes(req.circuit.n)
                    self.inflight += 1
                    self.max_inflight = max(self.max_inflight, self.inflight)
                    th = threading.Thread(target=self._worker,
                                          args=(slot, req, time.perf_counter() - t0, t0), daemon=True)
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
            "makespan_s": last - first}
