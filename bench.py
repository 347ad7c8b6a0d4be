#!/usr/bin/env python3
"""Benchmark: amplitude-updates/s of the sliced state-vector path on one MI355X.

Workload (default): the 30-qubit 5x6-grid ABCDCDAB random circuit of depth 14
(621 gates: 450 single-qubit + 171 fSim), complex64 state of 2^30
amplitudes (8 GiB, resident in HBM), gates aggregated into dense blocks of
at most 5 qubits, output = norm + amplitudes of 2^16 seeded bitstrings with
FP64 cross-entropy sums.

One step = reset the state to |0...0> + every HBM pass of the planned
circuit (staged passes of several 4/5-qubit blocks, single sweeps for the
rest) + the FP64 gather / norm / cross-entropy reduction, with the circuit
already planned (host planning is not timed) and the state already
allocated in HBM.  After the reset, passes visit only the tiles whose
amplitudes can be non-zero until every qubit has been touched (the others
are zero and are zero-filled if still unwritten when the state is read);
amps_visited_frac gives the share of the full passes' amplitudes visited,
and dense_start the same steps with every pass over the whole state.

roofline: the kernel kind with the most time in the timed steps.  Staged
passes in the split-fp16 form (the default: complex64 products on the fp16
matrix cores, 24 2^k issued flops per amplitude per block, a small share of
the fp16 peak) are HBM bound: 16 bytes per amplitude visited, 8 when the
pass starts from |0...0> or takes an amplitude as zero; the fp32 figures
(algorithmic flops = 8 2^k - 2 per amplitude per block, the complex dot
product, over the fp32 matrix peak) stay in the line for comparison with
the fp32 form (3M, 6 2^k issued), which is matrix-core bound.  Single
sweeps: HBM bound, 16 bytes per amplitude per launch.  Durations from HIP
events on the kernels' stream; hbm_frac_run: the bytes those launches
moved per step over the step time.

value = 621 * 2^30 * steps / t  (each circuit gate counted once, the
un-aggregated work over aggregated time).

Other workloads (one JSON line each, same fields where they apply):
  --config 3   sliced run through the pinned host tier: ABCDCDAB depth 20 on the
               near-square grid of --n qubits (default 34: 16 slices of 2^30
               amplitudes, 128 GiB of pinned host memory), slice sets = the
               four corners and the central 2 x 2 block, alternating per
               phase, FP64 reduction of 2^20 bitstrings.

  --config 4   batch of 256 independent ABCDCDAB circuits (n ~ U{20..28},
               depth ~ U{10..20}, complex64) recorded as one graph-captured
               batch; fusion width (k in 3..6) and staged tile limit (12..14
               positions) autotuned per qubit count on this GPU;
               1024 bitstrings per circuit; compared with the complex128 batch.

  --config 5   serving: seeded trace of 1000 Poisson arrivals at 50 req/s,
               n ~ U{16..32}, depth ~ U{8..20}, 1024 bitstrings + norm per
               request, complex64 states admitted by a 250 GB HBM budget,
               continuous batching over 8 slot streams; circuits/s and
               p50 / p99 latency (plus a lighter trace at about 80% load).

  --config 7   resident re-layouts of the 30-qubit complex64 state (random,
               reversed and half-swapped orders), HBM roofline of the
               tiled permutation kernel.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--kmax 5] [--config 2|3|4|5|6|7]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("amp-updates/s & % HBM peak, 30q d14 complex64; served circuits/s + p99 latency")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP16_PEAK_TFLOPS = 2500.0          # dense fp16 matrix cores
FP64_PEAK_TFLOPS = 78.6            # FP64 (vector and matrix cores)


KERNEL_SOURCES = ("paper_1910_09534_amd/csrc/sv_device.h", "paper_1910_09534_amd/csrc/sv_kernels.hip",
                  "paper_1910_09534_amd/csrc/sv_mfma.hip", "paper_1910_09534_amd/csrc/sv_stage.hip",
                  "paper_1910_09534_amd/csrc/sv_internal.h")
TRAFFIC_FILE = "profiles/staged_pass_30q_d14_traffic.json"
BATCH_TUNED = "profiles/batch_256_circuits_tuned.json"


def kernel_hash() -> str:
    """Hash of the kernel sources with comments and blank space removed (a
    comment edit does not invalidate the counter figures)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def counter_traffic(kind: str, alg_bytes: float):
    """HBM bytes per launch of one kernel kind ("staged" passes or single
    "sweep"s) from the committed counter runs (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy of known size), or None when the kernel sources
    changed since the counters were taken or the launches moved other
    algorithmic bytes (another plan)."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None
    e = d.get("per_kind", {}).get(kind, {})
    if abs(e.get("algorithmic_bytes_per_launch", 0.0) - alg_bytes) > 1e-6 * alg_bytes:
        return None
    return e.get("traffic_bytes_per_launch")


def calibrate_copy() -> int:
    import torch
    torch.cuda.set_device(0)
    nbytes = 4 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)
    return 0


def cpu_baseline(circuit, budget_s: float = 15.0):
    """The oracle as it stands (plain per-gate complex128 simulation, OpenMP
    over all host cores) on a bounded sample of the same workload: the first
    gates of the same circuit on the full 2^n state, until `budget_s`."""
    from oracle import oracle as orc
    n = circuit.n
    psi = orc.zero_state(n)
    done = 0
    t0 = time.perf_counter()
    for g in circuit.gates:
        orc.apply_dense(psi, g.qubits, g.matrix)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t = time.perf_counter() - t0
    del psi
    host = host_info()
    single = single_core_points(orc)
    return {"value": done * float(1 << n) / t, "unit": "amp-updates/s", "cores": orc.threads(),
            "kind": "oracle",
            "sample": f"first {done} of {len(circuit.gates)} gates of the same {n}-qubit circuit "
                      f"on the full 2^{n} complex128 state ({t:.1f} s)",
            "host": host,
            # a per-gate sweep reads and writes 32 B per complex128 amplitude
            "host_copy_bound_amp_updates_per_s": host["copy_GBps"] * 1e9 / 32.0,
            "single_core": single}


def single_core_points(orc, budget_s: float = 3.0):
    """The oracle on one core: the whole 16-qubit depth-8 circuit (all 192
    gates), and the first gates of a 24-qubit depth-14 circuit for ~3 s."""
    from paper_1910_09534_amd import workload as W
    nt = orc.threads()
    out = {}
    try:
        orc.set_threads(1)
        c1 = W.config_circuit(1)
        t0 = time.perf_counter()
        orc.simulate(c1)
        t = time.perf_counter() - t0
        out["16q_d8_all_gates"] = len(c1.gates) * float(1 << c1.n) / t
        c24 = W.sycamore_circuit(24, 14, seed=1024)
        psi = orc.zero_state(24)
        done = 0
        t0 = time.perf_counter()
        for g in c24.gates:
            orc.apply_dense(psi, g.qubits, g.matrix)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        t = time.perf_counter() - t0
        out["24q_d14_first_gates"] = done * float(1 << 24) / t
        out["unit"] = "amp-updates/s"
    finally:
        orc.set_threads(nt)
    return out


def host_info():
    """CPU model, logical CPUs and a STREAM-like copy rate (1 GiB, one
    numpy copy per logical CPU in parallel, best of 3) of the machine the
    oracle runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    from concurrent.futures import ThreadPoolExecutor
    a = np.ones(1 << 27, dtype=np.float64)        # 1 GiB
    b = np.empty_like(a)
    nt = os.cpu_count() or 1
    step = -(-a.size // nt)
    spans = [(i, min(i + step, a.size)) for i in range(0, a.size, step)]

    def part(sp):
        np.copyto(b[sp[0]:sp[1]], a[sp[0]:sp[1]])

    best = float("inf")
    with ThreadPoolExecutor(nt) as ex:
        for _ in range(3):
            t0 = time.perf_counter()
            list(ex.map(part, spans))
            best = min(best, time.perf_counter() - t0)
    gbps = 2 * a.nbytes / best / 1e9               # read + write
    del a, b
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "copy_GBps": round(gbps, 1)}


def time_dense_start(h, circ, bits, args) -> float:
    """ms per step of the headline steps with every pass over the whole
    state (no sparse start after the reset), the plan ranked for that."""
    import torch
    from paper_1910_09534_amd import planner, sv
    dense_ops = planner.pack(planner.plan(circ.gates, args.kmax), sv.SV_C64)

    def dense_step():
        sv.reset(h)
        planner.enqueue(h, dense_ops, sv.SV_C64)
        return sv.reduce_slices(h, bits)

    sv.set_option(h, sv.SV_OPT_SPARSE_START, 0)
    dense_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        amps, stats = dense_step()
    torch.cuda.synchronize()
    sv.set_option(h, sv.SV_OPT_SPARSE_START, 1)
    return 1e3 * (time.perf_counter() - t0) / args.steps, amps, stats


def bench_c128(circ, bits, args, steps: int = 3):
    """The same 30-qubit workload in complex128 (FP64 arithmetic, the paper's
    in-memory precision, Sec. 5) on the same GPU, in two forms, the faster
    kept: runs of 4/5-qubit blocks as FP64 staged passes (3M on the FP64
    matrix cores, one 512-lane workgroup per CU; planned as the complex64
    headline, from a reset), or every block as a single sweep on the vector
    units (HBM bound: 32 bytes per amplitude per sweep); blocks of at most
    kmax = 4 or 5 qubits; FP64 reduction; amplitudes against the stored
    oracle amplitudes (tolerance 1e-12).  Returns a dict for the line."""
    import torch
    from paper_1910_09534_amd import planner, sv
    n = circ.n
    buf = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    h = sv.create_state_ext(n, 0, "c128", stream, buf.data_ptr(), buf.numel() * 16)
    best = None
    tried = []
    try:
        for kmax in ([args.c128_kmax] if args.c128_kmax else [4, 5]):
            for staged in (True, False):
                tmax = planner.stage_tmax(n, "c128")
                sv.set_option(h, sv.SV_OPT_STAGE, tmax if staged else 0)
                ops = (planner.plan(circ.gates, kmax, sparse_start=True, tmax=tmax) if staged
                       else planner.plan(circ.gates, kmax, staged=False))
                packed = planner.pack(ops, sv.SV_C128)

                def step():
                    sv.reset(h)
                    planner.enqueue(h, packed, sv.SV_C128)
                    return sv.reduce_slices(h, bits)

                step()
                sv.sweep_profile(h)
                sv.set_option(h, sv.SV_OPT_TIMING, 1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    amps, stats = step()
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                prof = sv.sweep_profile(h)
                sv.set_option(h, sv.SV_OPT_TIMING, 0)
                ms = 1e3 * t / steps
                kind = "staged" if prof["staged"]["ms"] > prof["sweep"]["ms"] else "sweep"
                p = prof[kind]
                gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] else 0.0
                tf = p["flops"] / (p["ms"] * 1e-3) / 1e12 if p["ms"] else 0.0
                issued = p["issued"] / (p["ms"] * 1e-3) / 1e12 if p["ms"] else 0.0
                if kind == "staged":
                    roof = {"kernel": "k_stage64 (staged pass: 2-8 dense 4/5-qubit blocks per HBM pass, FP64 3M on "
                                      "the FP64 matrix cores)",
                            "hbm": {"achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)},
                            "fp64": {"achieved_tflops": round(tf, 2), "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                     "issued_tflops": round(issued, 2),
                                     "issued_frac": round(issued / FP64_PEAK_TFLOPS, 4)}}
                    if issued / FP64_PEAK_TFLOPS > gbs / HBM_PEAK_GBS:
                        roof.update({"bound": "mfma", "achieved": round(issued, 2), "peak": FP64_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": round(issued / FP64_PEAK_TFLOPS, 4)})
                    else:
                        roof.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)})
                else:
                    roof = {"bound": "hbm", "kernel": "k_dense<double> (one dense block per HBM pass, FP64)",
                            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(gbs / HBM_PEAK_GBS, 4)}
                roof.update({"avg_launch_ms": round(p["ms"] / max(p["count"], 1), 4),
                             "launches_per_step": p["count"] // steps,
                             "share_of_step": round(p["ms"] / (steps * ms), 4)})
                r = {"kmax": kmax, "form": "staged" if staged else "sweeps", "ms_per_step": round(ms, 2),
                     "value": len(circ.gates) * float(1 << n) / (ms * 1e-3),
                     "unit": "amp-updates/s", "dtype": "c128", "steps": steps,
                     "staged_passes": prof["staged"]["count"] // steps, "sweeps": prof["sweep"]["count"] // steps,
                     "roofline": roof, "accuracy": accuracy_vs_stored(amps, stats, bits)}
                if r["accuracy"]:
                    r["accuracy"]["tolerance"] = 1e-12
                tried.append({"kmax": kmax, "form": r["form"], "ms_per_step": r["ms_per_step"]})
                if best is None or r["ms_per_step"] < best["ms_per_step"]:
                    best = r
    finally:
        sv.destroy_state(h)
        del buf
        torch.cuda.empty_cache()
    if best is not None:
        best["tried"] = tried
    return best


GOLDEN_HEADLINE = os.path.join(ROOT, "tests", "golden", "headline_30q_d14.npz")


def time_single_blocks(h, n: int, reps: int = 4) -> dict:
    """One lone unitary 5-qubit block on the dense resident state (after the
    headline steps), at three target sets: as a one-block staged pass (the
    route a lone unitary block takes; tile of 14 positions) and as a plain
    fused sweep (`k_dense_mfma`).  `reps` launches after one warm-up, HIP
    events on the state's stream: the best and the average launch, each
    with its HBM fraction of the 16 B moved per amplitude."""
    from paper_1910_09534_amd import planner, sv
    from paper_1910_09534_amd import workload as W
    u = W.random_unitary(32, np.random.default_rng(55)).astype(np.complex64)
    out = {}
    sv.set_option(h, sv.SV_OPT_TIMING, 1)
    for qs in ([0, 1, 2, 3, 4], [10, 11, 12, 13, 14], [20, 21, 22, 23, 24]):
        row = {}
        for form, t in (("staged", planner.stage_tmax(n)), ("sweep", 0)):
            sv.set_option(h, sv.SV_OPT_STAGE, t)
            runs = []
            for i in range(reps + 1):
                sv.sweep_profile(h)
                sv.apply_fused(h, qs, u, "c64")
                sv.sync_state(h)
                p = sv.sweep_profile(h)
                if i:
                    runs.append((p["staged"]["ms"] + p["sweep"]["ms"], p["staged"]["bytes"] + p["sweep"]["bytes"]))
            best = min(runs)
            avg = sum(r[0] for r in runs) / len(runs)
            row[form] = {"ms": round(best[0], 4), "hbm_frac": round(best[1] / (best[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "avg_ms": round(avg, 4), "bytes": best[1]}
        out["-".join(str(q) for q in (qs[0], qs[-1]))] = row
    sv.set_option(h, sv.SV_OPT_TIMING, 0)
    sv.set_option(h, sv.SV_OPT_STAGE, planner.stage_tmax(n))
    return out


def accuracy_vs_stored(amps, stats, bits):
    """Relative L2 error of the step's amplitudes against the complex128
    amplitudes the CPU oracle stored for the same circuit and bitstrings
    (tests/golden/make_golden.py); norm and cross-entropy sums beside it.
    Computed after the timed region; None if the file is absent."""
    if not os.path.exists(GOLDEN_HEADLINE):
        return None
    g = np.load(GOLDEN_HEADLINE)
    if not np.array_equal(g["bitstrings"], bits):
        return None
    ref = g["amps"]
    err = float(np.linalg.norm(amps - ref) / np.linalg.norm(ref))
    return {"rel_l2_vs_oracle": err, "tolerance": 1e-4,
            "norm": stats[0], "norm_oracle": float(g["norm"]),
            "sum_Np": stats[1], "sum_Np_oracle": float(g["xeb"][0]),
            "sum_ln_Np": stats[2], "sum_ln_Np_oracle": float(g["xeb"][1]),
            "oracle": "complex128 CPU oracle, one gate at a time (stored amplitudes)"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kmax", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense-start", action="store_true",
                    help="skip the comparison run with dense passes (profiling: every launch is a step's)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--pins", action="store_true", help="config 3: also run the mirror pin")
    ap.add_argument("--batch-unstaged", action="store_true",
                    help="config 4: autotuned single sweeps instead of staged passes")
    ap.add_argument("--slots", type=int, default=0, help="config 5: slot streams (default 8)")
    ap.add_argument("--tune-cache", default=None,
                    help="config 4: JSON file of tuned fusion widths and tile limits (read if present, else written)")
    ap.add_argument("--defer-cycles", type=int, default=2, help="config 6: cycles run as two tensors")
    ap.add_argument("--tier-dir", default=None,
                    help="config 3: keep the host tier in files in this directory (one per logical file)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="config 6: skip the whole deferred run after the timed contractions (profiling)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving summary in the default line")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests of the serving summary in the default line")
    ap.add_argument("--no-single-block", action="store_true",
                    help="leave out the lone 5-qubit block timings after the headline steps")
    ap.add_argument("--no-contraction", action="store_true",
                    help="leave out the contraction-deferral timings of the default line")
    ap.add_argument("--no-batch", action="store_true",
                    help="leave out the 256-circuit batch summary of the default line")
    ap.add_argument("--no-c128", action="store_true",
                    help="skip the complex128 form of the default workload")
    ap.add_argument("--c128-kmax", type=int, default=0,
                    help="fusion width of the complex128 form (0: try 4 and 5, keep the faster)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 4 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args(argv)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design only.", file=sys.stderr)
        return 2

    if args.config == 3:
        return bench_sliced(args)
    if args.config == 4:
        return bench_batch(args)
    if args.config == 5:
        return bench_serve(args)
    if args.config == 6:
        return bench_contract(args)
    if args.config == 8:
        return bench_single(args)
    if args.config == 7:
        return bench_permute(args)

    # planning processes for the serving summary, started before this
    # process touches the GPU
    from paper_1910_09534_amd import serve as serve_mod
    pool = None if args.no_serve else serve_mod.planning_pool(PLAN_WORKERS)

    import torch
    from paper_1910_09534_amd import planner, sv
    from paper_1910_09534_amd import workload as W

    circ = W.config_circuit(2)
    bits = W.config_bitstrings(2)
    n = circ.n
    ops = planner.plan(circ.gates, args.kmax, sparse_start=True)   # each step starts from a reset
    for o in ops:                                 # pre-cast once (host, untimed)
        o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    pst = planner.stats(ops)
    ndense = pst["dense"]

    torch.cuda.set_device(0)
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    h = sv.create_state_ext(n, 0, "c64", stream, buf.data_ptr(), buf.numel() * 8)
    sv.set_option(h, sv.SV_OPT_STAGE, planner.stage_tmax(n))   # the tile limit the plan was made for
    packed = planner.pack(ops, sv.SV_C64)          # the whole plan queued by one library call

    def step():
        sv.reset(h)
        planner.enqueue(h, packed, sv.SV_C64)
        return sv.reduce_slices(h, bits)

    for _ in range(args.warmup):
        step()
    sv.sweep_profile(h)                            # clear
    sv.set_option(h, sv.SV_OPT_TIMING, 1)          # HIP events around every sweep / staged pass
    c0 = sv.counters(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        amps, stats = step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_per_step = 1e3 * t / args.steps
    gates = len(circ.gates)
    value = gates * float(1 << n) * args.steps / t
    c1 = sv.counters(h)
    passes = (c1["dense_sweeps"] - c0["dense_sweeps"]) / args.steps

    # per kernel kind, every launch of the timed steps bracketed by HIP events
    # on the stream the kernels run on; the dominant kind is the roofline's
    prof = sv.sweep_profile(h)
    forms = sv.stage_forms(h)
    split_form = forms["split"] > 0 and forms["fp32"] == 0
    sv.set_option(h, sv.SV_OPT_TIMING, 0)
    visited = (c1["amps_swept"] - c0["amps_swept"]) / args.steps

    # for comparison: every pass over the whole state (no sparse start
    # after the reset), with the plan ranked for that
    accuracy = accuracy_vs_stored(amps, stats, bits)
    dense_ms = dense_acc = None
    if not args.no_dense_start:
        dense_ms, damps, dstats = time_dense_start(h, circ, bits, args)
        dense_acc = accuracy_vs_stored(damps, dstats, bits)
    single = None if args.no_single_block else time_single_blocks(h, n)

    def kind_roof(kind):
        p = prof[kind]
        if p["count"] == 0:
            return None
        avg_ms = p["ms"] / p["count"]
        gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        tflops = p["flops"] / (p["ms"] * 1e-3) / 1e12          # algorithmic
        issued = p["issued"] / (p["ms"] * 1e-3) / 1e12         # as executed (3M on the matrix cores)
        fp16 = kind == "staged" and split_form
        ipeak = FP16_PEAK_TFLOPS if fp16 else FP32_PEAK_TFLOPS
        r = {"launches": p["count"], "avg_launch_ms": round(avg_ms, 4),
             "share_of_step": round(p["ms"] / (args.steps * ms_per_step), 4),
             "hbm": {"achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": p["bytes"] / p["count"]},
             "fp32": {"achieved_tflops": round(tflops, 2), "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
                      "flops_per_launch": p["flops"] / p["count"]},
             "issued": {"dtype": "fp16" if fp16 else "fp32", "tflops": round(issued, 2), "peak": ipeak,
                        "frac": round(issued / ipeak, 4)},
             "traffic": counter_traffic(kind, p["bytes"] / p["count"])}
        if kind == "staged" and fp16:
            r.update({"kernel": "k_stage, split-fp16 form (staged pass: 2-8 dense 4/5-qubit blocks per HBM "
                                "pass, fp16 matrix cores)",
                      "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)})
        elif kind == "staged":
            r.update({"kernel": "k_stage, fp32 form (staged pass: 2-8 dense 4/5-qubit blocks per HBM pass, "
                                "fp32 matrix cores)",
                      "bound": "mfma", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4)})
        else:
            r.update({"kernel": "k_dense / k_dense_mfma (one dense block per HBM pass)",
                      "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)})
        return r

    kinds = {k: kind_roof(k) for k in ("staged", "sweep")}
    dom = max((k for k in kinds if kinds[k]), key=lambda k: prof[k]["ms"])
    roof = dict(kinds[dom])
    roof = {key: roof[key] for key in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                       "avg_launch_ms", "launches", "share_of_step", "hbm", "fp32", "issued")}
    other = [k for k in kinds if k != dom and kinds[k]]
    if other:
        roof["other_kernel"] = kinds[other[0]]
    run_bytes = (prof["staged"]["bytes"] + prof["sweep"]["bytes"]) / args.steps
    run_hbm_frac = run_bytes / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9)

    sv.destroy_state(h)
    del buf
    torch.cuda.empty_cache()

    c128 = None if args.no_c128 else bench_c128(circ, bits, args)
    batch = None
    if not args.no_batch:
        # the batch workload with the committed tuned table (autotuned on an
        # MI355X by bench.py --config 4 --tune-cache ...), replays timed on
        # the host; its parity with the oracle is a GPU test
        tc = os.path.join(ROOT, BATCH_TUNED)                # tuned here (not saved) if it is missing
        b = batch_summary(args, 256, 3, 1, tc if os.path.exists(tc) else None, compare_c128=False)
        batch = {k: b[k] for k in ("value", "unit", "ms_per_step", "steps", "amp_updates_per_s", "kmax_by_n",
                                   "stage_t_by_n", "t_tune_s", "t_plan_s")}
        batch["ms_per_batch"] = batch.pop("ms_per_step")
        batch["launches_per_batch"] = b["config"]["launches_per_batch"]
        batch["workload"] = b["config"]["workload"]
        torch.cuda.empty_cache()
    contraction = None
    if not args.no_contraction:
        # the contraction-deferral leg (--config 6) without its oracle
        # sample and deferred pipeline: both kernels timed with HIP events
        ca = argparse.Namespace(**vars(args))
        ca.n, ca.steps, ca.warmup, ca.no_cpu_baseline, ca.no_pipeline = 0, 3, 1, True, True
        c = contract_summary(ca)
        r = c["roofline"]
        contraction = {"workload": c["config"]["workload"], "kernel": "k_contract_split",
                       "avg_launch_ms": r["avg_launch_ms"], "issued_tflops": r["achieved"],
                       "frac_of_fp16_peak": r["frac"], "complex_equivalent_tflops": r["complex_equivalent_tflops"],
                       "traffic": r["traffic"], "fp32_form_avg_launch_ms": r["fp32_form"]["avg_launch_ms"]}
        torch.cuda.empty_cache()
    serving = None
    if pool is not None:
        serving = serve_summary(pool, args.kmax, count=args.serve_requests)
        pool.shutdown()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(circ, args.cpu_budget)

    line = {
        "metric": METRIC, "value": value, "unit": "amp-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "30-qubit 5x6 ABCDCDAB random circuit, depth 14, complex64, "
                               "fusion k<=%d (fSim phases applied to the outputs of their block), "
                               "norm + 2^16 bitstrings" % args.kmax,
                   "n": n, "depth": circ.depth, "gates": gates, "kmax": args.kmax,
                   "bitstrings": int(bits.size), "blocks": ndense, "hbm_passes": passes,
                   "k_hist": pst["k_hist"]},
        "hbm_frac_run": round(run_hbm_frac, 4),
        "amps_visited_frac": round(visited / (passes * float(1 << n)), 4),
        "accuracy": accuracy,
        "dense_start": None if dense_ms is None else
        {"ms_per_step": round(dense_ms, 3), "value": gates * float(1 << n) / (dense_ms * 1e-3),
         "rel_l2_vs_oracle": dense_acc and dense_acc["rel_l2_vs_oracle"]},
        "single_block_30q": single,
        "block_amp_updates_per_s": ndense * float(1 << n) * args.steps / t,
        "norm": stats[0],
        "roofline": roof,
        "c128": c128,
        "batch": batch,
        "contraction": contraction,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_sliced(args) -> int:
    """Sliced evolution with slices staged through pinned host memory."""
    import torch
    from paper_1910_09534_amd import planner, runner, sv
    from paper_1910_09534_amd import workload as W

    n = args.n or 34
    depth = 20
    circ = W.sycamore_circuit(n, depth, seed=1003)
    bits = W.bitstrings(n, 1 << 20, seed=2003)
    A, B = runner.grid_slice_sets(n)
    t0 = time.perf_counter()
    sched = planner.phase_schedule(circ, A, B, args.kmax)
    for ph in sched.phases:
        for o in ph.ops:
            o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    t_plan = time.perf_counter() - t0
    torch.cuda.set_device(0)
    mask = sum(1 << q for q in sched.phases[0].sliced)
    t0 = time.perf_counter()
    st = sv.State(n, mask, "c64", tier=True, tier_dir=args.tier_dir)
    sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(n - len(sched.phases[0].sliced)))
    t_alloc = time.perf_counter() - t0
    print(f"# tier allocated in {t_alloc:.1f} s; {len(sched.phases)} phases", file=sys.stderr,
          flush=True)
    sv.set_option(st.h, sv.SV_OPT_TIMING, 1)

    def run(s, label=""):
        t_start = time.perf_counter()
        for i, ph in enumerate(s.phases):
            sv.permute_qubits(st.h, ph.order)      # returns once the previous phase's pass is done
            if i:
                print(f"# {label}phase {i} done at {time.perf_counter() - t_start:.1f} s", file=sys.stderr,
                      flush=True)
            planner.enqueue(st.h, ph.ops, sv.SV_C64)
        out = sv.reduce_slices(st.h, bits, s.trailing)
        print(f"# {label}last phase + reduction done at {time.perf_counter() - t_start:.1f} s",
              file=sys.stderr, flush=True)
        return out

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    amps, stats = run(sched)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    cnt = sv.counters(st.h)
    sweep_ms, nswept = sv.sweep_time(st.h)
    p = (amps.real ** 2 + amps.imag ** 2) * float(1 << n)
    gates = len(circ.gates)
    line = {
        "metric": "sliced host-tier run: amp-updates/s, host-link GB/s", "value": gates * float(1 << n) / t,
        "unit": "amp-updates/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * t, 1),
        "higher_is_better": True, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"{n}-qubit ABCDCDAB depth {depth}, complex64, 4 sliced qubits "
                               f"(16 slices of 2^{n - 4}) in a host-memory tier"
                               + (" backed by files (one per logical file)" if args.tier_dir else "")
                               + ", 2^20 bitstrings",
                   "n": n, "gates": gates, "slice_sets": [list(A), list(B)],
                   "phases": len(sched.phases), "sweeps_per_slice": sum(len(p_.ops) for p_ in sched.phases),
                   "trailing_gates": len(sched.trailing_gate_ids)},
        "host_link_GBps": round((cnt["bytes_h2d"] + cnt["bytes_d2h"]) / t / 1e9, 2),
        "tier": ("files (shared mappings) + pinned bounce buffers" if args.tier_dir else
                 "pinned" if (1 << n) * 8 <= (48 << 30) else "pageable + pinned bounce buffers"),
        "bytes_h2d": cnt["bytes_h2d"], "bytes_d2h": cnt["bytes_d2h"],
        "zero_slices_skipped": cnt["zero_slices_skipped"],
        "dense_sweep_ms_total": round(sweep_ms, 1), "dense_sweeps": nswept,
        "t_alloc_s": round(t_alloc, 1), "t_plan_s": round(t_plan, 2),
        "norm": stats[0], "mean_Np": float(p.mean()), "mean_Np2": float((p ** 2).mean()),
    }
    if args.pins:
        inv = [W.Gate(g.qubits, g.matrix.conj().T) for g in reversed(circ.gates)]
        mirror = W.Circuit(n, circ.gates + inv, 2 * depth)
        sv.reset(st.h)
        ms = planner.phase_schedule(mirror, A, B, args.kmax)
        mb = np.concatenate([np.zeros(1, np.uint64), bits[:4095]])
        ma, _ = run_pins(st, ms, mb, planner, sv)
        print("# mirror pin done", file=sys.stderr, flush=True)
        line["mirror_abs_amp0"] = float(abs(ma[0]))
        line["mirror_max_other"] = float(np.abs(ma[1:]).max())
    st.close()
    print(json.dumps(line), flush=True)
    return 0


def bench_batch(args) -> int:
    """256 independent circuits, one graph-captured batch per step."""
    print(json.dumps(batch_summary(args, args.n or 256, args.steps, args.warmup, args.tune_cache,
                                   compare_c128=not args.no_c128)), flush=True)
    return 0


def batch_summary(args, count: int, steps: int, warmup: int, tune_cache, compare_c128: bool) -> dict:
    """The batch workload's line: `count` circuits of 20-28 qubits, fusion
    width and tile limit per qubit count from `tune_cache` (or tuned on
    this GPU first), `warmup` + `steps` graph replays timed on the host;
    with compare_c128 also the same circuits as a complex128 batch."""
    import torch
    from paper_1910_09534_amd import autotune, planner, runner, sv
    from paper_1910_09534_amd import workload as W

    torch.cuda.set_device(0)
    specs = W.batch_specs(count)
    circs = [W.sycamore_circuit(s["n"], s["depth"], s["seed"]) for s in specs]
    bits = [W.bitstrings(s["n"], 1024, s["bit_seed"]) for s in specs]
    t0 = time.perf_counter()
    ns = sorted({c.n for c in circs})
    if args.batch_unstaged:
        tuned = autotune.tune(ns)
        tuned["stage_t"] = {n: 0 for n in ns}
    elif tune_cache and os.path.exists(tune_cache):
        tuned = autotune.load(tune_cache)
    else:
        # fusion width k in {3..6} and staged tile limit in {12, 13, 14} per
        # qubit count, timed on this GPU
        tuned = autotune.tune_staged(ns)
        if tune_cache:
            autotune.save(tuned, tune_cache)
    tuned.setdefault("mfma_min_k", {n: 4 for n in ns})
    t_tune = time.perf_counter() - t0
    t0 = time.perf_counter()
    staged = not args.batch_unstaged
    # one staged aggregation per circuit (plan_fast): within ~2 % of the full
    # candidate search by the cost model, at 1/35 of its planning time
    plans = [planner.plan_fast(c.gates, tuned["kmax"][c.n], nloc=c.n, sparse_start=True,
                               tmax=tuned["stage_t"][c.n])
             if staged else planner.plan(c.gates, tuned["kmax"][c.n], staged=False) for c in circs]
    for p in plans:
        for o in p:
            o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    t_plan = time.perf_counter() - t0
    res = runner.run_batch(circs, bits, "c64", kmax=tuned["kmax"], mfma_min_k=tuned["mfma_min_k"],
                           graph=True, repeats=warmup + steps, plans=plans, staged=staged,
                           stage_t=tuned["stage_t"] if staged else None)
    times = res["times"][warmup:]
    t = sum(times) / len(times)
    gate_amps = sum(len(c.gates) * float(1 << c.n) for c in circs)
    swept = res["info"]["amps_swept"]
    # complex128 batch on the same GPU (two halves: 227 GiB at once is too close to HBM size)
    err = []
    half = (count + 1) // 2
    t128 = 0.0
    for lo in ((0, half) if compare_c128 else ()):
        sub = slice(lo, min(lo + half, count))
        r = runner.run_batch(circs[sub], bits[sub], "c128", kmax=4, graph=True)
        t128 += r["times"][-1]
        for a64, a128 in zip(res["amps"][sub], r["amps"]):
            err.append(float(np.linalg.norm(a64 - a128) / np.linalg.norm(a128)))
    line = {
        "metric": "batch: circuits/s and amp-updates/s, one graph-captured batch",
        "value": count / t, "unit": "circuits/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(1e3 * t, 2), "higher_is_better": True,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"{count} ABCDCDAB circuits, n ~ U{{20..28}}, depth ~ U{{10..20}}, "
                               "complex64, 1024 bitstrings each",
                   "circuits": count, "gates": sum(len(c.gates) for c in circs),
                   "sweeps": sum(res["sweeps"]), "launches_per_batch": res["info"]["launches"]},
        "amp_updates_per_s": gate_amps / t,
        "amps_visited_per_batch": swept,
        "hbm_GBps_visited": 16.0 * swept / t / 1e9,
        "kmax_by_n": tuned["kmax"], "stage_t_by_n": tuned["stage_t"], "mfma_min_k_by_n": tuned["mfma_min_k"],
        "staged": staged, "tuned_ms_by_n": tuned.get("ms"),
        "t_tune_s": round(t_tune, 2), "t_plan_s": round(t_plan, 2),
        "c128_batch_s": round(t128, 3) if err else None,
        "rel_l2_vs_c128_max": max(err) if err else None,
    }
    return line


def bench_contract(args) -> int:
    """Contraction deferral line (`contract_summary`)."""
    print(json.dumps(contract_summary(args)), flush=True)
    return 0


def contract_summary(args) -> dict:
    """Contraction deferral: the bridging gates of the first cycles of an
    ABCDCDAB circuit as EI / E2Q on two tensors (left and right grid halves),
    then the tensor 1 x tensor 2 contraction over the entanglement indices;
    the contraction is timed (HIP events on its stream)."""
    import torch
    from paper_1910_09534_amd import deferral, planner, runner, sv
    from paper_1910_09534_amd import workload as W

    torch.cuda.set_device(0)
    n = args.n or 30
    depth = 14
    circ = W.sycamore_circuit(n, depth, seed=1006)
    sp = deferral.split(circ, deferral.grid_halves(n), args.defer_cycles)
    n1, n2, e = sp.n1, sp.n2, sp.e
    nt1, nt2 = n1 + e, n2 + e
    # the two tensors on the GPU, entanglement indices at the top positions
    states = []
    for ops, nq, order in ((sp.ops1, nt1, sp.order1), (sp.ops2, nt2, sp.order2)):
        st = sv.State(nq, 0, "c64")
        sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(nq))
        p = planner.plan(ops, args.kmax, nloc=nq, sparse_start=True)
        for o in p:
            o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
        planner.enqueue(st.h, p, st.dtype)
        sv.permute_qubits(st.h, order)
        sv.sync_state(st.h)
        states.append(st)
    p1, _ = sv.device_buffer(states[0].h)
    p2, _ = sv.device_buffer(states[1].h)
    out = torch.empty(1 << (n1 + n2), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fp32):
        for _ in range(args.warmup):
            sv.contract(p1, p2, out.data_ptr(), n1, n2, e, "c64", stream.cuda_stream, fp32=fp32)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            sv.contract(p1, p2, out.data_ptr(), n1, n2, e, "c64", stream.cuda_stream, fp32=fp32)
            b.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, sum(a.elapsed_time(b) for a, b in evs) / args.steps

    # the fp32 3M form for comparison, then the split-fp16 form (the default,
    # whose output the sampled check below reads)
    t32, kms32 = timed(True)
    t, kms = timed(False)
    flops = 8.0 * float(1 << (n1 + n2)) * float(1 << e)        # complex multiply-add per term
    hbm = 8.0 * ((1 << nt1) + (1 << nt2) + (1 << (n1 + n2)))     # read both tensors, write the joint state
    # sampled outputs against the oracle's own tensors (never the GPU's)
    rng = np.random.default_rng(6)
    xs = rng.integers(0, 1 << (n1 + n2), size=1024, dtype=np.int64)
    got = out[torch.from_numpy(xs).cuda()].cpu().numpy().astype(np.complex128)
    for st in states:
        st.close()
    # CPU baseline leg (the only place the oracle runs here): the oracle
    # builds both tensors itself, its values at the sampled outputs are
    # compared with the GPU's, and its contraction is timed on a bounded
    # sample (all of tensor 1 against the first 2^k columns of tensor 2)
    cpu = None
    err = None
    t_or = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        from oracle import deferral as odf
        from oracle import brute
        t_or = time.perf_counter()
        ot = []
        for ops, nq, order in ((sp.ops1, nt1, sp.order1), (sp.ops2, nt2, sp.order2)):
            s = orc.zero_state(nq)
            for g in ops:
                orc.apply_dense(s, list(g.qubits), g.matrix)
            ot.append(brute.permute_state(s, nq, order).reshape(1 << e, -1))
            del s
        x1 = xs & ((1 << n1) - 1)
        x2 = xs >> n1
        ref = np.einsum("ek,ek->k", ot[0][:, x1], ot[1][:, x2])
        t_or = round(time.perf_counter() - t_or, 1)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        k = 4
        while True:
            t1c = time.perf_counter()
            odf.contract_matrix(ot[0].reshape(-1), np.ascontiguousarray(ot[1][:, :1 << k]).reshape(-1),
                                n1, k, e)
            dt = time.perf_counter() - t1c
            if dt > args.cpu_budget / 4 or k >= n2:
                break
            k += 1
        try:
            from threadpoolctl import threadpool_info
            cores = max([p["num_threads"] for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
        except Exception:
            cores = None
        cpu = {"value": 8.0 * float(1 << (n1 + k)) * float(1 << e) / dt / 1e12, "unit": "TFLOP/s",
               "cores": cores, "kind": "oracle",
               "sample": f"contraction of tensor 1 with the first 2^{k} of 2^{n2} columns of tensor 2 "
                         f"(complex128 matrix product, {dt:.1f} s)"}
        del ot
    # the whole deferred run once, for context
    res = None
    if not args.no_pipeline:
        res = runner.simulate_deferred(circ, W.bitstrings(n, 1 << 16, seed=2006), sp.part1,
                                       args.defer_cycles, kmax=args.kmax)
    tf = flops / (kms * 1e-3) / 1e12
    # the kernel's own arithmetic: four real products of three split terms
    # on the fp16 matrix cores, 24 flops per complex multiply-add; the
    # roofline is priced on those (the fp32 form: three real products, 3M)
    flops_split = 3.0 * flops
    tf16 = flops_split / (kms * 1e-3) / 1e12
    flops_3m = 0.75 * flops
    tf3 = flops_3m / (kms32 * 1e-3) / 1e12
    line = {
        "metric": "contraction deferral: tensor 1 x tensor 2 contraction TFLOP/s "
                  "(complex-equivalent, 8 flops per complex multiply-add)",
        "value": tf, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * t, 3), "higher_is_better": True, "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit ABCDCDAB depth {depth}: bridging gates of the first "
                               f"{args.defer_cycles} cycles between the grid halves as EI / E2Q, "
                               f"two tensors of {nt1} and {nt2} qubits ({e} entanglement indices), "
                               f"contracted into the 2^{n1 + n2} joint state",
                   "n": n, "n1": n1, "n2": n2, "e": e, "bridging_gates": sp.n_bridging},
        "roofline": {"bound": "mfma", "achieved": round(tf16, 2), "peak": FP16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf16 / FP16_PEAK_TFLOPS, 4), "traffic": contract_traffic(),
                     "kernel": "k_contract_split (split-fp16 form: complex64 products at single-precision "
                               "accuracy on the fp16 matrix cores)",
                     "avg_launch_ms": round(kms, 4), "flops_per_launch": flops_split,
                     "flops": "24 M N K: four real M x N x K products of three split terms each",
                     "complex_equivalent_tflops": round(tf, 2),
                     "complex_equivalent_frac_of_fp32_peak": round(tf / FP32_PEAK_TFLOPS, 4),
                     "hbm": {"bytes_per_launch": hbm, "achieved_gbs": round(hbm / (kms * 1e-3) / 1e9, 1)},
                     "fp32_form": {"kernel": "k_contract_mfma (3M form on FP32 matrix cores)",
                                   "avg_launch_ms": round(kms32, 4), "achieved": round(tf3, 2),
                                   "peak": FP32_PEAK_TFLOPS, "frac": round(tf3 / FP32_PEAK_TFLOPS, 4),
                                   "flops": "6 M N K: the 3M form's three real M x N x K products",
                                   "traffic": contract_traffic("k_contract_mfma"),
                                   # counter traffic (L2 refills, mostly from the last-level
                                   # cache) as a rate: far below HBM bandwidth, so the refills
                                   # cost the matrix-core-bound kernel no time
                                   "traffic_gbs": None if contract_traffic("k_contract_mfma") is None else
                                   round(contract_traffic("k_contract_mfma") / (kms32 * 1e-3) / 1e9, 1)}},
        "sampled_rel_l2_vs_oracle": err, "oracle_sample_s": t_or,
        "pipeline": None if res is None else
        {"t_run_s": round(res["t_run"], 3), "t_tensors_s": round(res["t_tensors"], 3),
         "contract_ms": round(res["contract_ms"], 3), "norm": res["norm"]},
        "cpu_baseline": cpu,
    }
    return line


def bench_single(args) -> int:
    """A single fused 5-qubit block on a dense 30-qubit complex64 state (the
    fused dense sweep of one aggregate gate, Sec. 5): a lone unitary block
    runs as a one-block staged pass on a 14-position tile; timed at targets
    0-4, 10-14 and 20-24 beside the plain `k_dense_mfma` sweep.  HBM
    roofline of the staged form: 16 B per amplitude over the average launch
    at targets 0-4 and 10-14 (a tile within one 2 MB page group), counter
    traffic from the committed profile."""
    import torch
    from paper_1910_09534_amd import sv
    from paper_1910_09534_amd import workload as W
    torch.cuda.set_device(0)
    n = 30
    st = sv.State(n, 0, "c64")
    rng = np.random.default_rng(8)
    for q0 in range(0, n, 5):                               # blocks covering every qubit: a dense state
        st.fused(list(range(q0, q0 + 5)), W.random_unitary(32, rng))
    sv.sync_state(st.h)
    res = time_single_blocks(st.h, n, reps=max(args.steps, 2))
    st.close()
    low = [res[k]["staged"] for k in ("0-4", "10-14")]
    avg = sum(r["avg_ms"] for r in low) / len(low)
    by = low[0]["bytes"]
    gbs = by / (avg * 1e-3) / 1e9
    line = {"metric": "single fused 5-qubit block on a 30-qubit state: HBM GB/s", "value": gbs, "unit": "GB/s",
            "n_gpus": 1, "steps": max(args.steps, 2), "warmup": 1, "ms_per_step": round(avg, 4),
            "higher_is_better": True, "dtype": "c64", "data": "synthetic",
            "config": {"workload": "30-qubit complex64 state (dense), one random unitary 5-qubit block at "
                                   "targets 0-4, 10-14 and 20-24", "n": n},
            "per_targets": res,
            "roofline": {"bound": "hbm", "kernel": "k_stage<14> (one-block staged pass, split-fp16 form)",
                         "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg, 4),
                         "bytes_per_launch": by,
                         "traffic": profile_traffic("single_block_30q_traffic.json",
                                                    "paper_1910_09534_amd/csrc/sv_stage.hip")}}
    print(json.dumps(line), flush=True)
    return 0


def bench_permute(args) -> int:
    """Resident re-layouts (Sec. 4: the index permutes that re-choose the
    sliced qubits; here the whole 30-qubit complex64 state is re-laid out in
    HBM): random orders, the reversal, and the swap of the low and high
    halves, each timed with HIP events on the state's stream (the tiled
    permutation kernel; the handle's two buffers swap roles, nothing is
    copied back).  HBM roofline: 16 bytes per amplitude per permute."""
    import torch
    from paper_1910_09534_amd import sv
    from paper_1910_09534_amd import workload as W
    torch.cuda.set_device(0)
    n = args.n or 30
    stream = torch.cuda.Stream()
    st = sv.State(n, 0, "c64", stream=stream.cuda_stream)
    rng = np.random.default_rng(7)
    for q0 in range(0, n, 5):                               # blocks covering every qubit: a dense state
        qs = list(range(q0, min(q0 + 5, n)))
        st.fused(qs, W.random_unitary(1 << len(qs), rng))
    bits = W.bitstrings(n, 1 << 12, seed=70)
    ref = st.gather(bits)
    orders = {"random": [int(x) for x in rng.permutation(n)], "reverse": list(range(n))[::-1],
              "halves": list(range(n // 2, n)) + list(range(n // 2))}
    ident = list(range(n))
    res = {}
    all_ms = []
    for name, order in orders.items():
        ms = []
        for _ in range(args.warmup + args.steps):
            for target in (order, ident):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                st.permute(target)
                b.record(stream)
                b.synchronize()
                ms.append(a.elapsed_time(b))
        ms = ms[2 * args.warmup:]
        all_ms += ms
        avg = sum(ms) / len(ms)
        res[name] = {"ms": round(avg, 4), "GBps": round(16.0 * (1 << n) / (avg * 1e-3) / 1e9, 1)}
    exact = bool(np.array_equal(st.gather(bits), ref))
    st.close()
    avg = sum(all_ms) / len(all_ms)
    gbs = 16.0 * (1 << n) / (avg * 1e-3) / 1e9
    line = {"metric": "resident permute: GB/s of the re-layout", "value": gbs, "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(avg, 4), "higher_is_better": True,
            "dtype": "c64", "data": "synthetic",
            "config": {"workload": f"{n}-qubit complex64 state (dense), permutes to random / reversed / "
                                   "half-swapped orders and back", "n": n},
            "per_order": res, "amplitudes_unchanged": exact,
            "roofline": {"bound": "hbm", "kernel": "k_bitperm_tiled (LDS-tiled bit permutation)",
                         "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": profile_traffic("permute_30q_traffic.json", "paper_1910_09534_amd/csrc/sv_kernels.hip")}}
    print(json.dumps(line), flush=True)
    return 0


def contract_traffic(kernel: str = "k_contract_split"):
    """HBM bytes per launch of a contraction kernel from the committed
    counter runs, or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "contract_30q_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash("paper_1910_09534_amd/csrc/sv_contract.hip"):
        return None
    return d.get("per_kernel", {}).get(kernel, {}).get("traffic_bytes_per_launch")


def profile_traffic(name: str, source: str):
    """HBM bytes per launch from a committed counter summary under
    profiles/, or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash(source):
        return None
    return d.get("traffic_bytes_per_launch")


def source_hash(rel: str) -> str:
    import hashlib
    import re
    with open(os.path.join(ROOT, rel)) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return hashlib.sha256(" ".join(src.split()).encode()).hexdigest()[:16]


PLAN_WORKERS = 12          # planning processes of the server (the GPU machine grants 16 CPUs)
SERVE_SLOTS = 8
SERVE_BUDGET = int(250e9)  # HBM budget of the request states


def _build_requests(trace):
    from paper_1910_09534_amd import serve
    from paper_1910_09534_amd import workload as W
    return [serve.Request(t["j"], t["t"], W.sycamore_circuit(t["n"], t["depth"], t["seed"]),
                          W.bitstrings(t["n"], 1024, t["bit_seed"])) for t in trace]


def serve_trace(pool, arena, kmax, count, rate=50.0, slots=None, seed=1005):
    """The seeded serving trace (Poisson arrivals at `rate`, n ~ U{16..32},
    depth ~ U{8..20}, 1024 bitstrings + norm each) through the server, states
    in `arena` (the 250 GB HBM budget); returns (server, results, summary)."""
    from paper_1910_09534_amd import serve
    from paper_1910_09534_amd import workload as W
    reqs = _build_requests(W.serving_trace(count, rate=rate, seed=seed))
    # warm the kernels on a few small requests
    serve.Server(slots=slots or SERVE_SLOTS, kmax=kmax, planner_pool=pool, arena=arena).serve(
        _build_requests(W.serving_trace(8, rate=1000.0, seed=77, nmin=16, nmax=20)), realtime=False)
    srv = serve.Server(slots=slots or SERVE_SLOTS, kmax=kmax, planner_pool=pool, arena=arena)
    res = srv.serve(reqs)
    return srv, res, serve.summarize(res)


def serve_summary(pool, kmax, count):
    """Serving half of the metric for the default line: the first `count`
    requests of the seeded 50 req/s trace."""
    import torch
    from paper_1910_09534_amd import serve
    arena = serve.BuddyArena(torch, SERVE_BUDGET)
    srv, res, s = serve_trace(pool, arena, kmax, count)
    inflight = srv.max_inflight
    del arena, srv                            # the server holds the arena
    torch.cuda.empty_cache()
    mu = s["circuits_per_s"]
    return {"metric": "served circuits/s and p50/p99 latency (continuous batching)",
            "value": mu, "unit": "circuits/s", "requests": count, "arrival_rate": 50.0,
            "p50_latency_s": s["p50_latency_s"], "p99_latency_s": s["p99_latency_s"],
            "makespan_s": s["makespan_s"],
            "mean_wait_admit_s": s["mean_wait_admit_s"], "mean_wait_plan_s": s["mean_wait_plan_s"],
            "mean_queue_s": s["mean_queue_s"], "mean_run_s": s["mean_run_s"], "launch_time_over_makespan": s["launch_time_over_makespan"],
            # measured: arrival rate over the completion rate the server sustained
            "offered_load_rho_measured": 50.0 / mu, "max_inflight": inflight,
            "max_norm_error": float(max(abs(r.norm - 1) for r in res)),
            "planning": f"{PLAN_WORKERS} processes, from arrival", "slots": SERVE_SLOTS}


def bench_serve(args) -> int:
    import torch
    from paper_1910_09534_amd import serve
    from paper_1910_09534_amd import workload as W

    pool = serve.planning_pool(PLAN_WORKERS)          # before the GPU is touched
    torch.cuda.set_device(0)
    count = args.n or 1000
    build = _build_requests
    arena = serve.BuddyArena(torch, SERVE_BUDGET)
    t0 = time.perf_counter()
    srv, res, s50 = serve_trace(pool, arena, args.kmax, count, slots=args.slots)
    t_run = time.perf_counter() - t0
    norms = np.array([r.norm for r in res])
    mu = s50["circuits_per_s"]
    line = {
        "metric": "serving: circuits/s and p50/p99 latency (continuous batching)",
        "value": mu, "unit": "circuits/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"{count} Poisson arrivals at 50 req/s, n ~ U{{16..32}}, "
                               "depth ~ U{8..20}, 1024 bitstrings + norm each, 250 GB HBM budget",
                   "requests": count, "slots": args.slots or SERVE_SLOTS, "kmax": args.kmax},
        "p50_latency_s": s50["p50_latency_s"], "p99_latency_s": s50["p99_latency_s"],
        "mean_latency_s": s50["mean_latency_s"], "makespan_s": s50["makespan_s"],
        "mean_wait_admit_s": s50["mean_wait_admit_s"], "mean_wait_plan_s": s50["mean_wait_plan_s"],
        "mean_queue_s": s50["mean_queue_s"], "mean_run_s": s50["mean_run_s"], "launch_time_over_makespan": s50["launch_time_over_makespan"],
        # measured: arrival rate over the completion rate the server sustained
        "offered_load_rho_measured": 50.0 / mu, "max_inflight": srv.max_inflight,
        "max_norm_error": float(np.abs(norms - 1).max()), "t_run_s": round(t_run, 1),
        "planning": f"{PLAN_WORKERS} processes, from arrival",
    }
    # extra: a lighter trace at about 80% of the measured capacity
    lam = 0.8 * mu
    light = build(W.serving_trace(min(count, 300), rate=lam, seed=1505))
    srv2 = serve.Server(slots=args.slots or SERVE_SLOTS, kmax=args.kmax, planner_pool=pool, arena=arena)
    s80 = serve.summarize(srv2.serve(light))
    line["extra_rho_0.8"] = {"rate": lam, "requests": len(light), **s80}
    pool.shutdown()
    print(json.dumps(line), flush=True)
    return 0


def run_pins(st, sched, bits, planner, sv):
    for ph in sched.phases:
        sv.permute_qubits(st.h, ph.order)
        planner.enqueue(st.h, ph.ops, sv.SV_C64)
    return sv.reduce_slices(st.h, bits, sched.trailing)


if __name__ == "__main__":
    sys.exit(main())
