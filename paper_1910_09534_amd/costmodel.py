"""Running-time model of Sec. 5 (the paper's estimate for Summit), written
from its description so that the tables can be checked and re-targeted.

* Time per aggregate gate on a 45-qubit disk slice: the Cori II figure
  2.38380 s scaled by the HPL ratio Cori II / Summit (14,014.70 / 148,600.00
  TFLOP/s); tensors 1 and 2 (<= 30 qubits) use 0.025097 s.  A row's compute
  time = kernels x slices x time per aggregate gate.
* Achieved FLOP rate of a gate row = gates x 30 flop x amplitudes / its
  compute time (flops counted without aggregation), where 30 = 4 complex
  multiplies (6 flop) + 3 complex additions (2 flop) per output of a 4 x 4
  matrix-vector product.  Amplitudes = 2^(socket rank + 13) (8,192 sockets)
  per disk slice, times the number of slices for the 45-qubit rows; the
  printed rates of the two <= 30-qubit rows count one slice's amplitudes
  (their times still cover every slice).
* Compute subtotal rate = (contraction FLOPs + every gate row's FLOPs) /
  compute time.
* Contraction of tensors 1 and 2: FLOPs / 116.73 PFLOP/s (14.249 TFLOP/s per
  socket: the single-precision rate scaled by 7.8 / 15.7).
* All-to-all: state bytes at 16 B per amplitude / (3.5 GiB/s x 8192
  sockets) per exchange; one exchange per row that has one, a fraction for
  the small rows, and one more per disk read or write.
* Disk: state bytes at 8 B per amplitude / (2 x 2^40 B/s) per transfer.
* Other depths (Tabs. 3 and 4): the 20-cycle table's tensors 1 and 2 and its
  contraction are kept; every further kernel is priced at the 45-qubit rate
  per slice; all-to-alls and disk transfers as above.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

DAY = 86400.0
T_CORI = 2.38380
HPL_CORI = 14014.70
HPL_SUMMIT = 148600.00
T_GATE_45Q = T_CORI * HPL_CORI / HPL_SUMMIT       # 0.22482 s
T_GATE_30Q = 0.025097
CONTRACTION_RATE = 116.73e15                       # FLOP/s
ALLTOALL_RATE = 3.5 * 2 ** 30 * 8192               # B/s, machine-wide
DISK_RATE = 2 * 2 ** 40                            # B/s
FLOP_PER_AMP_2Q = 30
SOCKETS_LOG2 = 13


@dataclasses.dataclass
class Row:
    name: str
    alltoalls: float
    kernels: int
    socket_rank: int
    gates: int


def small_tensor(row: Row) -> bool:
    """Tensors 1 and 2: at most 30 qubits, priced with the 30-qubit figure."""
    return row.name in ("1", "2")


def gate_row_seconds(row: Row, slices: int) -> float:
    t = T_GATE_30Q if small_tensor(row) else T_GATE_45Q
    return row.kernels * slices * t


def gate_row_flops(row: Row, slices: int) -> float:
    amps = 2.0 ** (row.socket_rank + SOCKETS_LOG2)
    if not small_tensor(row):
        amps *= slices
    return row.gates * FLOP_PER_AMP_2Q * amps


def gate_row_pflops(row: Row, slices: int) -> float:
    return gate_row_flops(row, slices) / gate_row_seconds(row, slices) / 1e15


def contraction_seconds(flops: float) -> float:
    return flops / CONTRACTION_RATE


def alltoall_seconds(count: float, n: int) -> float:
    return count * 2.0 ** n * 16 / ALLTOALL_RATE


def disk_seconds(transfers: int, n: int) -> float:
    return transfers * 2.0 ** n * 8 / DISK_RATE


def disk_space_pib(n: int) -> float:
    return 2.0 ** n * 8 / 2 ** 50


def table(n: int, rows: List[Row], contraction_flops: float, disk_transfers: int) -> Dict[str, float]:
    """Recompute a Tab. 1 / Tab. 2 style summary (times in days)."""
    slices = 2 ** (n - 45)
    out: Dict[str, float] = {}
    compute = 0.0
    flops = contraction_flops
    for r in rows:
        s = gate_row_seconds(r, slices)
        out[f"days_{r.name}"] = s / DAY
        out[f"pflops_{r.name}"] = gate_row_pflops(r, slices)
        compute += s
        flops += gate_row_flops(r, slices)
    c = contraction_seconds(contraction_flops)
    out["contraction_days"] = c / DAY
    compute += c
    out["compute_days"] = compute / DAY
    out["compute_pflops"] = flops / compute / 1e15
    a2a = sum(r.alltoalls for r in rows) + disk_transfers
    out["alltoall_count"] = a2a
    out["alltoall_days"] = alltoall_seconds(a2a, n) / DAY
    out["disk_days"] = disk_seconds(disk_transfers, n) / DAY
    out["total_days"] = out["compute_days"] + out["alltoall_days"] + out["disk_days"]
    out["kernels_total"] = sum(r.kernels for r in rows)
    out["gates_total"] = sum(r.gates for r in rows)
    return out


def depth_estimate_days(n: int, kernels: int, alltoalls: float, disk_transfers: int,
                        base: Dict[str, float], small_kernels: int) -> float:
    """Run time for another depth (Tabs. 3 and 4): `base` is the 20-cycle
    table (`table(...)` output) whose tensors 1, 2 and contraction are kept;
    kernels beyond the small tensors' `small_kernels` cost the 45-qubit rate."""
    slices = 2 ** (n - 45)
    fixed = base["contraction_days"] + base["days_1"] + base["days_2"]
    gates = (kernels - small_kernels) * slices * T_GATE_45Q / DAY
    return fixed + gates + alltoall_seconds(alltoalls, n) / DAY + disk_seconds(disk_transfers, n) / DAY
