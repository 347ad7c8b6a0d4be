"""Seeded synthetic workloads: Sycamore-style ABCDCDAB random circuits.

This module is the one place that draws random inputs.  Both the product
path and the CPU oracle consume what it produces; it contains none of the
simulation arithmetic (no state vectors, no gate application, no fusion).
It only *defines* circuits: which gate acts on which qubits, with its
explicit unitary matrix, plus the bitstrings whose amplitudes are asked for.

Circuit class (paper, Sec. 3 "Sycamore circuits"): cycles made of a layer of
single-qubit gates drawn from {sqrt(X), sqrt(Y), sqrt(W)} followed by a layer
of two-qubit gates, then a final single-qubit layer.  The two-qubit unitary
is Eq. (1) (the fSim family) with nominal theta = 90 deg and phi = 30 deg.
Two-qubit layers follow the ABCDCDAB pattern (Sec. 3): four disjoint
couplings A, B, C, D applied in the order A B C D C D A B, repeating.

Readings where the paper is silent (its Sycamore layout figures are not
available):
  * grid: rows = floor(sqrt(n)), cols = ceil(n / rows), qubit (r, c) =
    r * cols + c, sites with index >= n absent;
  * A = horizontal (r,c)-(r,c+1) with r+c even, B = horizontal with r+c odd,
    C = vertical (r,c)-(r+1,c) with r+c even, D = vertical with r+c odd;
  * detunings of Eq. (1) are zero, and at theta = pi/2 the cosine and sine
    are taken exactly as 0 and 1;
  * single-qubit draws: cycle 0 uniform over the three gates, later layers
    (including the final one) uniform over the two gates that differ from
    the previous gate on that qubit; RNG = NumPy PCG64 default_rng(seed);
  * matrix index convention for a gate on qubits (q0, q1, ...): row/column
    index = b(q0) + 2 b(q1) + 4 b(q2) + ... ; amplitude index little-endian
    (bit q of the index is qubit q).
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

PATTERN = "ABCDCDAB"

_S = 1.0 / math.sqrt(2.0)
# sqrt(X) = RX(pi/2), sqrt(Y) = RY(pi/2), sqrt(W) = RW(pi/2), W = (X+Y)/sqrt(2)
SQRT_X = np.array([[_S, -1j * _S], [-1j * _S, _S]], dtype=np.complex128)
SQRT_Y = np.array([[_S, -_S], [_S, _S]], dtype=np.complex128)
SQRT_W = np.array(
    [[_S, -_S * np.exp(0.25j * math.pi)], [_S * np.exp(-0.25j * math.pi), _S]],
    dtype=np.complex128,
)
ONE_QUBIT_GATES = {"sqrt_x": SQRT_X, "sqrt_y": SQRT_Y, "sqrt_w": SQRT_W}
ONE_QUBIT_NAMES = ("sqrt_x", "sqrt_y", "sqrt_w")


def fsim(theta: float = math.pi / 2, phi: float = math.pi / 6) -> np.ndarray:
    """Eq. (1) with all detunings set to zero (basis |00>,|01>,|10>,|11>,
    index = b(q0) + 2 b(q1)).  cos/sin are exact at theta = pi/2."""
    if theta == math.pi / 2:
        c, s = 0.0, 1.0
    else:
        c, s = math.cos(theta), math.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = c
    m[1, 2] = -1j * s
    m[2, 1] = -1j * s
    m[2, 2] = c
    m[3, 3] = np.exp(-1j * phi)
    return m


@dataclasses.dataclass
class Gate:
    qubits: Tuple[int, ...]
    matrix: np.ndarray          # (2^k, 2^k) complex128, index = sum_j b(qubits[j]) 2^j
    name: str = "u"
    cycle: int = -1

    @property
    def k(self) -> int:
        return len(self.qubits)


@dataclasses.dataclass
class Circuit:
    n: int
    gates: List[Gate]
    depth: int = 0
    seed: int = 0
    final_layer: bool = True
    rows: int = 0
    cols: int = 0

    def counts(self) -> Dict[str, int]:
        one = sum(1 for g in self.gates if g.k == 1)
        two = sum(1 for g in self.gates if g.k == 2)
        return {"1q": one, "2q": two, "total": len(self.gates)}

    # ---- circuit file (JSON) ------------------------------------------------
    def to_json(self) -> str:
        return json.dumps({
            "n": self.n, "depth": self.depth, "seed": self.seed,
            "final_layer": self.final_layer, "rows": self.rows, "cols": self.cols,
            "gates": [{"q": list(g.qubits), "name": g.name, "cycle": g.cycle,
                       "re": g.matrix.real.ravel().tolist(),
                       "im": g.matrix.imag.ravel().tolist()} for g in self.gates],
        })

    @staticmethod
    def from_json(text: str) -> "Circuit":
        d = json.loads(text)
        gates = []
        for g in d["gates"]:
            dim = 1 << len(g["q"])
            m = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(dim, dim)
            gates.append(Gate(tuple(g["q"]), m.astype(np.complex128), g["name"], g["cycle"]))
        return Circuit(d["n"], gates, d["depth"], d["seed"], d["final_layer"],
                       d["rows"], d["cols"])


def grid_shape(n: int) -> Tuple[int, int]:
    rows = max(1, int(math.isqrt(n)))
    cols = -(-n // rows)
    return rows, cols


def couplings(n: int) -> Dict[str, List[Tuple[int, int]]]:
    """The four disjoint couplings A-D of the grid holding n qubits."""
    rows, cols = grid_shape(n)
    out: Dict[str, List[Tuple[int, int]]] = {"A": [], "B": [], "C": [], "D": []}
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            if q >= n:
                continue
            even = (r + c) % 2 == 0
            if c + 1 < cols and q + 1 < n:
                out["A" if even else "B"].append((q, q + 1))
            if r + 1 < rows and q + cols < n:
                out["C" if even else "D"].append((q, q + cols))
    return out


def sycamore_circuit(n: int, depth: int, seed: int, final_layer: bool = True,
                     theta: float = math.pi / 2, phi: float = math.pi / 6) -> Circuit:
    """ABCDCDAB random circuit of `depth` cycles on the near-square grid."""
    rng = np.random.default_rng(seed)
    rows, cols = grid_shape(n)
    cpl = couplings(n)
    two = fsim(theta, phi)
    prev = [-1] * n
    gates: List[Gate] = []

    def one_layer(cycle: int) -> None:
        for q in range(n):
            if prev[q] < 0:
                g = int(rng.integers(0, 3))
            else:
                choices = [i for i in range(3) if i != prev[q]]
                g = choices[int(rng.integers(0, 2))]
            prev[q] = g
            name = ONE_QUBIT_NAMES[g]
            gates.append(Gate((q,), ONE_QUBIT_GATES[name].copy(), name, cycle))

    for cyc in range(depth):
        one_layer(cyc)
        for (a, b) in cpl[PATTERN[cyc % len(PATTERN)]]:
            gates.append(Gate((a, b), two.copy(), "fsim", cyc))
    if final_layer:
        one_layer(depth)
    return Circuit(n, gates, depth, seed, final_layer, rows, cols)


def bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    """Uniform bitstrings in [0, 2^n) with replacement (bit q = qubit q)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << n, size=count, dtype=np.uint64)


# ---- generic random inputs (tests) -------------------------------------------

def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary (QR of a complex Ginibre matrix, phases fixed)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return (q * (d / np.abs(d))).astype(np.complex128)


def random_phases(count: int, rng: np.random.Generator) -> np.ndarray:
    return np.exp(1j * rng.uniform(0, 2 * math.pi, size=count)).astype(np.complex128)


def random_state(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


def random_generic_circuit(n: int, ngates: int, seed: int, max_arity: int = 2) -> Circuit:
    """Random circuit of Haar-random gates on random distinct qubit tuples
    (asymmetric gates: pins qubit-order conventions)."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(ngates):
        k = int(rng.integers(1, min(max_arity, n) + 1))
        qs = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        gates.append(Gate(qs, random_unitary(1 << k, rng), "haar"))
    return Circuit(n, gates, 0, seed, False)


# ---- named configurations ----------------------------------------------------

CONFIGS = {
    1: dict(n=16, depth=8, dtype="c128", kmax=4, nbits=1 << 16, all_amplitudes=True),
    2: dict(n=30, depth=14, dtype="c64", kmax=5, nbits=1 << 16),
    3: dict(n=36, depth=20, dtype="c64", kmax=5, nbits=1 << 20,
            slice_sets=((0, 5, 30, 35), (14, 15, 20, 21))),
}


def config_circuit(idx: int) -> Circuit:
    c = CONFIGS[idx]
    return sycamore_circuit(c["n"], c["depth"], seed=1000 + idx)


def config_bitstrings(idx: int) -> np.ndarray:
    c = CONFIGS[idx]
    if c.get("all_amplitudes"):
        return np.arange(1 << c["n"], dtype=np.uint64)
    return bitstrings(c["n"], c["nbits"], seed=2000 + idx)


def batch_specs(count: int = 256, seed: int = 1004, nmin: int = 20, nmax: int = 28,
                dmin: int = 10, dmax: int = 20) -> List[Dict[str, int]]:
    """Independent circuits of a batch: n ~ U{nmin..nmax}, d ~ U{dmin..dmax};
    circuit j uses seed 10000 + j, its bitstrings seed 20000 + j."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    ds = rng.integers(dmin, dmax + 1, size=count)
    return [dict(j=j, n=int(ns[j]), depth=int(ds[j]), seed=10000 + j, bit_seed=20000 + j)
            for j in range(count)]


def serving_trace(count: int = 1000, rate: float = 50.0, seed: int = 1005,
                  nmin: int = 16, nmax: int = 32, dmin: int = 8, dmax: int = 20
                  ) -> List[Dict[str, float]]:
    """Poisson arrivals (exponential gaps at `rate` per second); request j has
    n ~ U{nmin..nmax}, depth ~ U{dmin..dmax}, circuit seed 10000 + j."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(nmin, nmax + 1, size=count)
    ds = rng.integers(dmin, dmax + 1, size=count)
    return [dict(j=j, t=float(t[j]), n=int(ns[j]), depth=int(ds[j]), seed=10000 + j,
                 bit_seed=20000 + j) for j in range(count)]
