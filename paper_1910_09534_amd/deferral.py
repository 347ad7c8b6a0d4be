"""Contraction deferral on the device (Sec. 2; App. A: the EI and E2Q
synthesized gates and the contraction over entanglement indices).

The qubits are split into two parts.  The leading cycles of the circuit run
as two separate tensors, one per part, each a device state with two extra
qubits per gate that bridges the parts (its entanglement indices):

- a gate inside one part is an ordinary gate on that part's state;
- a bridging gate on (a, b), a in part 1: EI on state 1 -- the old position
  of a becomes entanglement index "a", a fresh position becomes qubit a and
  another fresh position (entanglement index a') is tied to it: the fresh
  pair |00> goes to |00> + |11>; E2Q on state 2 -- two fresh positions hold
  the indices a and a', and the gate maps (a, b) to (a', b''): the 8 x 8
  operator on (a, a', b) sends |0, 0, b> to sum_{x, y, b''}
  2Q[y, b''; x, b] |x, y, b''>.

Both are dense operators on fresh positions (not unitary), applied with
`apply_fused` like any other block.  Each state is then permuted so its
open qubits sit at the low positions and the entanglement indices, in the
same order in both, at the top; `sv_contract` sums over them into the joint
state, on which the rest of the circuit runs.  This module holds the
bookkeeping only (positions, operator matrices); every step runs in the
library.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .workload import Gate

# |00> -> |00> + |11> on (new open position, new entanglement position)
EI_MATRIX = np.zeros((4, 4), dtype=np.complex128)
EI_MATRIX[0, 0] = 1.0
EI_MATRIX[3, 0] = 1.0


def e2q_matrix(gate_qubits: Sequence[int], matrix: np.ndarray, a: int, b: int) -> np.ndarray:
    """The E2Q operator on (entanglement index a, entanglement index a',
    qubit b), index bit 0 = a, bit 1 = a', bit 2 = b: column |0, 0, b>
    holds 2Q[a' = y, b''; a = x, b] at row |x, y, b''>; every other column
    is zero (the fresh positions start at |0>)."""
    g = np.asarray(matrix, dtype=np.complex128)
    ia = list(gate_qubits).index(a)
    ib = list(gate_qubits).index(b)

    def gidx(bit_a, bit_b):
        return (bit_a << ia) | (bit_b << ib)

    out = np.zeros((8, 8), dtype=np.complex128)
    for bin_ in range(2):
        for x in range(2):
            for y in range(2):
                for bout in range(2):
                    out[x | (y << 1) | (bout << 2), bin_ << 2] = g[gidx(y, bout), gidx(x, bin_)]
    return out


@dataclasses.dataclass
class DeferredSplit:
    part1: List[int]                 # circuit qubits of tensor 1, ascending
    part2: List[int]
    n_bridging: int                  # D; each tensor has 2 D entanglement indices
    ops1: List[Gate]                 # on state 1 (qubit labels = state-1 positions)
    ops2: List[Gate]
    order1: List[int]                # permutation bringing state 1 to [open part1 | e_0 .. e_2D-1]
    order2: List[int]
    rest: List[Gate]                 # the remaining gates on the joint state (joint labels)
    joint_of: Dict[int, int]         # circuit qubit -> joint position

    @property
    def n1(self) -> int:
        return len(self.part1)

    @property
    def n2(self) -> int:
        return len(self.part2)

    @property
    def e(self) -> int:
        return 2 * self.n_bridging

    def joint_bits(self, bits: np.ndarray) -> np.ndarray:
        """Bitstrings over circuit qubits -> indices of the joint state."""
        b = np.asarray(bits, dtype=np.uint64)
        out = np.zeros_like(b)
        for q, j in self.joint_of.items():
            out |= ((b >> np.uint64(q)) & np.uint64(1)) << np.uint64(j)
        return out


def split(circuit, part1: Sequence[int], ncycles: int) -> DeferredSplit:
    """Defer the gates of the first `ncycles` cycles (a prefix of the gate
    list) into two tensors over part1 and the other qubits."""
    n = circuit.n
    p1 = sorted(set(part1))
    p2 = [q for q in range(n) if q not in set(p1)]
    pre = [g for g in circuit.gates if 0 <= g.cycle < ncycles]
    assert all(x is y for x, y in zip(circuit.gates, pre)), "the deferred cycles must be a prefix of the gate list"
    rest_gates = circuit.gates[len(pre):]
    D = sum(1 for g in pre if len(g.qubits) == 2 and ((g.qubits[0] in p1) != (g.qubits[1] in p1)))
    pos1 = {q: i for i, q in enumerate(p1)}          # circuit qubit -> state-1 position
    pos2 = {q: i for i, q in enumerate(p2)}
    fresh1, fresh2 = len(p1), len(p2)
    ent1: Dict[int, int] = {}                        # entanglement index -> state-1 position
    ent2: Dict[int, int] = {}
    ops1: List[Gate] = []
    ops2: List[Gate] = []
    ne = 0
    s1 = set(p1)
    for g in pre:
        qs = list(g.qubits)
        inside = [q in s1 for q in qs]
        if all(inside):
            ops1.append(Gate(tuple(pos1[q] for q in qs), g.matrix, g.name, g.cycle))
        elif not any(inside):
            ops2.append(Gate(tuple(pos2[q] for q in qs), g.matrix, g.name, g.cycle))
        else:
            assert len(qs) == 2
            a = qs[0] if inside[0] else qs[1]
            b = qs[1] if inside[0] else qs[0]
            # EI: old position of a -> entanglement index ne; fresh -> a; fresh -> ne + 1
            ent1[ne] = pos1[a]
            pos1[a], ent1[ne + 1] = fresh1, fresh1 + 1
            ops1.append(Gate((fresh1, fresh1 + 1), EI_MATRIX, "EI", g.cycle))
            fresh1 += 2
            # E2Q: fresh -> index ne (a), fresh -> index ne + 1 (a'); b keeps its position
            ent2[ne], ent2[ne + 1] = fresh2, fresh2 + 1
            ops2.append(Gate((fresh2, fresh2 + 1, pos2[b]), e2q_matrix(qs, g.matrix, a, b), "E2Q", g.cycle))
            fresh2 += 2
            ne += 2
    assert ne == 2 * D
    order1 = [pos1[q] for q in p1] + [ent1[j] for j in range(ne)]
    order2 = [pos2[q] for q in p2] + [ent2[j] for j in range(ne)]
    joint_of = {q: i for i, q in enumerate(p1)}
    joint_of.update({q: len(p1) + i for i, q in enumerate(p2)})
    rest = [Gate(tuple(joint_of[q] for q in g.qubits), g.matrix, g.name, g.cycle) for g in rest_gates]
    return DeferredSplit(p1, p2, D, ops1, ops2, order1, order2, rest, joint_of)


def grid_halves(n: int) -> List[int]:
    """Part 1 = the left half of the grid's columns."""
    from .workload import grid_shape
    _, cols = grid_shape(n)
    return [q for q in range(n) if q % cols < cols // 2]
