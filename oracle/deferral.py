"""CPU oracle for contraction deferral (TEST INFRASTRUCTURE ONLY: only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it).

A tensor is a complex128 NumPy array with one axis of length 2 per index,
together with a list of index labels, one per axis.  Labels are
("q", qubit) for the open index of a qubit and ("e", j) for entanglement
index j.  Every step is the plain definition from the paper, written with
einsum over named axes:

- a gate on open qubits applies its matrix to those axes (the gate matrix
  index is sum_j b(q_j) 2^j over the gate's qubit list);
- EI (App. A): for a two-qubit gate bridging qubit a of tensor 1 and qubit
  b of tensor 2, tensor 1 becomes phi'[a'', a', a] = I[a'', a'] phi[a]: the
  old index of a turns into entanglement index "a", a new open index a''
  is added for qubit a, and a new entanglement index a' equal to it;
- E2Q (App. A): tensor 2 becomes chi'[b'', a', a] = sum_b 2Q[a', b''; a, b]
  chi[b];
- the contraction (App. A; Sec. 2: contraction deferral sums shared
  indices and takes the outer product over the others) sums every label
  the two tensors share.

Then sum_{a', a} phi' chi' = sum_{a, b} 2Q[a'', b''; a, b] phi[a] chi[b]:
the gate applied to the product of the two tensors (the first equation of
App. A).  The functions below do not rely on that identity; the tests
check it.
"""
from __future__ import annotations

import string
from typing import Dict, List, Sequence, Tuple

import numpy as np

Label = Tuple[str, int]


def zero_tensor(qubits: Sequence[int]) -> Tuple[np.ndarray, List[Label]]:
    """|0...0> over the open indices of `qubits`."""
    t = np.zeros((2,) * len(qubits), dtype=np.complex128)
    t[(0,) * len(qubits)] = 1.0
    return t, [("q", q) for q in qubits]


def from_state(psi: np.ndarray, qubits: Sequence[int]) -> Tuple[np.ndarray, List[Label]]:
    """Tensor of a state vector over `qubits` (bit j of the index = qubits[j])."""
    k = len(qubits)
    t = np.asarray(psi, dtype=np.complex128).reshape((2,) * k)
    # reshape puts the highest index bit first: axis i holds bit k-1-i
    return t, [("q", qubits[k - 1 - i]) for i in range(k)]


def _letters(n: int) -> str:
    return (string.ascii_letters)[:n]


def gate_tensor(matrix: np.ndarray, k: int) -> np.ndarray:
    """The k-qubit gate as a 2k-axis tensor G[o_0..o_{k-1}, i_0..i_{k-1}],
    o_j / i_j the output / input bit of the gate's j-th qubit."""
    m = np.asarray(matrix, dtype=np.complex128).reshape((2,) * (2 * k))
    # axes of the reshape: output bits k-1..0, then input bits k-1..0
    perm = [k - 1 - j for j in range(k)] + [2 * k - 1 - j for j in range(k)]
    return m.transpose(perm)


def apply_gate(t: np.ndarray, labels: List[Label], qubits: Sequence[int], matrix: np.ndarray):
    """A gate on open qubits of the tensor."""
    k = len(qubits)
    n = t.ndim
    L = _letters(n + k)
    src = L[:n]
    ax = [labels.index(("q", q)) for q in qubits]
    outs = L[n:n + k]
    g = "".join(outs) + "".join(src[a] for a in ax)
    dst = list(src)
    for j, a in enumerate(ax):
        dst[a] = outs[j]
    out = np.einsum(f"{g},{src}->{''.join(dst)}", gate_tensor(matrix, k), t)
    return out, list(labels)


def ei(t: np.ndarray, labels: List[Label], a: int, e_a: int, e_ap: int):
    """EI on the tensor holding qubit a: phi'[a'', a', a] = I[a'', a'] phi[a].
    The old index of a becomes entanglement index e_a; a new open index for
    a (a'') and entanglement index e_ap (a') are appended."""
    new_labels = [("e", e_a) if lb == ("q", a) else lb for lb in labels]
    out = np.einsum("...,ij->...ij", t, np.eye(2, dtype=np.complex128))
    return out, new_labels + [("q", a), ("e", e_ap)]


def e2q(t: np.ndarray, labels: List[Label], gate_qubits: Sequence[int], matrix: np.ndarray,
        a: int, b: int, e_a: int, e_ap: int):
    """E2Q on the tensor holding qubit b, for the two-qubit gate on
    (gate_qubits) that bridges qubit a (other tensor) and b:
    chi'[b'', a', a] = sum_b 2Q[a', b''; a, b] chi[b]."""
    g = gate_tensor(matrix, 2)                       # G[o0, o1, i0, i1] over gate_qubits order
    ia, ib = list(gate_qubits).index(a), list(gate_qubits).index(b)
    # G4[a', b'', a, b]
    g4 = g.transpose([ia, ib, 2 + ia, 2 + ib])
    n = t.ndim
    L = _letters(n + 3)
    src = L[:n]
    xb = labels.index(("q", b))
    ap, bpp, aa = L[n], L[n + 1], L[n + 2]
    dst = list(src)
    dst[xb] = bpp
    out = np.einsum(f"{ap}{bpp}{aa}{src[xb]},{src}->{''.join(dst)}{ap}{aa}", g4, t)
    return out, list(labels) + [("e", e_ap), ("e", e_a)]


def contract(t1: np.ndarray, l1: List[Label], t2: np.ndarray, l2: List[Label]):
    """Sum over every label the two tensors share; outer product over the
    rest (labels of t1 first, then those of t2)."""
    names: Dict[Label, str] = {}
    letters = iter(string.ascii_letters)
    for lb in list(l1) + list(l2):
        if lb not in names:
            names[lb] = next(letters)
    shared = set(l1) & set(l2)
    out_labels = [lb for lb in l1 if lb not in shared] + [lb for lb in l2 if lb not in shared]
    spec = "".join(names[lb] for lb in l1) + "," + "".join(names[lb] for lb in l2) + "->" + \
        "".join(names[lb] for lb in out_labels)
    return np.einsum(spec, t1, t2), out_labels


def to_state(t: np.ndarray, labels: List[Label], qubits: Sequence[int]) -> np.ndarray:
    """State vector over `qubits` (bit j of the index = qubits[j]) of a tensor
    with only open indices."""
    assert sorted(labels) == sorted(("q", q) for q in qubits), "tensor still has entanglement indices"
    k = len(qubits)
    order = [labels.index(("q", qubits[k - 1 - i])) for i in range(k)]
    return np.ascontiguousarray(t.transpose(order)).reshape(-1)


def contract_matrix(t1: np.ndarray, t2: np.ndarray, n1: int, n2: int, e: int) -> np.ndarray:
    """The contraction in the memory layout of the GPU call: t1[e * 2^n1 + x1],
    t2[e * 2^n2 + x2] -> out[x2 * 2^n1 + x1] = sum_e t1[e, x1] t2[e, x2]."""
    a = np.asarray(t1, dtype=np.complex128).reshape(1 << e, 1 << n1)
    b = np.asarray(t2, dtype=np.complex128).reshape(1 << e, 1 << n2)
    return (b.T @ a).reshape(-1)


def deferred_simulate(circuit, part1: Sequence[int]) -> np.ndarray:
    """The whole circuit as two tensors (qubits in part1, the rest): gates
    inside one part apply to that tensor; every gate bridging the parts
    becomes EI on the tensor holding its first bridged qubit and E2Q on the
    other; at the end the two tensors are contracted.  Returns the state
    vector over qubits 0..n-1."""
    n = circuit.n
    p1 = set(part1)
    q1 = [q for q in range(n) if q in p1]
    q2 = [q for q in range(n) if q not in p1]
    t1, l1 = zero_tensor(q1)
    t2, l2 = zero_tensor(q2)
    ne = 0
    for g in circuit.gates:
        qs = list(g.qubits)
        in1 = [q in p1 for q in qs]
        if all(in1):
            t1, l1 = apply_gate(t1, l1, qs, g.matrix)
        elif not any(in1):
            t2, l2 = apply_gate(t2, l2, qs, g.matrix)
        else:
            assert len(qs) == 2, "only two-qubit gates bridge the parts"
            a = qs[0] if in1[0] else qs[1]
            b = qs[1] if in1[0] else qs[0]
            t1, l1 = ei(t1, l1, a, ne, ne + 1)
            t2, l2 = e2q(t2, l2, qs, g.matrix, a, b, ne, ne + 1)
            ne += 2
    t, lab = contract(t1, l1, t2, l2)
    return to_state(t, lab, list(range(n)))
