"""Brute-force full-unitary reference for tiny circuits.  TEST INFRASTRUCTURE ONLY.

Builds every gate as an explicit 2^n x 2^n matrix from Kronecker products of
2 x 2 elementary matrices, multiplies the whole circuit out, and applies it to
e_0.  This construction shares no index arithmetic with `sv_oracle.c`
(no bit insertion, no strides): it is a direct writing-out of
M = sum_{a,b} M[a,b] |a><b| on the gate's qubits tensored with identities
elsewhere, with qubit 0 the right-most Kronecker factor (little-endian
amplitude index).  Intended for n <= 10.
"""
from __future__ import annotations

from functools import reduce
from typing import Sequence

import numpy as np

_E = [[np.array([[1, 0], [0, 0]], dtype=np.complex128), np.array([[0, 1], [0, 0]], dtype=np.complex128)],
      [np.array([[0, 0], [1, 0]], dtype=np.complex128), np.array([[0, 0], [0, 1]], dtype=np.complex128)]]
_I = np.eye(2, dtype=np.complex128)


def embed(n: int, qubits: Sequence[int], m: np.ndarray) -> np.ndarray:
    """Full 2^n x 2^n operator of gate m on `qubits` (m index = sum_j b(q_j) 2^j)."""
    k = len(qubits)
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for a in range(1 << k):
        for b in range(1 << k):
            if m[a, b] == 0:
                continue
            factors = []
            for q in range(n - 1, -1, -1):           # left-most factor = qubit n-1
                if q in qubits:
                    j = list(qubits).index(q)
                    factors.append(_E[(a >> j) & 1][(b >> j) & 1])
                else:
                    factors.append(_I)
            full += m[a, b] * reduce(np.kron, factors)
    return full


def circuit_unitary(n: int, gates) -> np.ndarray:
    u = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        u = embed(n, g.qubits, g.matrix) @ u
    return u


def brute_state(n: int, gates) -> np.ndarray:
    return circuit_unitary(n, gates)[:, 0].copy()


def permute_state(psi: np.ndarray, n: int, order: Sequence[int]) -> np.ndarray:
    """Physical layout after placing logical qubit order[p] at bit position p:
    out[sum_p b_{order[p]}(x) 2^p] = psi[x].  Written with numpy.transpose on
    the 2 x ... x 2 tensor (axis a of the reshaped array is qubit n-1-a)."""
    t = psi.reshape([2] * n)
    # new axis a holds position n-1-a, i.e. logical qubit order[n-1-a],
    # which sits on old axis n-1-order[n-1-a]
    axes = [n - 1 - order[n - 1 - a] for a in range(n)]
    return np.ascontiguousarray(np.transpose(t, axes)).reshape(-1)
