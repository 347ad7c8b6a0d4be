"""CPU oracle (Python side).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps `liboracle.so` (plain C, complex128, built
from `sv_oracle.c`) and adds the few definitions that are clearer in NumPy.
It imports nothing from the GPU package except the seeded input generator
(`paper_1910_09534_amd.workload`), which holds no simulation arithmetic.

What is computed is the plain definition of the method's result:
psi = U_L ... U_1 |0^n>, the amplitudes psi[x] for requested bitstrings x,
the norm sum |psi|^2, and for a sliced run the reduction
out[x] = sum_s T[x_S, s] psi_s(x_L), which is the same as applying the
trailing operator T to the sliced qubits of the unsliced state and then
reading psi[x] (Sec. 2, tensor slicing: fixing index values re-orders the
sum, it does not change it).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sv_oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_init_zero.argtypes = [P, ctypes.c_int]
        L.orc_apply_dense.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_apply_diag.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_simulate.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P]
        L.orc_apply_gates.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        L.orc_gather.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P]
        L.orc_norm.argtypes = [P, ctypes.c_int]
        L.orc_norm.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the following oracle calls (timing only)."""
    lib().orc_set_threads(int(n))


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_init_zero(_ptr(psi), n)
    return psi


def apply_dense(psi: np.ndarray, qubits: Sequence[int], m: np.ndarray) -> np.ndarray:
    """In place: dense 2^k x 2^k gate on `qubits` (index = sum_j b(q_j) 2^j)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    n = int(psi.size).bit_length() - 1
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    mm = np.ascontiguousarray(m, dtype=np.complex128)
    assert mm.shape == (1 << len(q), 1 << len(q))
    rc = lib().orc_apply_dense(_ptr(psi), n, len(q), _ptr(q), _ptr(mm))
    if rc:
        raise ValueError("oracle apply_dense: bad qubits")
    return psi


def apply_diag(psi: np.ndarray, qubits: Sequence[int], d: np.ndarray) -> np.ndarray:
    """In place: psi[i] *= d[sum_j b_{q_j}(i) 2^j]."""
    n = int(psi.size).bit_length() - 1
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    dd = np.ascontiguousarray(d, dtype=np.complex128)
    assert dd.size == 1 << len(q)
    rc = lib().orc_apply_diag(_ptr(psi), n, len(q), _ptr(q), _ptr(dd))
    if rc:
        raise ValueError("oracle apply_diag: bad qubits")
    return psi


def _flatten(gates):
    arity = np.array([len(g.qubits) for g in gates], dtype=np.int32)
    qubits = np.array([q for g in gates for q in g.qubits], dtype=np.int32)
    mats = np.concatenate([np.ascontiguousarray(g.matrix, dtype=np.complex128).ravel()
                           for g in gates]) if gates else np.zeros(1, np.complex128)
    return arity, qubits, mats


def simulate(circuit, psi: Optional[np.ndarray] = None) -> np.ndarray:
    """psi = U_L ... U_1 |0^n> for circuit.gates in list order."""
    n = circuit.n
    if psi is None:
        psi = np.empty(1 << n, dtype=np.complex128)
    arity, qubits, mats = _flatten(circuit.gates)
    rc = lib().orc_simulate(_ptr(psi), n, len(circuit.gates), _ptr(arity), _ptr(qubits),
                            _ptr(mats))
    if rc:
        raise ValueError(f"oracle simulate failed at gate {-rc - 1}")
    return psi


def apply_gates(psi: np.ndarray, gates) -> np.ndarray:
    """In place: apply `gates` (objects with .qubits, .matrix) in order."""
    n = int(psi.size).bit_length() - 1
    arity, qubits, mats = _flatten(list(gates))
    rc = lib().orc_apply_gates(_ptr(psi), n, 0, len(arity), _ptr(arity), _ptr(qubits),
                               _ptr(mats))
    if rc:
        raise ValueError("oracle apply_gates failed")
    return psi


def gather(psi: np.ndarray, bits: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    out = np.empty(b.size, dtype=np.complex128)
    if lib().orc_gather(_ptr(psi), n, b.size, _ptr(b), _ptr(out)):
        raise ValueError("oracle gather: bitstring out of range")
    return out


def norm(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return float(lib().orc_norm(_ptr(psi), n))


def xeb_sums(n: int, amps: np.ndarray):
    """Sum over the returned x of N p(x) and of ln(N p(x)), p = |a(x)|^2
    (cross-entropy sums; zero probabilities give -inf in the log sum)."""
    p = (amps.real ** 2 + amps.imag ** 2) * float(1 << n)
    with np.errstate(divide="ignore"):
        return float(p.sum()), float(np.log(p).sum())


def reduce_slices_ref(psi_full: np.ndarray, sliced_qubits: Sequence[int],
                      trailing: Optional[np.ndarray], bits: np.ndarray):
    """Reference for the cross-slice reduction: apply the trailing operator T
    (2^s x 2^s over the sliced qubits, row/col bit j <-> sliced_qubits[j];
    None = identity) to the full state, then read the amplitudes and the
    norm and cross-entropy sums of the result."""
    psi = psi_full.copy()
    if trailing is not None:
        apply_dense(psi, sliced_qubits, trailing)
    amps = gather(psi, bits)
    n = int(psi.size).bit_length() - 1
    s1, s2 = xeb_sums(n, amps)
    return amps, (norm(psi), s1, s2)


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    den = float(np.linalg.norm(ref))
    return float(np.linalg.norm(np.asarray(a) - ref)) / (den if den > 0 else 1.0)
