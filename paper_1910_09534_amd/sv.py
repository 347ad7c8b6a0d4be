"""Python binding of libsv (ctypes).  Argument marshalling only: every step of
the path runs in the HIP library.  The names follow the C-ABI (include/sv.h).

The library must have been built (`python -m paper_1910_09534_amd.build`);
there is no fallback: importing this module without libsv.so raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_ESLICED, SV_ESTATE, SV_EIO = 0, -1, -2, -3, -4, -5, -6
SV_C64, SV_C128 = 0, 1
SV_FLAG_TIER, SV_FLAG_KEEP, SV_FLAG_PAGEABLE, SV_FLAG_STORE32 = 0x100, 0x200, 0x400, 0x800
SV_OPT_TIMING, SV_OPT_MFMA, SV_OPT_FOLD_DIAG, SV_OPT_SLOTS, SV_OPT_STAGE, SV_OPT_FAIL_IO = 1, 2, 3, 4, 5, 6
SV_OPT_SPARSE_START = 7
SV_OPT_KEEP_FILES = 8
SV_OPT_SPLIT = 9
SV_OP_FUSED, SV_OP_DIAG = 0, 1

ERROR_NAMES = {SV_EINVAL: "SV_EINVAL", SV_ENOMEM: "SV_ENOMEM", SV_EDEVICE: "SV_EDEVICE",
               SV_ESLICED: "SV_ESLICED", SV_ESTATE: "SV_ESTATE", SV_EIO: "SV_EIO"}

EXPORTS = ("create_state", "create_state_ext", "create_state_files", "destroy_state", "apply_fused", "apply_diag",
           "apply_ops", "permute_qubits", "gather_amplitudes", "reduce_slices", "sync_state", "sv_reset", "last_error",
           "sv_get_order", "sv_device_buffer", "sv_set_option", "sv_counters", "sv_stage_forms", "sv_sweep_time",
           "sv_sweep_profile", "sv_batch_prepare", "sv_batch_launch", "sv_batch_sync", "sv_batch_info",
           "sv_batch_destroy", "sv_batch_error", "sv_contract", "reduce_slices_noalloc", "sv_checkpoint",
           "open_state_files")
SV_BATCH_GRAPH = 1


class SVError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libsv.so (raises if it has not been built)."""
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsv.so not built ({LIB_PATH}); run python -m paper_1910_09534_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, U64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    L.create_state.argtypes = [I, U64, I, P, ctypes.POINTER(P)]
    L.create_state_ext.argtypes = [I, U64, I, P, P, SZ, ctypes.POINTER(P)]
    L.create_state_files.argtypes = [I, U64, I, P, ctypes.c_char_p, ctypes.POINTER(P)]
    L.destroy_state.argtypes = [P]
    L.apply_fused.argtypes = [P, I, P, P]
    L.apply_diag.argtypes = [P, I, P, P]
    L.apply_ops.argtypes = [P, I, P, P, P, P]
    L.permute_qubits.argtypes = [P, P]
    L.gather_amplitudes.argtypes = [P, I64, P, P]
    L.reduce_slices.argtypes = [P, P, I64, P, P, P]
    L.reduce_slices_noalloc.argtypes = [P, P, I64, P, P, P]
    L.sv_checkpoint.argtypes = [P, I64]
    L.open_state_files.argtypes = [ctypes.c_char_p, P, ctypes.POINTER(P), ctypes.POINTER(I64)]
    L.sync_state.argtypes = [P]
    L.sv_reset.argtypes = [P]
    L.last_error.argtypes = [P]
    L.last_error.restype = ctypes.c_char_p
    L.sv_get_order.argtypes = [P, P]
    L.sv_device_buffer.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(SZ)]
    L.sv_set_option.argtypes = [P, I, I64]
    L.sv_counters.argtypes = [P, P]
    L.sv_stage_forms.argtypes = [P, P, ctypes.POINTER(ctypes.c_double)]
    L.sv_sweep_time.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
    L.sv_sweep_profile.argtypes = [P, P, P, P, P, P]
    L.sv_batch_prepare.argtypes = [I, P, I, P, ctypes.POINTER(P)]
    L.sv_batch_launch.argtypes = [P]
    L.sv_batch_sync.argtypes = [P]
    L.sv_batch_info.argtypes = [P, P]
    L.sv_batch_destroy.argtypes = [P]
    L.sv_batch_error.argtypes = [P]
    L.sv_contract.argtypes = [P, P, P, I, I, I, I, P]
    for name in EXPORTS:
        text = name in ("last_error", "sv_batch_error")
        getattr(L, name).restype = ctypes.c_char_p if text else ctypes.c_int
    return L


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, h=None):
    if rc != SV_OK:
        msg = lib().last_error(h)
        raise SVError(rc, msg.decode() if msg else "")


def _dtype_code(dtype) -> int:
    if dtype in ("c64", "complex64", np.complex64, SV_C64):
        return SV_C64
    if dtype in ("c128", "complex128", np.complex128, SV_C128):
        return SV_C128
    raise ValueError(f"dtype {dtype!r}")


def np_dtype(code: int):
    return np.complex64 if code == SV_C64 else np.complex128


def create_state(n: int, slice_mask: int = 0, dtype="c64", stream=None, tier: bool = False,
                 pageable: bool = False, store32: bool = False):
    """Returns an opaque handle (int)."""
    h = ctypes.c_void_p()
    code = _dtype_code(dtype) | (SV_FLAG_TIER if tier else 0) | (SV_FLAG_PAGEABLE if pageable else 0) | \
        (SV_FLAG_STORE32 if store32 else 0)
    _check(lib().create_state(n, slice_mask, code, stream, ctypes.byref(h)))
    return h.value


def create_state_ext(n: int, slice_mask: int, dtype, stream, dev_ptr: int, nbytes: int,
                     keep: bool = False):
    h = ctypes.c_void_p()
    code = _dtype_code(dtype) | (SV_FLAG_KEEP if keep else 0)
    _check(lib().create_state_ext(n, slice_mask, code, stream, dev_ptr, nbytes, ctypes.byref(h)))
    return h.value


def create_state_files(n: int, slice_mask: int, dtype, stream, directory: str, store32: bool = False):
    """Tiered state whose logical files are files in `directory`."""
    h = ctypes.c_void_p()
    code = _dtype_code(dtype) | (SV_FLAG_STORE32 if store32 else 0)
    _check(lib().create_state_files(n, slice_mask, code, stream, directory.encode(), ctypes.byref(h)))
    return h.value


def checkpoint(h, tag: int) -> None:
    """Make a state whose tier is in files a restart point (sv_checkpoint)."""
    _check(lib().sv_checkpoint(h, int(tag)), h)


def open_state_files(directory: str, stream=None):
    """(handle, tag) of the last checkpoint in `directory`."""
    h = ctypes.c_void_p()
    tag = ctypes.c_int64()
    _check(lib().open_state_files(directory.encode(), stream, ctypes.byref(h), ctypes.byref(tag)))
    return h.value, tag.value


def destroy_state(h) -> None:
    _check(lib().destroy_state(h))


def apply_fused(h, qubits: Sequence[int], matrix: np.ndarray, dtype) -> int:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(matrix, dtype=np_dtype(_dtype_code(dtype)))
    rc = lib().apply_fused(h, len(q), _ptr(q), _ptr(m))
    _check(rc, h)
    return rc


def apply_diag(h, qubits: Sequence[int], phases: np.ndarray, dtype) -> int:
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    d = np.ascontiguousarray(phases, dtype=np_dtype(_dtype_code(dtype)))
    rc = lib().apply_diag(h, len(q), _ptr(q), _ptr(d))
    _check(rc, h)
    return rc


class PackedOps:
    """An operation list laid out for apply_ops: kinds, widths, concatenated
    qubit lists and concatenated matrices / phase tables in one dtype."""

    def __init__(self, ops, dtype):
        code = _dtype_code(dtype)
        dt = np_dtype(code)
        kinds, widths, qubits, data = [], [], [], []
        for kind, qs, m in ops:
            kinds.append(SV_OP_FUSED if kind == "dense" else SV_OP_DIAG)
            widths.append(len(qs))
            qubits.extend(int(q) for q in qs)
            data.append(np.ascontiguousarray(m, dtype=dt).ravel())
        self.count = len(kinds)
        self.kinds = np.array(kinds, dtype=np.int32)
        self.widths = np.array(widths, dtype=np.int32)
        self.qubits = np.array(qubits, dtype=np.int32)
        self.data = np.concatenate(data) if data else np.zeros(1, dtype=dt)


def apply_ops(h, packed: PackedOps) -> None:
    """Queue a whole PackedOps list with one library call."""
    _check(lib().apply_ops(h, packed.count, _ptr(packed.kinds), _ptr(packed.widths), _ptr(packed.qubits),
                           _ptr(packed.data)), h)


def permute_qubits(h, order: Sequence[int]) -> None:
    o = np.ascontiguousarray(order, dtype=np.int32)
    _check(lib().permute_qubits(h, _ptr(o)), h)


def gather_amplitudes(h, bitstrings: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    out = np.empty(b.size, dtype=np.complex128)
    _check(lib().gather_amplitudes(h, b.size, _ptr(b), _ptr(out)), h)
    return out


def reduce_slices(h, bitstrings: np.ndarray, trailing: Optional[np.ndarray] = None):
    """Returns (amplitudes complex128, stats (norm, sum N p, sum ln N p))."""
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    out = np.empty(b.size, dtype=np.complex128)
    stats = np.zeros(3, dtype=np.float64)
    t = None if trailing is None else np.ascontiguousarray(trailing, dtype=np.complex128)
    _check(lib().reduce_slices(h, None if t is None else _ptr(t), b.size, _ptr(b), _ptr(out),
                               _ptr(stats)), h)
    return out, tuple(float(x) for x in stats)


NOALLOC_MAX_BITSTRINGS, NOALLOC_MAX_SLICED, NOALLOC_MAX_QUEUED_BYTES = 1 << 20, 6, 8 << 20


def reduce_slices_noalloc(h, bitstrings: np.ndarray, trailing: Optional[np.ndarray] = None):
    """As reduce_slices, through the entry point that allocates no device
    memory (its work buffers are a fixed array of the library)."""
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    out = np.empty(b.size, dtype=np.complex128)
    stats = np.zeros(3, dtype=np.float64)
    t = None if trailing is None else np.ascontiguousarray(trailing, dtype=np.complex128)
    _check(lib().reduce_slices_noalloc(h, None if t is None else _ptr(t), b.size, _ptr(b), _ptr(out),
                                       _ptr(stats)), h)
    return out, tuple(float(x) for x in stats)


def sync_state(h) -> None:
    _check(lib().sync_state(h), h)


def reset(h) -> None:
    _check(lib().sv_reset(h), h)


def last_error(h=None) -> str:
    m = lib().last_error(h)
    return m.decode() if m else ""


def get_order(h, n: int) -> list:
    o = np.zeros(n, dtype=np.int32)
    _check(lib().sv_get_order(h, _ptr(o)))
    return o.tolist()


def device_buffer(h):
    p = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    _check(lib().sv_device_buffer(h, ctypes.byref(p), ctypes.byref(sz)))
    return p.value, sz.value


def set_option(h, option: int, value: int) -> None:
    _check(lib().sv_set_option(h, option, value), h)


def stage_forms(h) -> dict:
    """Staged passes run in the split-fp16 and fp32 forms since creation,
    and the state's amplitude bound (sv_stage_forms)."""
    c = np.zeros(2, dtype=np.int64)
    b = ctypes.c_double()
    _check(lib().sv_stage_forms(h, _ptr(c), ctypes.byref(b)))
    return {"split": int(c[0]), "fp32": int(c[1]), "amp_bound": b.value}


def counters(h) -> dict:
    c = np.zeros(8, dtype=np.int64)
    _check(lib().sv_counters(h, _ptr(c)))
    keys = ("dense_sweeps", "diag_sweeps", "perm_sweeps", "amps_swept", "bytes_h2d", "bytes_d2h",
            "zero_slices_skipped", "staged_blocks")
    return dict(zip(keys, (int(x) for x in c)))


def sweep_time(h):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().sv_sweep_time(h, ctypes.byref(ms), ctypes.byref(cnt)), h)
    return ms.value, cnt.value


def sweep_profile(h) -> dict:
    """Timed launches by kind ("sweep": single dense sweeps, "staged":
    staged passes): ms, count, algorithmic flops, issued flops, HBM bytes
    moved.  Resets the timing accumulators."""
    ms = np.zeros(2, dtype=np.float64)
    cnt = np.zeros(2, dtype=np.int64)
    fl = np.zeros(2, dtype=np.float64)
    iss = np.zeros(2, dtype=np.float64)
    by = np.zeros(2, dtype=np.float64)
    _check(lib().sv_sweep_profile(h, _ptr(ms), _ptr(cnt), _ptr(fl), _ptr(iss), _ptr(by)), h)
    return {kind: {"ms": float(ms[i]), "count": int(cnt[i]), "flops": float(fl[i]), "issued": float(iss[i]),
                   "bytes": float(by[i])}
            for i, kind in enumerate(("sweep", "staged"))}


SV_CONTRACT_FP32 = 0x1000


def contract(t1_ptr: int, t2_ptr: int, out_ptr: int, n1: int, n2: int, e: int, dtype, stream=None,
             fp32: bool = False) -> None:
    """out[x2 2^n1 + x1] = sum_c t1[c 2^n1 + x1] t2[c 2^n2 + x2] on device
    buffers (see sv_contract in include/sv.h).  Asynchronous on `stream`.
    fp32: complex64 products in the 3M form on the fp32 matrix cores instead
    of the split-fp16 form."""
    code = _dtype_code(dtype) | (SV_CONTRACT_FP32 if fp32 else 0)
    _check(lib().sv_contract(t1_ptr, t2_ptr, out_ptr, n1, n2, e, code, stream))


def _bcheck(rc: int, b=None):
    if rc != SV_OK:
        msg = lib().sv_batch_error(b)
        raise SVError(rc, msg.decode() if msg else "")


def batch_prepare(handles, graph: bool = True, stream=None):
    """Record the queued operations of `handles` as one batch (handle list of
    resident states, same dtype).  Returns an opaque batch pointer."""
    arr = (ctypes.c_void_p * len(handles))(*handles)
    b = ctypes.c_void_p()
    _bcheck(lib().sv_batch_prepare(len(handles), arr, SV_BATCH_GRAPH if graph else 0, stream,
                                   ctypes.byref(b)))
    return b.value


def batch_launch(b) -> None:
    _bcheck(lib().sv_batch_launch(b), b)


def batch_sync(b) -> None:
    _bcheck(lib().sv_batch_sync(b), b)


def batch_info(b) -> dict:
    i = np.zeros(4, dtype=np.int64)
    _bcheck(lib().sv_batch_info(b, _ptr(i)), b)
    return {"launches": int(i[0]), "sweeps": int(i[1]), "amps_swept": int(i[2]), "graph": bool(i[3])}


def batch_destroy(b) -> None:
    lib().sv_batch_destroy(b)


class State:
    """Owning wrapper around a handle (context manager)."""

    def __init__(self, n: int, slice_mask: int = 0, dtype="c64", stream=None, tier: bool = False,
                 pageable: bool = False, tier_dir: Optional[str] = None, store32: bool = False):
        self.n, self.slice_mask, self.dtype = n, slice_mask, _dtype_code(dtype)
        if tier_dir is not None:
            self.h = create_state_files(n, slice_mask, dtype, stream, tier_dir, store32)
        else:
            self.h = create_state(n, slice_mask, dtype, stream, tier, pageable, store32)

    @classmethod
    def open(cls, directory: str, n: int, slice_mask: int, dtype="c64", stream=None) -> "State":
        """The state of the last checkpoint in `directory` (open_state_files)
        of an n-qubit state with this slice mask and dtype; the checkpoint's
        tag is in .tag."""
        h, tag = open_state_files(directory, stream)
        st = cls.__new__(cls)
        st.h, st.tag = h, tag
        st.n, st.slice_mask, st.dtype = n, slice_mask, _dtype_code(dtype)
        return st

    def fused(self, qubits, matrix):
        apply_fused(self.h, qubits, matrix, self.dtype)

    def diag(self, qubits, phases):
        apply_diag(self.h, qubits, phases, self.dtype)

    def permute(self, order):
        permute_qubits(self.h, order)

    def gather(self, bits):
        return gather_amplitudes(self.h, bits)

    def reduce(self, bits, trailing=None):
        return reduce_slices(self.h, bits, trailing)

    def sync(self):
        sync_state(self.h)

    def order(self):
        return get_order(self.h, self.n)

    def close(self):
        if self.h:
            destroy_state(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
