"""GPU checks of the split-fp16 form of the staged passes: the complex64
products on the fp16 matrix cores, each fp32 operand split into a high and
a low fp16 part with fp32 accumulation, the tile scaled by a power of two
taken from the state's amplitude bound.

- unitary blocks take the split form, SV_OPT_SPLIT 0 the fp32 form; both
  equal the complex128 oracle to complex64 accuracy and each other;
- states of any norm (1e-6 .. 3e7) keep that accuracy (the scale follows
  the bound);
- a non-unitary block sends its run to the fp32 form and raises the bound;
- amplitudes the caller wrote (SV_FLAG_KEEP, sv_device_buffer) make the
  bound unknown until the next queue measures the norm on the device;
- a batch run from a reset takes the split form and equals the same plan
  run alone (bitwise); its other variant takes the fp32 form."""
import ctypes
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1910_09534_amd import planner, sv
from paper_1910_09534_amd import workload as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ext_state(psi):
    """Resident complex64 state adopting a device copy of psi (SV_FLAG_KEEP)."""
    torch = _torch()
    n = int(psi.size).bit_length() - 1
    t = torch.from_numpy(psi.astype(np.complex64)).to("cuda")
    torch.cuda.synchronize()
    h = sv.create_state_ext(n, 0, "c64", None, t.data_ptr(), t.numel() * 8, keep=True)
    return h, t


def _read(h, n):
    return sv.gather_amplitudes(h, np.arange(1 << n, dtype=np.uint64))


def _blocks(n, rng, count=10, spread=True):
    """4/5-qubit unitary blocks whose targets fit 13-position tiles."""
    hi = list(range(4, n))
    pool = [int(x) for x in rng.choice(hi, size=min(len(hi), 9), replace=False)] + [0, 1, 2, 3]
    if not spread:
        pool = list(range(min(n, 9)))
    ops = []
    for _ in range(count):
        k = int(rng.choice([4, 5]))
        qs = [int(x) for x in rng.choice(pool, size=k, replace=False)]
        ops.append((qs, W.random_unitary(1 << k, rng)))
    return ops


def _oracle(psi, ops):
    ref = psi.astype(np.complex128).copy()
    for qs, u in ops:
        orc.apply_dense(ref, qs, u)
    return ref


def _run(psi, ops, split, stage=13):
    n = int(psi.size).bit_length() - 1
    h, t = _ext_state(psi)
    try:
        sv.set_option(h, sv.SV_OPT_STAGE, stage)
        sv.set_option(h, sv.SV_OPT_SPLIT, split)
        for qs, u in ops:
            sv.apply_fused(h, qs, u, "c64")
        out = _read(h, n)
        return out, sv.stage_forms(h), sv.counters(h)
    finally:
        sv.destroy_state(h)


@pytest.mark.parametrize("n", [12, 15, 18, 21])
def test_split_and_fp32_forms_match_oracle(n):
    rng = np.random.default_rng(700 + n)
    psi = W.random_state(n, rng)
    ops = _blocks(n, rng)
    ref = _oracle(psi, ops)
    got = {}
    for split in (1, 0):
        out, forms, cnt = _run(psi, ops, split)
        assert cnt["staged_blocks"] >= 2, "no staged pass was formed"
        if split:
            assert forms["split"] >= 1 and forms["fp32"] == 0, forms
            # measured from the norm (1) through unitary blocks
            assert abs(forms["amp_bound"] - 1.0) < 1e-4, forms
        else:
            assert forms["split"] == 0 and forms["fp32"] >= 1, forms
        got[split] = out
        assert orc.rel_l2(out, ref) <= 1e-5, (split, orc.rel_l2(out, ref))
    assert orc.rel_l2(got[1], got[0]) <= 3e-6


@pytest.mark.parametrize("scale", [1e-6, 1e-3, 1e3, 3e7])
def test_split_accuracy_independent_of_norm(scale):
    """The tile scale follows the amplitude bound: the relative error of a
    state of norm `scale` is that of a normalised one."""
    n = 16
    rng = np.random.default_rng(71)
    psi = W.random_state(n, rng) * scale
    ops = _blocks(n, rng)
    out, forms, _ = _run(psi, ops, 1)
    assert forms["split"] >= 1 and forms["fp32"] == 0, forms
    assert forms["amp_bound"] == pytest.approx(scale, rel=1e-4)
    ref = _oracle(psi, ops)
    assert np.all(np.isfinite(out))
    assert orc.rel_l2(out, ref) <= 1e-5, orc.rel_l2(out, ref)


def test_non_unitary_block_takes_fp32_form():
    n = 15
    rng = np.random.default_rng(72)
    psi = W.random_state(n, rng)
    ops = _blocks(n, rng, count=6, spread=False)
    qs, u = ops[2]
    ops[2] = (qs, 2.0 * u)                         # growth 2, not unitary
    out, forms, _ = _run(psi, ops, 1)
    assert forms["fp32"] >= 1, forms
    assert forms["amp_bound"] == pytest.approx(2.0, rel=1e-4)
    ref = _oracle(psi, ops)
    assert orc.rel_l2(out, ref) <= 1e-5


def test_device_buffer_write_then_measured_bound():
    """sv_device_buffer hands out the amplitudes: the bound becomes unknown;
    the next queue with stageable blocks measures the norm (here 5) and
    takes the split form with the matching scale."""
    torch = _torch()
    n = 16
    rng = np.random.default_rng(73)
    psi = W.random_state(n, rng) * 5.0
    ops = _blocks(n, rng)
    st = sv.State(n, 0, "c64")
    try:
        assert sv.stage_forms(st.h)["amp_bound"] == 1.0
        ptr, nbytes = sv.device_buffer(st.h)
        assert nbytes == (1 << n) * 8
        assert math.isinf(sv.stage_forms(st.h)["amp_bound"])
        sv.sync_state(st.h)                          # |0...0> written on the state's stream first
        src = torch.from_numpy(psi.astype(np.complex64)).to("cuda")
        torch.cuda.synchronize()
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        assert hip.hipMemcpy(ptr, src.data_ptr(), nbytes, 3) == 0          # device to device
        sv.set_option(st.h, sv.SV_OPT_STAGE, 13)
        for q, u in ops:
            sv.apply_fused(st.h, q, u, "c64")
        out = _read(st.h, n)
        forms = sv.stage_forms(st.h)
    finally:
        st.close()
    assert forms["split"] >= 1 and forms["fp32"] == 0, forms
    assert forms["amp_bound"] == pytest.approx(5.0, rel=1e-4)
    ref = _oracle(psi, ops)
    assert orc.rel_l2(out, ref) <= 1e-5


@pytest.mark.parametrize("graph", [True, False])
def test_batch_reset_variant_split_form(graph):
    """Circuits run as a batch from a reset take the split form and equal
    the same plans run alone (bitwise) and the oracle; launched again
    without a reset, the batch takes the fp32 form and applies the circuits
    a second time."""
    _torch()
    specs = W.batch_specs(4, seed=31, nmin=17, nmax=21, dmin=8, dmax=10)
    circs = [W.sycamore_circuit(s["n"], s["depth"], s["seed"]) for s in specs]
    plans = [planner.plan_fast(c.gates, 5, nloc=c.n, sparse_start=True) for c in circs]
    states = [sv.State(c.n, 0, "c64") for c in circs]
    b = None
    try:
        for st, c, p in zip(states, circs, plans):
            sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(c.n))
            sv.reset(st.h)
            planner.enqueue(st.h, p, st.dtype)
        b = sv.batch_prepare([st.h for st in states], graph=graph)
        forms = [sv.stage_forms(st.h) for st in states]
        assert sum(f["split"] for f in forms) >= 1 and sum(f["fp32"] for f in forms) == 0, forms
        for st in states:
            sv.reset(st.h)
        sv.batch_launch(b)
        sv.batch_sync(b)
        once = [_read(st.h, c.n) for st, c in zip(states, circs)]
        sv.batch_launch(b)                          # not reset: the fp32 variant, applied again
        sv.batch_sync(b)
        twice = [_read(st.h, c.n) for st, c in zip(states, circs)]
    finally:
        if b is not None:
            sv.batch_destroy(b)
        for st in states:
            st.close()
    for c, p, a1, a2 in zip(circs, plans, once, twice):
        st = sv.State(c.n, 0, "c64")
        try:
            sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(c.n))
            planner.enqueue(st.h, p, st.dtype)
            alone = _read(st.h, c.n)
            f = sv.stage_forms(st.h)
            assert f["fp32"] == 0 and (f["split"] >= 1 or planner.stage_tmax(c.n) == 0), f
        finally:
            st.close()
        assert np.array_equal(alone, a1), "batched result differs from the same plan alone"
        ref = orc.simulate(c)
        assert orc.rel_l2(a1, ref) <= 1e-4
        ref2 = ref.copy()
        for g in c.gates:
            orc.apply_dense(ref2, list(g.qubits), g.matrix)
        assert orc.rel_l2(a2, ref2) <= 1e-4
