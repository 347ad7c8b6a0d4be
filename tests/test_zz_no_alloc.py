"""reduce_slices_noalloc (the reduction that allocates no device memory)
against reduce_slices, through the C-ABI: two calls in a row on the shared
work array, the second with a smaller input (fewer bitstrings, fewer
qubits, a trailing operator on sliced qubits), each bitwise equal to the
allocating entry point on an identical state and within the complex64
tolerance of the oracle; limits rejected with SV_EINVAL."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1910_09534_amd import planner, runner, sv
from paper_1910_09534_amd import workload as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run_both(circ, bits, sched=None):
    """The same operations on two resident states; one reduced through each
    entry point.  Returns ((amps, stats) allocating, (amps, stats) no-alloc)."""
    outs = []
    for noalloc in (False, True):
        if sched is None:
            ops = planner.plan(circ.gates, 5, sparse_start=True)
            st = sv.State(circ.n, 0, "c64")
            try:
                sv.reset(st.h)
                planner.enqueue(st.h, ops, st.dtype)
                outs.append(sv.reduce_slices_noalloc(st.h, bits) if noalloc else sv.reduce_slices(st.h, bits))
            finally:
                st.close()
        else:
            mask = sum(1 << q for q in sched.phases[0].sliced)
            st = sv.State(circ.n, mask, "c64")
            try:
                for ph in sched.phases:
                    sv.permute_qubits(st.h, ph.order)
                    planner.enqueue(st.h, ph.ops, st.dtype)
                f = sv.reduce_slices_noalloc if noalloc else sv.reduce_slices
                outs.append(f(st.h, bits, sched.trailing))
            finally:
                st.close()
    return outs


def test_noalloc_equals_reduce_slices_twice():
    _gpu()
    # first call: 20 qubits, unsliced, 2^16 bitstrings, the norm folded into the last pass
    c1 = W.sycamore_circuit(20, 12, seed=501)
    b1 = W.bitstrings(20, 1 << 16, seed=502)
    (a_ref, s_ref), (a_na, s_na) = _run_both(c1, b1)
    assert np.array_equal(a_ref, a_na) and s_ref == s_na
    psi = orc.simulate(c1)
    assert orc.rel_l2(a_na, orc.gather(psi, b1)) <= 1e-4
    assert abs(s_na[0] - 1.0) <= 1e-4
    # second call, smaller: 16 qubits, 4 sliced (16 resident slices), a
    # trailing operator on them, 1000 bitstrings; the array still holds the
    # first call's accumulators
    c2 = W.sycamore_circuit(16, 10, seed=503)
    b2 = W.bitstrings(16, 1000, seed=504)
    A, B = runner.grid_slice_sets(16)
    sched = planner.phase_schedule(c2, A, B, 5)
    (a_ref, s_ref), (a_na, s_na) = _run_both(c2, b2, sched)
    assert np.array_equal(a_ref, a_na) and s_ref == s_na
    ref, (nrm, x1, x2) = orc.reduce_slices_ref(orc.simulate(c2), (), None, b2)
    assert orc.rel_l2(a_na, ref) <= 1e-4
    assert abs(s_na[0] - nrm) <= 1e-4


def test_noalloc_limits():
    _gpu()
    st = sv.State(12, 0, "c64")
    try:
        st.fused([0, 1], W.random_unitary(4, np.random.default_rng(1)))
        too_many = np.zeros(sv.NOALLOC_MAX_BITSTRINGS + 1, dtype=np.uint64)
        with pytest.raises(sv.SVError) as e:
            sv.reduce_slices_noalloc(st.h, too_many)
        assert e.value.code == sv.SV_EINVAL
        sv.set_option(st.h, sv.SV_OPT_TIMING, 1)
        with pytest.raises(sv.SVError) as e:
            sv.reduce_slices_noalloc(st.h, np.zeros(4, dtype=np.uint64))
        assert e.value.code == sv.SV_EINVAL
        sv.set_option(st.h, sv.SV_OPT_TIMING, 0)
        amps, stats = sv.reduce_slices_noalloc(st.h, np.arange(4, dtype=np.uint64))   # still usable
        assert abs(stats[0] - 1.0) <= 1e-5
    finally:
        st.close()
    tiered = sv.State(12, (1 << 3) | (1 << 9), "c64", tier=True)
    try:
        with pytest.raises(sv.SVError) as e:
            sv.reduce_slices_noalloc(tiered.h, np.zeros(4, dtype=np.uint64))
        assert e.value.code == sv.SV_EINVAL
    finally:
        tiered.close()
