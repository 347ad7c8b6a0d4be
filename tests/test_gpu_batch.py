"""GPU checks of the batched execution: many circuits of different qubit
counts in one graph-captured launch sequence.  Each result equals the same
plan run alone (bitwise), and the oracle (rel-L2 <= 1e-4 complex64,
<= 1e-12 complex128)."""
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


def _batch(count=10, nmin=12, nmax=20, seed=5):
    specs = W.batch_specs(count, seed=seed, nmin=nmin, nmax=nmax, dmin=6, dmax=12)
    circs = [W.sycamore_circuit(s["n"], s["depth"], s["seed"]) for s in specs]
    bits = [W.bitstrings(s["n"], 1024, s["bit_seed"]) for s in specs]
    return circs, bits


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_alone_and_oracle(graph):
    _gpu()
    circs, bits = _batch()
    kmax = {n: (4 if n % 2 else 5) for n in range(12, 21)}
    plans = [planner.plan(c.gates, kmax[c.n], staged=False) for c in circs]
    res = runner.run_batch(circs, bits, "c64", kmax=kmax, graph=graph, repeats=2, plans=plans)
    assert res["info"]["graph"] == graph
    for c, b, amps, p in zip(circs, bits, res["amps"], plans):
        st = sv.State(c.n, 0, "c64")
        try:
            planner.enqueue(st.h, p, st.dtype)
            alone = st.gather(b)
        finally:
            st.close()
        assert np.array_equal(alone, amps), "batched result differs from the same plan alone"
        ref = orc.gather(orc.simulate(c), b)
        assert orc.rel_l2(amps, ref) <= 1e-4


@pytest.mark.parametrize("graph", [True, False])
def test_staged_batch_equals_alone_and_oracle(graph):
    """States of 2^18..2^21 amplitudes with staged passes in the batch (tile
    limit n - 9): each equals the same plan and tile limit alone (bitwise)
    and the oracle; replays after sv_reset give the same result."""
    _gpu()
    circs, bits = _batch(count=6, nmin=18, nmax=21, seed=13)
    res = runner.run_batch(circs, bits, "c64", kmax=5, graph=graph, repeats=2, staged=True)
    plans = [planner.plan_fast(c.gates, 5, nloc=c.n) for c in circs]
    staged_blocks = 0
    for c, b, amps, p in zip(circs, bits, res["amps"], plans):
        st = sv.State(c.n, 0, "c64")
        try:
            sv.set_option(st.h, sv.SV_OPT_STAGE, planner.stage_tmax(c.n))
            planner.enqueue(st.h, p, st.dtype)
            alone = st.gather(b)
            staged_blocks += sv.counters(st.h)["staged_blocks"]
        finally:
            st.close()
        assert np.array_equal(alone, amps), "batched result differs from the same plan alone"
        ref = orc.gather(orc.simulate(c), b)
        assert orc.rel_l2(amps, ref) <= 1e-4
    assert staged_blocks > 0


def test_batch_c128_vs_c64_vs_oracle():
    _gpu()
    circs, bits = _batch(count=6, nmin=10, nmax=16, seed=9)
    r64 = runner.run_batch(circs, bits, "c64", kmax=5)
    r128 = runner.run_batch(circs, bits, "c128", kmax=4)
    for c, b, a64, a128, s128 in zip(circs, bits, r64["amps"], r128["amps"], r128["stats"]):
        ref = orc.gather(orc.simulate(c), b)
        assert orc.rel_l2(a128, ref) <= 1e-12
        assert orc.rel_l2(a64, a128) <= 1e-4
        assert abs(s128[0] - 1) < 1e-12


def test_batch_rejects_bad_inputs():
    _gpu()
    a = sv.State(10, 0, "c64")
    c = sv.State(10, 0, "c128")
    t = sv.State(10, 1 << 9, "c64", tier=True)
    try:
        with pytest.raises(sv.SVError):
            sv.batch_prepare([a.h, c.h])          # mixed dtypes
        with pytest.raises(sv.SVError):
            sv.batch_prepare([a.h, a.h])          # duplicate
        with pytest.raises(sv.SVError):
            sv.batch_prepare([a.h, t.h])          # tiered state
    finally:
        a.close(); c.close(); t.close()
