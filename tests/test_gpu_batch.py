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
            sv.set_option(st.h, sv.SV_OPT_STAGE, 0)          # as in the batch: no staged passes
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
    plans = [planner.plan_fast(c.gates, 5, nloc=c.n, sparse_start=True) for c in circs]
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


@pytest.mark.parametrize("graph", [True, False])
def test_batch_reset_variant(graph):
    """States all reset before the launch run the batch's reset variant:
    staged passes from |0...0> that visit only the tiles inside each state's
    support, |0...0> written only ahead of a plain sweep, and the part of the
    state no pass reached cleared at the end.  Covers a plain sweep early in
    a plan, a state with no ops, a state whose support stays partial, and a
    planned circuit; the buffers hold the previous run's values at every
    reset.  A launch without a reset runs the ordinary variant on the
    current states (the ops applied twice)."""
    _gpu()
    rng = np.random.default_rng(17)
    U = lambda k: W.random_unitary(1 << k, rng)
    c = W.sycamore_circuit(20, 10, seed=71)
    specs = [
        (18, 9, [([4, 5, 6, 7, 8], U(5)), ([5, 6, 7, 8, 9], U(5)), ([15, 16, 17], U(3)),
                 ([10, 11, 12, 13], U(4)), ([12, 13, 14, 15], U(4))]),
        (19, 10, []),
        (18, 9, [([14, 15, 16], U(3)), ([4, 5, 6, 7], U(4)), ([6, 7, 8, 9], U(4))]),
        (22, 13, [([0, 1, 2, 3, 4], U(5)), ([2, 3, 4, 5, 6], U(5)), ([6, 7, 8, 9], U(4))]),
        (20, 11, [(list(o.qubits), o.matrix) for o in
                  planner.plan_fast(c.gates, 5, nloc=20, sparse_start=True)]),
    ]
    states, b = [], None
    try:
        for n, tmax, ops in specs:
            st = sv.State(n, 0, "c64")
            sv.set_option(st.h, sv.SV_OPT_STAGE, tmax)
            for qs, m in ops:
                st.fused(qs, np.asarray(m).astype(np.complex64))
            states.append(st)
        b = sv.batch_prepare([st.h for st in states], graph=graph)
        refs = []
        for n, _, ops in specs:
            psi = orc.zero_state(n)
            for qs, m in ops:
                orc.apply_dense(psi, qs, m)
            refs.append(psi)
        for rep in range(3):
            for st in states:
                sv.reset(st.h)
            sv.batch_launch(b)
            for st, (n, _, _), ref in zip(states, specs, refs):
                got = st.gather(np.arange(1 << n, dtype=np.uint64))
                assert orc.rel_l2(got, ref) <= 1e-4, (n, rep)
        info_reset = sv.batch_info(b)
        # no reset: the batch applies its ops to the states as they are
        sv.batch_launch(b)
        info_plain = sv.batch_info(b)
        assert info_reset["amps_swept"] < info_plain["amps_swept"]
        assert info_reset["sweeps"] == info_plain["sweeps"]
        for st, (n, _, ops), ref in zip(states, specs, refs):
            twice = ref.copy()
            for qs, m in ops:
                orc.apply_dense(twice, qs, m)
            got = st.gather(np.arange(1 << n, dtype=np.uint64))
            assert orc.rel_l2(got, twice) <= 2e-4, n
    finally:
        if b is not None:
            sv.batch_destroy(b)
        for st in states:
            st.close()


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
        # a state re-laid out after the batch was prepared is refused at launch
        u = W.random_unitary(4, np.random.default_rng(2)).astype(np.complex64)
        a.fused([0, 1], u)
        b = sv.batch_prepare([a.h])
        try:
            a.fused([2, 3], u)
            a.sync()
            a.permute(list(range(10))[::-1])
            with pytest.raises(sv.SVError):
                sv.batch_launch(b)
        finally:
            sv.batch_destroy(b)
    finally:
        a.close(); c.close(); t.close()


def test_tuned_staged_batch_matches_c128_batch_and_oracle():
    """The staged batch with the fusion width and tile limit chosen per qubit
    count by the autotuner (timed on this GPU): every result within the
    complex64 tolerance of the complex128 batch of the same circuits and of
    the oracle; the tuned choices are among the candidates."""
    _gpu()
    from paper_1910_09534_amd import autotune
    tuned = autotune.tune_staged([19, 21], kmaxes=(4, 5, 6), tiles=(10, 12), depth=8, reps=1)
    assert set(tuned["kmax"].values()) <= {4, 5, 6} and set(tuned["stage_t"].values()) <= {10, 12}
    pairs = [(c, b) for c, b in zip(*_batch(count=8, nmin=19, nmax=21, seed=29)) if c.n in (19, 21)]
    assert pairs
    circs, bits = [p[0] for p in pairs], [p[1] for p in pairs]
    res = runner.run_batch(circs, bits, "c64", kmax=tuned["kmax"], graph=True, repeats=2, staged=True,
                           stage_t=tuned["stage_t"])
    r128 = runner.run_batch(circs, bits, "c128", kmax=4, graph=True)
    for c, b, a64, a128 in zip(circs, bits, res["amps"], r128["amps"]):
        assert orc.rel_l2(a64, a128) <= 1e-4
        ref = orc.gather(orc.simulate(c), b)
        assert orc.rel_l2(a128, ref) <= 1e-12
        assert orc.rel_l2(a64, ref) <= 1e-4
