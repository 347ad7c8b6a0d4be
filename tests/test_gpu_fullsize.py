"""GPU parity at full size: the 30-qubit headline in the launch configuration
the benchmark times, element by element against amplitudes the CPU oracle
stored (tests/golden/make_golden.py); states and slices of 2^32 amplitudes
against exact product-circuit amplitudes; the batch's own qubit counts
(20..28) against stored oracle amplitudes; and the kernel variant with
64-bit lane offsets.  Every call goes through libsv.so."""
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1910_09534_amd import planner, runner, serve, sv
from paper_1910_09534_amd import workload as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL64 = 1e-4


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: run tests/golden/make_golden.py")
    return np.load(path)


def product_circuit(n, depth, seed):
    """ABCDCDAB circuit on the near-square grid of n qubits with the vertical
    couplings removed: grid rows evolve independently."""
    full = W.sycamore_circuit(n, depth, seed=seed)
    rows, cols = W.grid_shape(n)
    keep = [g for g in full.gates if g.k == 1 or (g.qubits[0] // cols == g.qubits[1] // cols)]
    return W.Circuit(n, keep, depth), rows, cols


def product_amplitudes(circuit, rows, cols, bits):
    """Exact amplitudes of a row-separable circuit: the product of each grid
    row's own oracle amplitude."""
    out = np.ones(len(bits), dtype=np.complex128)
    for r in range(rows):
        sub = [W.Gate(tuple(q - r * cols for q in g.qubits), g.matrix) for g in circuit.gates
               if all(r * cols <= q < (r + 1) * cols for q in g.qubits)]
        psi = orc.simulate(W.Circuit(cols, sub))
        idx = ((bits.astype(np.uint64) >> np.uint64(r * cols)) & np.uint64((1 << cols) - 1)).astype(np.int64)
        out *= psi[idx]
    return out


@pytest.mark.parametrize("start,tile", [("sparse", 14), ("dense", 14), ("sparse", 13)])
def test_headline_vs_stored_oracle(start, tile):
    """30 qubits, depth 14, complex64, k <= 5: resident state in a torch
    buffer (create_state_ext), sv_reset, the plan for a run from |0...0>
    (sparse start) or the plan with every pass over the whole state, tiles
    of at most 14 positions (the default) or 13, FP64 reduction of the 2^16
    seeded bitstrings; all 2^16 amplitudes, the norm and the cross-entropy
    sums against the oracle's complex128 run."""
    torch = _torch()
    g = _golden("headline_30q_d14.npz")
    circ = W.config_circuit(2)
    bits = W.config_bitstrings(2)
    assert np.array_equal(bits, g["bitstrings"])
    n = circ.n
    assert planner.stage_tmax(n) == 14
    ops = planner.plan(circ.gates, 5, sparse_start=(start == "sparse"), tmax=tile)
    for o in ops:
        o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    h = sv.create_state_ext(n, 0, "c64", torch.cuda.current_stream().cuda_stream, buf.data_ptr(),
                            buf.numel() * 8)
    try:
        sv.set_option(h, sv.SV_OPT_STAGE, tile)
        sv.set_option(h, sv.SV_OPT_SPARSE_START, 1 if start == "sparse" else 0)
        sv.reset(h)
        c0 = sv.counters(h)["amps_swept"]
        planner.enqueue(h, ops, sv.SV_C64)
        amps, stats = sv.reduce_slices(h, bits)
        cnt = sv.counters(h)
        swept = cnt["amps_swept"] - c0
    finally:
        sv.destroy_state(h)
        del buf
        torch.cuda.empty_cache()
    err = orc.rel_l2(amps, g["amps"])
    print(f"headline {start} tile {tile}: rel_l2={err:.3e} norm={stats[0]:.9f} staged={cnt['staged_blocks']}", flush=True)
    assert cnt["staged_blocks"] > 0
    # the passes visit what the planner's model of the device says (tile
    # widening, support growth); every pass visits the whole state otherwise
    if start == "sparse":
        model = sum(1 << lv for _, lv in planner.sparse_passes(ops, n, None, tile))
    else:
        model = len(planner.stage_runs(ops, None, tile)) * (1 << n)
    assert swept == model, (swept, model)
    assert err <= TOL64
    assert abs(stats[0] - float(g["norm"])) <= 1e-5
    ref1, ref2 = (float(x) for x in g["xeb"])
    assert abs(stats[1] - ref1) <= TOL64 * ref1
    assert abs(stats[2] - ref2) <= 1e-3 * bits.size          # mean ln(N p) within 1e-3
    # the device's sums of its own amplitudes are the definition applied to them
    s1, s2 = orc.xeb_sums(n, amps)
    assert abs(stats[1] - s1) <= 1e-9 * s1 and abs(stats[2] - s2) <= 1e-9 * abs(s2)


@pytest.mark.parametrize("sparse", [1, 0])
def test_wide_lane_offsets_30q(sparse):
    """Two 5-qubit blocks on positions 25..29 of a 30-qubit complex64 state
    holding stale values.  From a sparse start the staged tile is positions
    0..3 and 25..29, so its lane bits reach position 29 and element offsets
    need 64 bits; with every pass over the whole state the tile widens with
    positions 4..7.  The 32 amplitudes whose set bits lie in 25..29 equal a
    5-qubit oracle run; others are zero."""
    torch = _torch()
    n = 30
    rng = np.random.default_rng(2929)
    qs = [25, 26, 27, 28, 29]
    us = [W.random_unitary(32, rng) for _ in range(2)]
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    buf.fill_(1.0 + 1.0j)                                   # stale contents
    torch.cuda.synchronize()                                # the library runs on a stream of its own
    h = sv.create_state_ext(n, 0, "c64", torch.cuda.current_stream().cuda_stream, buf.data_ptr(),
                            buf.numel() * 8, keep=True)
    try:
        sv.set_option(h, sv.SV_OPT_SPARSE_START, sparse)
        sv.reset(h)
        for u in us:
            sv.apply_fused(h, qs, u.astype(np.complex64), "c64")
        idx = np.array([sum(((c >> j) & 1) << qs[j] for j in range(5)) for c in range(32)], dtype=np.uint64)
        other = W.bitstrings(n, 64, seed=3) | np.uint64(1)     # bit 0 set: outside the block
        got = sv.gather_amplitudes(h, np.concatenate([idx, other]))
        cnt = sv.counters(h)
    finally:
        sv.destroy_state(h)
        del buf
        torch.cuda.empty_cache()
    ref = orc.zero_state(5)
    for u in us:
        orc.apply_dense(ref, [0, 1, 2, 3, 4], u)
    assert cnt["staged_blocks"] == 2
    assert orc.rel_l2(got[:32], ref) <= 1e-5
    assert np.abs(got[32:]).max() == 0.0


def test_resident_32q_product_circuit():
    """A resident 2^32-amplitude complex64 state (32 GiB) through the default
    unsliced path: 32 qubits on the 5 x 7 grid, depth 14, horizontal
    couplings only; 2^14 uniform bitstrings against exact amplitudes."""
    _torch()
    n = 32
    c, rows, cols = product_circuit(n, 14, seed=3232)
    bits = W.bitstrings(n, 1 << 14, seed=32)
    res = runner.simulate(c, bits, dtype="c64", kmax=5)
    ref = product_amplitudes(c, rows, cols, bits)
    err = orc.rel_l2(res["amps"], ref)
    print(f"resident 32q: rel_l2={err:.3e} norm={res['norm']:.9f} "
          f"staged={res['counters']['staged_blocks']}", flush=True)
    assert res["counters"]["staged_blocks"] > 0
    assert err <= TOL64
    assert abs(res["norm"] - 1.0) <= 1e-4


def test_sliced_34q_slices_of_2_32():
    """34 qubits with two sliced qubits: four slices of 2^32 amplitudes
    (32 GiB each) staged whole through the pageable host tier (128 GiB),
    slice sets alternating between two corner qubits and two central ones,
    the last gates on the sliced qubits applied by the FP64 cross-slice
    reduction; 2^14 bitstrings against exact product-circuit amplitudes."""
    _torch()
    n = 34
    c, rows, cols = product_circuit(n, 10, seed=3434)
    A, B = runner.grid_slice_sets(n)
    A2, B2 = (A[0], A[1]), (B[0], B[1])
    bits = W.bitstrings(n, 1 << 14, seed=34)
    res = runner.simulate_sliced(c, bits, A2, B2, dtype="c64", kmax=5, tier=True, pageable=True)
    ref = product_amplitudes(c, rows, cols, bits)
    err = orc.rel_l2(res["amps"], ref)
    print(f"sliced 34q (4 x 2^32): rel_l2={err:.3e} norm={res['norm']:.9f} phases={res['phases']} "
          f"h2d={res['counters']['bytes_h2d']}", flush=True)
    assert res["phases"] >= 2
    assert res["counters"]["bytes_h2d"] >= (1 << 32) * 8
    assert err <= TOL64
    assert abs(res["norm"] - 1.0) <= 1e-4


def test_serving_request_32q():
    """One 32-qubit request (a 32 GiB state) through the serving path's
    per-request runner, against exact product-circuit amplitudes."""
    torch = _torch()
    n = 32
    c, rows, cols = product_circuit(n, 12, seed=3200)
    bits = W.bitstrings(n, 1024, seed=320)
    req = serve.Request(0, 0.0, c, bits)
    st = torch.cuda.Stream()
    amps, norm, sweeps = serve.run_one(torch, st, req, kmax=5)
    torch.cuda.empty_cache()
    ref = product_amplitudes(c, rows, cols, bits)
    assert sweeps > 0
    assert orc.rel_l2(amps, ref) <= TOL64
    assert abs(norm - 1.0) <= 1e-4


def test_batch_qubit_counts_vs_stored_oracle():
    """One circuit of the 256-circuit batch specification per qubit count
    20..28, run as one staged, graph-captured batch (the benchmark's batch
    path, replayed twice); 1024 amplitudes each against stored oracle
    amplitudes."""
    _torch()
    g = _golden("batch_samples.npz")
    specs = {s["j"]: s for s in W.batch_specs()}
    circs, bits = [], []
    for j in g["j"]:
        s = specs[int(j)]
        circs.append(W.sycamore_circuit(s["n"], s["depth"], s["seed"]))
        bits.append(W.bitstrings(s["n"], 1024, s["bit_seed"]))
    assert [c.n for c in circs] == list(range(20, 29))
    plans = [planner.plan_fast(c.gates, 5, nloc=c.n, sparse_start=True) for c in circs]
    for p in plans:
        for o in p:
            o.matrix = np.ascontiguousarray(o.matrix, dtype=np.complex64)
    res = runner.run_batch(circs, bits, "c64", kmax=5, mfma_min_k=4, graph=True, repeats=2,
                           plans=plans, staged=True)
    for c, a, ref in zip(circs, res["amps"], g["amps"]):
        err = orc.rel_l2(a, ref)
        print(f"batch {c.n}q d{c.depth}: rel_l2={err:.3e}", flush=True)
        assert err <= TOL64
    assert res["info"]["graph"] == 1


@pytest.mark.parametrize("dtype,n", [("c64", 30), ("c128", 28)])
def test_permute_full_size_preserves_amplitudes(dtype, n):
    """A dense state of 2^30 (complex64) or 2^28 (complex128) amplitudes,
    re-laid-out by random permutations, a reversal and a swap of the low and
    high halves of the positions: the amplitudes of 2^16 logical bitstrings
    are bitwise the same after every permute (a permute moves amplitudes,
    it computes nothing)."""
    _torch()
    rng = np.random.default_rng(n)
    st = sv.State(n, 0, dtype)
    try:
        for q0 in range(0, n, 5):                            # blocks covering every qubit: a dense state
            qs = list(range(q0, min(q0 + 5, n)))
            st.fused(qs, W.random_unitary(1 << len(qs), rng))
        bits = W.bitstrings(n, 1 << 16, seed=n + 1)
        ref = st.gather(bits)
        assert np.count_nonzero(ref) > 0
        orders = [[int(x) for x in rng.permutation(n)] for _ in range(2)]
        orders += [list(range(n))[::-1], list(range(n // 2, n)) + list(range(n // 2))]
        for order in orders:
            st.permute(order)
            assert st.order() == order
            got = st.gather(bits)
            assert np.array_equal(got, ref)
    finally:
        st.close()
