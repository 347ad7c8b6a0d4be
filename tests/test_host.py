"""CPU-only checks of the host logic: the planner (fusion and diagonal
extraction are exact re-associations, checked on the oracle), and that the
C-ABI library loads and exports every function include/sv.h declares."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1910_09534_amd import planner
from paper_1910_09534_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def apply_ops_on_oracle(n, ops):
    psi = orc.zero_state(n)
    for o in ops:
        if o.kind == "dense":
            orc.apply_dense(psi, o.qubits, o.matrix)
        elif o.kind == "diag":
            orc.apply_diag(psi, o.qubits, o.matrix)
        else:
            raise AssertionError("unexpected op")
    return psi


@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("fold", [False, True])
def test_fusion_equals_sequential(kmax, fold):
    c = W.sycamore_circuit(12, 8, seed=31)
    ops = planner.fuse(c.gates, kmax if kmax >= 2 else 2, fold_diag=fold)
    for o in ops:
        if o.kind == "dense":
            assert len(o.qubits) <= max(kmax, 2)
    ref = orc.simulate(c)
    got = apply_ops_on_oracle(12, ops)
    assert np.abs(got - ref).max() < 1e-13
    assert sum(o.ngates for o in ops) == len(c.gates)


def test_fusion_generic_asymmetric_gates():
    c = W.random_generic_circuit(9, 60, seed=4, max_arity=3)
    for kmax in (3, 4, 5):
        for ops in (planner.fuse(c.gates, kmax), planner.fuse_grow(c.gates, kmax),
                    planner.plan(c.gates, kmax), planner.plan_fast(c.gates, kmax),
                    planner.plan(c.gates, kmax, staged=False),
                    planner.fuse_grow(c.gates, kmax, window=4, last_gain=0.5)):
            assert np.abs(apply_ops_on_oracle(9, ops) - orc.simulate(c)).max() < 1e-13


@pytest.mark.parametrize("kmax", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("window", [2, 4, 8])
def test_grow_fusion_equals_sequential(kmax, window):
    c = W.sycamore_circuit(12, 10, seed=32)
    ops = planner.fuse_grow(c.gates, kmax, window=window)
    assert all(len(o.qubits) <= kmax for o in ops)
    assert sum(o.ngates for o in ops) == len(c.gates)
    assert np.abs(apply_ops_on_oracle(12, ops) - orc.simulate(c)).max() < 1e-13


def test_split_eq1_is_exact():
    f = W.fsim()
    d, x = planner.split_eq1(f)
    assert np.abs(np.diag(d) @ x - f).max() == 0
    assert np.abs(x @ np.diag(d) - f).max() == 0        # the factors commute
    assert planner.split_eq1(W.random_unitary(4, np.random.default_rng(1))) is None


def test_embed_in_matches_oracle():
    rng = np.random.default_rng(2)
    g = W.random_unitary(4, rng)
    block = [5, 2, 7]
    e = planner.embed_in(block, (7, 5), g)
    psi = W.random_state(8, rng)
    a = orc.apply_dense(psi.copy(), block, e)
    b = orc.apply_dense(psi.copy(), (7, 5), g)
    assert np.abs(a - b).max() < 1e-14


def test_cfg2_plan_counts():
    c = W.config_circuit(2)
    ops = planner.plan(c.gates, 5)
    st = planner.stats(ops)
    assert sum(o.ngates for o in ops) == 621
    assert max(st["k_hist"]) <= 5
    # aggregation must cut the sweep count well below the gate count
    assert st["dense"] <= 40


def test_cfg2_sparse_plan_shape():
    """Regression pin on the 30-qubit depth-14 plan that the benchmark runs
    from |0...0> on 14-position tiles: every gate once, at most 13 HBM
    passes, and the passes visit at most 58 % of what as many full passes
    would (the device's visit counter is checked against this model in a
    GPU test)."""
    c = W.config_circuit(2)
    tmax = planner.stage_tmax(c.n)
    assert tmax == 14
    ops = planner.plan(c.gates, 5, sparse_start=True)
    assert sum(o.ngates for o in ops) == 621
    passes = planner.sparse_passes(ops, c.n, None, tmax)
    assert len(passes) <= 13
    visited = sum(1 << lv for _, lv in passes) / (len(passes) * (1 << c.n))
    assert visited <= 0.58


def test_stage_lds_budget_and_widening():
    """The LDS a staged pass needs: the padded tile (each group of 16
    elements takes 17 slots of 8 bytes: one pad per 16), then Re / Im of
    every block's matrix in float.  Three 5-qubit blocks fill a
    14-position tile's 160 KiB exactly, a fourth does not fit; [5, 4, 4]
    fills a 13-position tile's 80 KiB (two workgroups per CU).  Widening
    takes the widest tile within the limit whose LDS fits, from support
    positions only (others only up to 9)."""
    for t in range(9, 15):
        slots = (1 << t) // 16 * 17
        assert max(i + (i >> 4) for i in range(1 << t)) < slots          # every element's slot inside
        assert planner._stage_lds(t, []) == slots * 8
    assert planner._stage_lds(14, [5, 5, 5]) == planner.STAGE_LDS14 == 160 * 1024
    assert planner._stage_lds(14, [5, 5, 5, 4]) > planner.STAGE_LDS14
    assert planner._stage_lds(14, [4] * 8) <= planner.STAGE_LDS14
    assert planner._stage_lds(13, [5, 4, 4]) == planner.STAGE_LDS == 80 * 1024
    assert planner._stage_lds(13, [5, 5, 4]) > planner.STAGE_LDS
    full = (1 << 30) - 1
    tg = 0xF | sum(1 << p for p in (8, 9, 12, 13, 17, 20, 21, 25))     # 12 positions
    mask = lambda ps: sum(1 << p for p in ps)                             # noqa: E731
    # two 5-qubit blocks: widened to 14 with the two lowest free positions
    assert planner._tile_positions(tg, [5, 5], full, 30, 14) == (tg | mask([4, 5]), 14)
    # three fill 160 KiB at 14; 13 would need two workgroups' 80 KiB and fails
    assert planner._tile_positions(tg, [5, 5, 5], full, 30, 14) == (tg | mask([4, 5]), 14)
    assert planner._tile_positions(tg, [5, 5, 5], full, 30, 13) == (tg, 12)
    # four do not fit 13 or 14 positions: the tile stays at its 12
    assert planner._tile_positions(tg, [5, 5, 5, 5], full, 30, 14) == (tg, 12)
    # only support positions widen it
    assert planner._tile_positions(tg, [5, 5], mask([6, 29]) | tg, 30, 14) == (tg | mask([6, 29]), 14)
    assert planner._tile_positions(0xF | mask([20, 21]), [4], 0, 30, 14) == (0xF | mask([4, 5, 6, 20, 21]), 9)


def _declared_functions():
    names = []
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    so = os.path.join(ROOT, "paper_1910_09534_amd", "libsv.so")
    if not os.path.exists(so):
        from paper_1910_09534_amd import build
        build.build()
    lib = ctypes.CDLL(so)
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"libsv.so does not export {n}"
    from paper_1910_09534_amd import sv
    assert set(sv.EXPORTS) == set(names)


@pytest.mark.parametrize("n,depth", [(16, 14), (20, 12)])
def test_phase_schedule_is_a_reassociation(n, depth):
    """Applying each phase's gates in phase order, then the trailing operator
    on the last sliced set, gives the sequential circuit's state (Sec. 4: the
    subcircuits are a re-association of the same product of gates)."""
    from paper_1910_09534_amd import runner
    c = W.sycamore_circuit(n, depth, seed=77 + n)
    A, B = runner.grid_slice_sets(n)
    sp = planner.phase_schedule(c, A, B, kmax=5)
    ids = [i for ph in sp.phases for i in ph.gate_ids] + list(sp.trailing_gate_ids)
    assert sorted(ids) == list(range(len(c.gates)))
    for ph in sp.phases:
        assert not any(set(c.gates[i].qubits) & set(ph.sliced) for i in ph.gate_ids)
        assert sorted(ph.order) == list(range(n))
        assert ph.order[-len(ph.sliced):] == sorted(ph.sliced)
    # consecutive phases alternate between the two sets
    for p, q in zip(sp.phases, sp.phases[1:]):
        assert {p.sliced, q.sliced} == {tuple(A), tuple(B)}
    psi = orc.zero_state(n)
    for ph in sp.phases:
        psi = orc.apply_gates(psi, [c.gates[i] for i in ph.gate_ids])
    if sp.trailing is not None:
        assert set(sp.trailing_qubits) >= {q for i in sp.trailing_gate_ids for q in c.gates[i].qubits}
        psi = orc.apply_dense(psi, list(sp.trailing_qubits), sp.trailing)
    ref = orc.simulate(c)
    assert orc.rel_l2(psi, ref) < 1e-12


def test_phase_schedule_order_matters_when_dependent():
    """Control for the test above: swapping two dependent gates between phases
    changes the state, so the re-association check can fail."""
    from paper_1910_09534_amd import runner
    n = 16
    c = W.sycamore_circuit(n, 12, seed=91)
    A, B = runner.grid_slice_sets(n)
    sp = planner.phase_schedule(c, A, B, kmax=5)
    first, second = sp.phases[0].gate_ids, sp.phases[1].gate_ids
    psi = orc.zero_state(n)
    psi = orc.apply_gates(psi, [c.gates[i] for i in second])
    psi = orc.apply_gates(psi, [c.gates[i] for i in first])
    for ph in sp.phases[2:]:
        psi = orc.apply_gates(psi, [c.gates[i] for i in ph.gate_ids])
    if sp.trailing is not None:
        psi = orc.apply_dense(psi, list(sp.trailing_qubits), sp.trailing)
    assert orc.rel_l2(psi, orc.simulate(c)) > 1e-3


def test_sliced_36q_schedule_structure():
    """The 36-qubit depth-20 sliced workload: every gate is scheduled once,
    each phase leaves its sliced set untouched, and the four-qubit sets give
    16 slices per phase."""
    from paper_1910_09534_amd import runner
    c = W.config_circuit(3)
    A, B = runner.grid_slice_sets(c.n)
    assert len(A) == len(B) == 4
    sp = planner.phase_schedule(c, A, B, kmax=5)
    ids = [i for ph in sp.phases for i in ph.gate_ids] + list(sp.trailing_gate_ids)
    assert sorted(ids) == list(range(len(c.gates)))
    assert 2 <= len(sp.phases) <= 16
    for ph in sp.phases:
        assert not any(set(c.gates[i].qubits) & set(ph.sliced) for i in ph.gate_ids)
        assert all(max(o.qubits) < c.n and len(o.qubits) <= 5 for o in ph.ops)


def test_staging_transforms_are_exact():
    """Widening small blocks with low qubits and reordering for staged runs
    keep the product (sequential application on the oracle), the order
    respects every qubit's gate order, and the planner mirror of the device
    run formation only groups 4/5-qubit blocks within the tile limits."""
    c = W.sycamore_circuit(16, 12, seed=41)
    for ops0 in (planner.fuse(c.gates, 3), planner.fuse_grow(c.gates, 5, window=4, last_gain=0.6)):
        wide = planner.widen_small_blocks(ops0)
        assert all(len(o.qubits) >= 4 for o in wide if o.kind == "dense")
        ordered = planner.order_for_staging(wide)
        ref = orc.simulate(c)
        for ops in (wide, ordered):
            assert np.abs(apply_ops_on_oracle(16, ops) - ref).max() < 1e-12
        for run in planner.stage_runs(ordered):
            if len(run) < 2:
                continue
            pos = set(range(4)) | {q for i in run for q in ordered[i].qubits}
            assert len(pos) <= planner.STAGE_T and len(run) <= planner.STAGE_MAX_OPS
            assert all(len(ordered[i].qubits) in (4, 5) for i in run)


def test_support_order_is_a_reassociation():
    """Running gates in the order that brings qubits into play late keeps
    every qubit's own gate order, hence the product (gates on disjoint
    qubits commute); checked on the oracle for every activation order."""
    c = W.sycamore_circuit(16, 10, seed=51)
    ref = orc.simulate(c)
    for act in planner.activation_orders(c.gates, c.n):
        assert sorted(act) == list(range(c.n))
        g2 = planner.support_order(c.gates, act)
        assert len(g2) == len(c.gates)
        for q in range(c.n):
            assert [id(g) for g in c.gates if q in g.qubits] == [id(g) for g in g2 if q in g.qubits]
        psi = orc.apply_gates(orc.zero_state(c.n), g2)
        assert orc.rel_l2(psi, ref) < 1e-12


def test_activation_order_follows_the_long_axis():
    """On the 5 x 6 grid the Fiedler order brings in whole columns of five
    (the narrow cut) one after another."""
    c = W.config_circuit(2)
    rows, cols = W.grid_shape(c.n)
    fied = planner.activation_orders(c.gates, c.n)[0]
    for j in range(0, c.n, rows):
        assert len({q % cols for q in fied[j:j + rows]}) == 1


def test_plan_sparse_start_is_exact_and_modelled():
    """The sparse-start plan is the circuit's product; the pass model with
    a full support reduces to the dense staged model plus launch overheads;
    from |0...0> the first pass visits one tile."""
    c = W.sycamore_circuit(16, 10, seed=52)
    tmax = planner.stage_tmax(c.n)
    ops = planner.plan(c.gates, 5, sparse_start=True, nloc=c.n)
    assert np.abs(apply_ops_on_oracle(c.n, ops) - orc.simulate(c)).max() < 1e-12
    full = (1 << c.n) - 1
    nruns = sum(1 for r in planner.stage_runs(ops, None, tmax) if len(r) >= 2)
    assert abs(planner.sparse_cost(ops, c.n, None, tmax, support=full)
               - planner.staged_cost(ops, None, tmax) - planner.STAGE_MS_LAUNCH * nruns) < 1e-9
    passes = planner.sparse_passes(ops, c.n, None, tmax)
    r0, lv0 = passes[0]
    if len(r0) >= 2:
        P = {q for i in r0 for q in ops[i].qubits} | set(range(4))
        assert lv0 == max(9, len(P))
    assert all(lv <= c.n for _, lv in passes)
    dense = planner.plan(c.gates, 5, nloc=c.n)
    assert planner.sparse_cost(ops, c.n, None, tmax) <= planner.sparse_cost(dense, c.n, None, tmax) + 1e-9


def test_pack_lays_out_ops_for_apply_ops():
    """pack(): runs of dense / diagonal ops become one apply_ops call each
    (kinds, widths, concatenated qubits and matrices in the state dtype, no
    padding); a permute ends a run and stays its own call."""
    from paper_1910_09534_amd import sv
    rng = np.random.default_rng(5)
    ops = [planner.Op("dense", (3, 1), W.random_unitary(4, rng)),
           planner.Op("diag", (0, 2, 5), W.random_phases(8, rng)),
           planner.Op("perm", order=[1, 0, 2, 3, 4, 5]),
           planner.Op("dense", (4,), W.random_unitary(2, rng))]
    items = planner.pack(ops, "c64")
    assert isinstance(items, planner.PackedPlan) and len(items) == 3
    a, p, b = items
    assert isinstance(a, sv.PackedOps) and p is ops[2] and isinstance(b, sv.PackedOps)
    assert a.count == 2 and a.kinds.tolist() == [sv.SV_OP_FUSED, sv.SV_OP_DIAG]
    assert a.widths.tolist() == [2, 3] and a.qubits.tolist() == [3, 1, 0, 2, 5]
    assert a.data.dtype == np.complex64 and a.data.size == 16 + 8
    assert np.array_equal(a.data[:16], ops[0].matrix.astype(np.complex64).ravel())
    assert np.array_equal(a.data[16:], ops[1].matrix.astype(np.complex64))
    assert b.count == 1 and b.qubits.tolist() == [4]
    c = planner.pack(ops[:2], "c128")
    assert len(c) == 1 and c[0].data.dtype == np.complex128


def test_buddy_arena_blocks_disjoint_and_merge_back():
    """The serving arena's buddy allocator: random admissions and releases
    of power-of-two states never overlap, stay inside the arena, refuse what
    does not fit, and merge back into whole top blocks when all are freed."""
    from paper_1910_09534_amd.serve import BuddyArena
    rng = np.random.default_rng(11)
    a = BuddyArena(None, budget_bytes=7 * (1 << 30) + 12345, max_block=1 << 30, min_block=1 << 19)
    assert a.top == 1 << 30 and a.count == 7 and a.size == 7 << 30
    live = {}
    for step in range(4000):
        if live and rng.random() < 0.45:
            off = list(live)[int(rng.integers(len(live)))]
            a.release(off, live.pop(off))
            continue
        nbytes = 1 << int(rng.integers(16, 31))
        off = a.alloc(nbytes)
        if off is None:                                     # refused only when no block is large enough
            assert not any(v for bs, v in a.free.items() if bs >= a.block_size(nbytes))
            continue
        b = a.block_size(nbytes)
        assert off % b == 0 and 0 <= off and off + b <= a.size
        for o2, n2 in live.items():
            b2 = a.block_size(n2)
            assert off + b <= o2 or o2 + b2 <= off, "blocks overlap"
        live[off] = nbytes
    for off, nb in list(live.items()):
        a.release(off, nb)
    assert a.free.get(a.top) == {i * a.top for i in range(7)}
    assert all(not v for b, v in a.free.items() if b != a.top)
    assert a.alloc((1 << 30) + 1) is None


def test_open_state_files_rejects_missing_or_malformed_checkpoints(tmp_path):
    """open_state_files reads the checkpoint's metadata before touching the
    device: no checkpoint is SV_EIO, malformed metadata (bad counts, a
    layout that is not a permutation, sliced qubits off the top positions,
    file names with a path) is SV_EINVAL."""
    from paper_1910_09534_amd import sv
    with pytest.raises(sv.SVError) as e:
        sv.open_state_files(str(tmp_path))
    assert e.value.code == sv.SV_EIO
    good = ["sv_checkpoint 1", "n 4", "slice_mask 8", "dtype 0", "tag 3", "order 0 1 2 3", "slice_zero 0 1",
            "files 4", "f0", "f1", "f2", "f3"]
    bad = [
        [l.replace("order 0 1 2 3", "order 0 1 1 3") for l in good],      # not a permutation
        [l.replace("order 0 1 2 3", "order 3 1 2 0") for l in good],      # sliced qubit 3 not on top
        [l.replace("files 4", "files 3") for l in good][:-1],              # wrong file count
        [l.replace("f2", "../f2") for l in good],                          # a path
        [l.replace("n 4", "n 99") for l in good],                          # size out of range
        good[:5],                                                           # truncated
    ]
    for lines in bad:
        (tmp_path / "sv_checkpoint.meta").write_text("\n".join(lines) + "\n")
        with pytest.raises(sv.SVError) as e:
            sv.open_state_files(str(tmp_path))
        assert e.value.code == sv.SV_EINVAL, lines


def test_counter_traffic_only_for_the_kernels_and_plan_it_was_taken_on(tmp_path, monkeypatch):
    """The benchmark reports counter traffic for the staged passes only when
    the kernel sources are those the counters were taken on and the
    launches move the same algorithmic bytes (the same plan); otherwise
    null."""
    import json
    import bench
    path = tmp_path / "traffic.json"
    alg = 9.0e9
    path.write_text(json.dumps({"kernel_hash": bench.kernel_hash(), "per_kind": {"staged": {
        "traffic_bytes_per_launch": 9.6e9, "algorithmic_bytes_per_launch": alg}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.counter_traffic("staged", alg) == 9.6e9
    assert bench.counter_traffic("staged", alg * 1.01) is None      # another plan
    assert bench.counter_traffic("sweep", alg) is None              # no such kind profiled
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)     # other kernel sources
    assert bench.counter_traffic("staged", alg) is None
