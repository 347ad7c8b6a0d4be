"""Pins of the contraction-deferral oracle (App. A: the EI and E2Q
synthesized gates and the contraction over entanglement indices; Sec. 2:
contraction deferral).  Each check compares the oracle with something
other than itself: the gate applied to the product of the two tensors
(closed form), the plain simulation of the whole circuit, brute-force sums
on tiny tensors, and a planted label swap that must be caught."""
import numpy as np
import pytest

from oracle import deferral as D
from oracle import oracle as orc
from paper_1910_09534_amd import workload as W


def _rand(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("a,b", [(0, 3), (2, 5), (1, 4)])
@pytest.mark.parametrize("a_first", [True, False])
def test_one_bridging_gate_is_the_gate_on_the_product(a, b, a_first):
    """sum_{a', a} EI(phi) E2Q(chi) = 2Q applied to phi (x) chi (the first
    equation of App. A), for a general (non-unitary, asymmetric) 4x4 gate
    and either order of the gate's qubits."""
    rng = np.random.default_rng(10 * a + b + a_first)
    phi = _rand(8, rng)                       # qubits 0, 1, 2
    chi = _rand(8, rng)                       # qubits 3, 4, 5
    g = _rand((4, 4), rng)
    qs = [a, b] if a_first else [b, a]
    t1, l1 = D.from_state(phi, [0, 1, 2])
    t2, l2 = D.from_state(chi, [3, 4, 5])
    t1, l1 = D.ei(t1, l1, a, 0, 1)
    t2, l2 = D.e2q(t2, l2, qs, g, a, b, 0, 1)
    t, lab = D.contract(t1, l1, t2, l2)
    got = D.to_state(t, lab, list(range(6)))
    ref = orc.apply_dense(np.kron(chi, phi), qs, g)
    assert np.abs(got - ref).max() < 1e-12


def test_planted_label_swap_is_caught():
    """Control: exchanging the two entanglement indices in E2Q (a plausible
    slip) changes the result, so the pin above can fail."""
    rng = np.random.default_rng(3)
    phi, chi, g = _rand(8, rng), _rand(8, rng), _rand((4, 4), rng)
    t1, l1 = D.from_state(phi, [0, 1, 2])
    t2, l2 = D.from_state(chi, [3, 4, 5])
    t1, l1 = D.ei(t1, l1, 1, 0, 1)
    t2, l2 = D.e2q(t2, l2, [1, 4], g, 1, 4, 1, 0)          # e_a and e_ap exchanged
    t, lab = D.contract(t1, l1, t2, l2)
    got = D.to_state(t, lab, list(range(6)))
    ref = orc.apply_dense(np.kron(chi, phi), [1, 4], g)
    assert np.abs(got - ref).max() > 1e-3


@pytest.mark.parametrize("n,depth,cols", [(8, 6, 2), (12, 5, 2), (12, 4, 3)])
def test_deferred_circuit_equals_simulation(n, depth, cols):
    """A whole ABCDCDAB circuit as two tensors (the first `cols` grid
    columns, the rest), every bridging gate deferred: the contraction equals
    the plain simulation of the circuit."""
    c = W.sycamore_circuit(n, depth, seed=200 + n + depth)
    rows, ncol = W.grid_shape(n)
    part1 = [q for q in range(n) if q % ncol < cols]
    bridging = sum(1 for g in c.gates if len(g.qubits) == 2
                   and ((g.qubits[0] in part1) != (g.qubits[1] in part1)))
    assert bridging >= 2
    got = D.deferred_simulate(c, part1)
    assert np.abs(got - orc.simulate(c)).max() < 1e-12


@pytest.mark.parametrize("n1,n2,e", [(1, 1, 1), (2, 1, 2), (1, 3, 0), (3, 2, 3)])
def test_contract_matrix_brute_force(n1, n2, e):
    """The GPU call's layout form, checked by explicit sums and against the
    label contraction."""
    rng = np.random.default_rng(n1 * 16 + n2 * 4 + e)
    t1 = _rand((1 << e) << n1, rng)
    t2 = _rand((1 << e) << n2, rng)
    got = D.contract_matrix(t1, t2, n1, n2, e)
    for x2 in range(1 << n2):
        for x1 in range(1 << n1):
            s = sum(t1[k * (1 << n1) + x1] * t2[k * (1 << n2) + x2] for k in range(1 << e))
            assert abs(got[x2 * (1 << n1) + x1] - s) < 1e-12
    # the same by labels: bits 0..n1-1 of t1 are qubits 0..n1-1, bits above are e
    l1 = [("q", j) if j < n1 else ("e", j - n1) for j in reversed(range(n1 + e))]
    l2 = [("q", n1 + j) if j < n2 else ("e", j - n2) for j in reversed(range(n2 + e))]
    t, lab = D.contract(t1.reshape((2,) * (n1 + e)), l1, t2.reshape((2,) * (n2 + e)), l2)
    assert np.abs(D.to_state(t, lab, list(range(n1 + n2))) - got).max() < 1e-12


@pytest.mark.parametrize("n,depth,ncycles", [(12, 6, 2), (16, 5, 3), (12, 4, 4)])
def test_device_bookkeeping_on_the_oracle(n, depth, ncycles):
    """The package's split (positions, EI / E2Q operator matrices, final
    permutations, relabelled remaining gates), replayed with the oracle's
    primitives, gives the plain simulation of the circuit."""
    from oracle import brute
    from paper_1910_09534_amd import deferral
    c = W.sycamore_circuit(n, depth, seed=300 + n)
    sp = deferral.split(c, deferral.grid_halves(n), ncycles)
    assert sp.n_bridging >= 1
    s1 = orc.zero_state(sp.n1 + sp.e)
    for g in sp.ops1:
        orc.apply_dense(s1, list(g.qubits), g.matrix)
    s2 = orc.zero_state(sp.n2 + sp.e)
    for g in sp.ops2:
        orc.apply_dense(s2, list(g.qubits), g.matrix)
    t1 = brute.permute_state(s1, sp.n1 + sp.e, sp.order1)
    t2 = brute.permute_state(s2, sp.n2 + sp.e, sp.order2)
    joint = D.contract_matrix(t1, t2, sp.n1, sp.n2, sp.e)
    for g in sp.rest:
        orc.apply_dense(joint, list(g.qubits), g.matrix)
    ref = orc.simulate(c)
    x = np.arange(1 << n, dtype=np.uint64)
    assert np.abs(joint[sp.joint_bits(x).astype(np.int64)] - ref).max() < 1e-12


def test_device_bookkeeping_any_gate_order():
    """Bridging gates listed in either qubit order, several on the same
    qubit, general (non-unitary) matrices, and gates after the deferred
    prefix: the package's split replayed on the oracle equals applying the
    gates in sequence."""
    from oracle import brute
    from paper_1910_09534_amd import deferral
    rng = np.random.default_rng(12)
    n = 9
    part1 = [0, 2, 3, 7]
    part2 = [q for q in range(n) if q not in part1]
    bridging = {5: (0, 1), 13: (5, 3), 22: (2, 8), 31: (6, 2)}   # either order, qubit 2 twice
    gates = []
    for i in range(40):
        if i in bridging:
            qs = bridging[i]
        else:
            side = part1 if rng.random() < 0.5 else part2
            k = int(rng.integers(1, 3))
            qs = tuple(int(x) for x in rng.choice(side, size=k, replace=False))
        gates.append(W.Gate(qs, _rand((1 << len(qs), 1 << len(qs)), rng), "g", i // 4))
    c = W.Circuit(n, gates, 10)
    ref = orc.zero_state(n)
    for g in gates:
        orc.apply_dense(ref, list(g.qubits), g.matrix)
    for ncycles in (3, 6, 10):
        sp = deferral.split(c, part1, ncycles)
        firsts = {g.qubits[0] in part1 for g in gates[:4 * ncycles] if len(g.qubits) == 2
                  and (g.qubits[0] in part1) != (g.qubits[1] in part1)}
        if ncycles == 10:
            assert firsts == {True, False}              # both orders occur
        s1 = orc.zero_state(sp.n1 + sp.e)
        for g in sp.ops1:
            orc.apply_dense(s1, list(g.qubits), g.matrix)
        s2 = orc.zero_state(sp.n2 + sp.e)
        for g in sp.ops2:
            orc.apply_dense(s2, list(g.qubits), g.matrix)
        joint = D.contract_matrix(brute.permute_state(s1, sp.n1 + sp.e, sp.order1),
                                  brute.permute_state(s2, sp.n2 + sp.e, sp.order2), sp.n1, sp.n2, sp.e)
        for g in sp.rest:
            orc.apply_dense(joint, list(g.qubits), g.matrix)
        x = np.arange(1 << n, dtype=np.uint64)
        got = joint[sp.joint_bits(x).astype(np.int64)]
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
