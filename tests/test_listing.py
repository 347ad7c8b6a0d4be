"""The implementation listings of App. A (tests/golden/listing_{53,54}q.txt,
extracted as printed by tests/golden/make_listing.py) against the paper's own
tables, and the planner's aggregation against the listings'.

- The listing's "cache" lines (the 5-qubit aggregate gates) and "gate" lines
  (two-qubit gates), counted per tensor and phase, give Tab. 1 / Tab. 2's
  "5Q kernels per disk slice" and "Num gates" columns row by row; tensor 2's
  gate count includes its E2Q synthesized gates (one per deferred bridging
  gate, Sec. 2 and App. A).
- Every aggregate spans at most 5 qubits and holds the qubits of the gates
  listed under it.
- The planner (`planner.plan`, k <= 5), run on each subcircuit's two-qubit
  gates in depth order, needs no more aggregate gates in total than the
  paper's aggregation, and at most one more per subcircuit."""
import collections
import os

import numpy as np
import pytest

from paper_1910_09534_amd import planner
from paper_1910_09534_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# table rows in order for each tensor's phases (Tabs. 1 and 2)
ROWS = {"1": ["1"], "2": ["2"], "3": ["3.3", "3.4", "3.5"], "4": ["4.4", "4.5"], "5": ["5.5", "5.6"]}


def listing(n):
    with open(os.path.join(GOLDEN, f"listing_{n}q.txt")) as f:
        return [line.rstrip("\n").split("\t") for line in f if not line.startswith("#")]


def table(fname):
    rows = {}
    totals = {}
    with open(os.path.join(GOLDEN, fname)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0][0].isdigit() and len(p) == 7:
                rows[p[0]] = {"kernels": int(p[2]), "gates": int(p[4])}
            elif len(p) == 2:
                totals[p[0]] = float(p[1])
    return rows, totals


def per_subcircuit(rows):
    """(tensor, phase) -> (aggregate count, two-qubit gates with depth)."""
    caches = collections.Counter()
    gates = collections.defaultdict(list)
    for r in rows:
        key = (r[0], int(r[1]))
        if r[2] == "new" and r[4] == "cache":
            caches[key] += 1
        elif r[2] == "gate":
            gates[key].append((int(r[3]), tuple(int(x) for x in r[5].split(","))))
    return caches, gates


@pytest.mark.parametrize("n,fname", [(53, "tab1_53q.txt"), (54, "tab2_54q.txt")])
def test_listing_counts_match_tables(n, fname):
    rows = listing(n)
    tab, totals = table(fname)
    caches, gates = per_subcircuit(rows)
    e2q = sum(1 for r in rows if r[2] == "entgl" and r[4] == "E2Q")
    ei = sum(1 for r in rows if r[2] == "entgl" and r[4] == "EI")
    assert e2q == ei > 0                                  # one of each per deferred bridging gate
    got = {}
    for tensor, labels in ROWS.items():
        phases = sorted(p for (t, p) in caches if t == tensor)
        if len(labels) == 1:
            k = sum(caches[(tensor, p)] for p in phases)
            g = sum(len(gates[(tensor, p)]) for p in phases) + (e2q if tensor == "2" else 0)
            got[labels[0]] = {"kernels": k, "gates": g}
        else:
            assert len(phases) == len(labels)
            for lab, p in zip(labels, phases):
                got[lab] = {"kernels": caches[(tensor, p)], "gates": len(gates[(tensor, p)])}
    assert got == tab
    assert sum(v["kernels"] for v in got.values()) == totals["kernels_total"]
    assert sum(v["gates"] for v in got.values()) == totals["gates_total"]


@pytest.mark.parametrize("n", [53, 54])
def test_listing_aggregates_valid(n):
    rows = listing(n)
    assert rows[0][2:5] == ["define", "0", "qubits"] and int(rows[0][5]) == n
    cache = None
    held = 0
    for r in rows:
        if r[2] == "new" and r[4] == "cache":
            cache = {int(x) for x in r[5].split(",")}
            assert 1 <= len(cache) <= 5
        elif r[2] == "gate":
            q = {int(x) for x in r[5].split(",")}
            assert len(q) == 2 and all(0 <= x < n for x in q)
            assert cache is not None and q <= cache, r
            held += 1
        elif r[2] in ("entgl", "all2all", "write", "read", "slice") or (r[2] == "new" and r[4] == "tensor"):
            cache = None                                   # an aggregate holds only the gates listed under it
    assert held == sum(1 for r in rows if r[2] == "gate")


@pytest.mark.parametrize("n", [53, 54])
def test_planner_aggregation_against_listing(n):
    caches, gates = per_subcircuit(listing(n))
    u = W.random_unitary(4, np.random.default_rng(n))
    ours, paper = 0, 0
    for key, gl in gates.items():
        seq = [W.Gate(q, u) for _, q in sorted(gl, key=lambda x: x[0])]     # depth order (stable)
        ops = planner.plan(seq, 5, staged=False)
        k = sum(1 for o in ops if o.kind == "dense")
        assert all(len(o.qubits) <= 5 for o in ops)
        assert k <= caches[key] + 1, (key, k, caches[key])
        ours += k
        paper += caches[key]
    assert ours <= paper, (ours, paper)
