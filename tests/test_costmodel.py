"""The Sec. 5 running-time model against the values Tab. 1 and Tab. 2 print
(tests/golden/tab1_53q.txt, tests/golden/tab2_54q.txt)."""
import os

import pytest

from paper_1910_09534_amd import costmodel as cm

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read(fname):
    rows, scal, contraction = [], {}, None
    for line in open(os.path.join(GOLD, fname)):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "contraction":
            contraction = (float(f[1]), float(f[2]), float(f[3]))
        elif len(f) == 7:
            rows.append((cm.Row(f[0], float(f[1]), int(f[2]), int(f[3]), int(f[4])), float(f[5]), float(f[6])))
        else:
            scal[f[0]] = float(f[1])
    return rows, scal, contraction


def rel(a, b):
    return abs(a - b) / abs(b)


def test_time_per_aggregate_gate():
    assert round(cm.T_GATE_45Q, 5) == 0.22482          # Sec. 5


@pytest.mark.parametrize("fname,n", [("tab1_53q.txt", 53), ("tab2_54q.txt", 54)])
def test_tables_reproduced(fname, n):
    rows, scal, (cflops, cdays, cpf) = read(fname)
    out = cm.table(n, [r for r, _, _ in rows], cflops, int(scal["disk_transfers"]))
    for r, days, pf in rows:
        assert abs(out[f"days_{r.name}"] - days) <= 1.5e-6, r.name      # printed to 6 decimals
        # Tab. 2 row 3.3 prints Tab. 1's rate (18.4865); its own gates and
        # kernels (59, 15) give 18.467, so that one entry is held to 0.2 %
        # (rates print 4 decimals: half a unit of the last digit is allowed too)
        tol = 2e-3 if (n == 54 and r.name == "3.3") else 3e-4
        got = out[f"pflops_{r.name}"]
        assert abs(got - pf) <= max(tol * pf, 5.1e-5), (r.name, got, pf)
    # the FLOP counts print 4 significant digits
    assert rel(out["contraction_days"], cdays) <= 5e-4
    assert rel(cflops / (cdays * cm.DAY) / 1e15, cpf) <= 5e-4
    assert abs(out["alltoall_count"] - scal["alltoall_count"]) <= 1e-6
    assert abs(out["alltoall_days"] - scal["alltoall_days"]) <= 1.5e-6
    assert abs(out["disk_days"] - scal["disk_days"]) <= 1.5e-6
    assert rel(out["compute_days"], scal["compute_days"]) <= 5e-4
    assert rel(out["compute_pflops"], scal["compute_pflops"]) <= 5e-4
    assert rel(out["total_days"], scal["total_days"]) <= 5e-5
    assert out["kernels_total"] == scal["kernels_total"]
    assert out["gates_total"] == scal["gates_total"]


def test_tables_internally_consistent():
    """Sums the tables print, recomputed from their own printed rows."""
    for fname in ("tab1_53q.txt", "tab2_54q.txt"):
        rows, scal, (_, cdays, _) = read(fname)
        assert abs(sum(d for _, d, _ in rows) + cdays - scal["compute_days"]) <= 5e-6
        assert abs(scal["compute_days"] + scal["alltoall_days"] + scal["disk_days"]
                   - scal["total_days"]) <= 2e-6


def test_disk_space():
    assert cm.disk_space_pib(53) == 64 and cm.disk_space_pib(54) == 128   # Sec. 5


@pytest.mark.parametrize("fname,base_name,n", [("tab3_53q_depths.txt", "tab1_53q.txt", 53),
                                               ("tab4_54q_depths.txt", "tab2_54q.txt", 54)])
def test_depth_tables(fname, base_name, n):
    """Tabs. 3 and 4 (run time per depth) follow from the 20-cycle table's
    fixed parts plus the per-kernel, per-all-to-all and per-transfer costs.
    Run times print two decimals; every printed value is reproduced within
    0.006 days (the 54-qubit 10-cycle row is the farthest, 0.0055)."""
    rows, scal, (cflops, _, _) = read(base_name)
    base = cm.table(n, [r for r, _, _ in rows], cflops, int(scal["disk_transfers"]))
    small = sum(r.kernels for r, _, _ in rows if cm.small_tensor(r))
    seen20 = False
    for line in open(os.path.join(GOLD, fname)):
        if not line.strip() or line.startswith("#"):
            continue
        cyc, dx, a2a, k, days = line.split()
        est = cm.depth_estimate_days(n, int(k), float(a2a), int(dx), base, small)
        assert abs(est - float(days)) <= 0.006, (cyc, est, days)
        if int(cyc) == 20:
            seen20 = True
            assert int(k) == scal["kernels_total"] and abs(float(a2a) - scal["alltoall_count"]) < 1e-3
    assert seen20
