"""GPU checks of the request server (continuous batching): results in the
mix equal results alone (bitwise: same plan, deterministic kernels) and the
oracle; admission respects the HBM budget; requests overlap."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1910_09534_amd import serve
from paper_1910_09534_amd import workload as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _requests(count, nmin, nmax, rate, seed=11):
    trace = W.serving_trace(count, rate=rate, seed=seed, nmin=nmin, nmax=nmax, dmin=6, dmax=12)
    return [serve.Request(t["j"], t["t"], W.sycamore_circuit(t["n"], t["depth"], t["seed"]),
                          W.bitstrings(t["n"], 1024, t["bit_seed"])) for t in trace]


def test_mix_equals_alone_and_oracle():
    torch = _gpu()
    reqs = _requests(24, 12, 20, rate=400.0)
    srv = serve.Server(budget_bytes=64 << 20, slots=6)      # tight budget: admission waits
    mixed = srv.serve(reqs)
    assert srv.max_inflight >= 2, "requests never overlapped"
    st = torch.cuda.Stream()
    for r, m in zip(reqs, mixed):
        amps, norm, _ = serve.run_one(torch, st, r, kmax=5)
        assert np.array_equal(amps, m.amps), f"request {r.rid}: mix differs from alone"
        ref = orc.gather(orc.simulate(r.circuit), r.bits)
        assert orc.rel_l2(m.amps, ref) <= 1e-4
        assert abs(m.norm - 1) < 1e-4
    s = serve.summarize(mixed)
    assert s["completed"] == 24 and s["p99_latency_s"] >= s["p50_latency_s"]


def test_budget_is_respected():
    _gpu()
    reqs = _requests(8, 16, 18, rate=1000.0, seed=3)
    budget = 2 * (1 << 18) * 8                                 # two 18-qubit states
    srv = serve.Server(budget_bytes=budget, slots=8)
    peak = []
    orig = srv._worker

    def spy(*args):
        peak.append(srv.mem_used)
        return orig(*args)
    srv._worker = spy
    srv.serve(reqs)
    assert max(peak) <= budget


def test_oversized_request_rejected():
    _gpu()
    reqs = _requests(1, 20, 20, rate=10.0)
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=1 << 20, slots=2).serve(reqs)
