"""GPU checks of contraction deferral: sv_contract against the oracle's
contraction (App. A) on seeded random tensors, on the matrix-core path and
the plain path, complex64 and complex128; argument errors; and the whole
deferred pipeline (two tensors with EI / E2Q, contraction, the rest of the
circuit on the joint state) against the plain simulation."""
import numpy as np
import pytest

from oracle import deferral as D
from oracle import oracle as orc
from paper_1910_09534_amd import deferral, runner, sv
from paper_1910_09534_amd import workload as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rand(size, rng):
    return (rng.standard_normal(size) + 1j * rng.standard_normal(size)) / np.sqrt(2)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n1,n2,e,dtype", [
    (6, 7, 4, "c64"), (7, 8, 5, "c64"), (8, 7, 6, "c64"), (10, 9, 8, "c64"), (6, 10, 10, "c64"),
    (5, 7, 4, "c64"), (6, 6, 4, "c64"), (6, 7, 3, "c64"), (2, 3, 1, "c64"), (0, 0, 0, "c64"),
    (3, 2, 0, "c64"), (5, 6, 3, "c128"), (7, 8, 5, "c128")])
def test_contract_matches_oracle(n1, n2, e, dtype, fp32):
    """Matrix-core tiles (2^n2 >= 128, 2^n1 >= 64, 2^e >= 16; the split-fp16
    form, or the fp32 3M form with fp32) and the plain kernel (every other
    size) against the oracle, element by element."""
    torch = _torch()
    rng = np.random.default_rng(n1 * 1000 + n2 * 10 + e)
    t1 = _rand((1 << e) << n1, rng)
    t2 = _rand((1 << e) << n2, rng)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    ndt = np.complex64 if dtype == "c64" else np.complex128
    g1 = torch.from_numpy(t1.astype(ndt)).cuda()
    g2 = torch.from_numpy(t2.astype(ndt)).cuda()
    out = torch.full((1 << (n1 + n2),), complex(7.0, 7.0), dtype=tdt, device="cuda")
    sv.contract(g1.data_ptr(), g2.data_ptr(), out.data_ptr(), n1, n2, e, dtype,
                torch.cuda.current_stream().cuda_stream, fp32=fp32)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    ref = D.contract_matrix(t1.astype(ndt), t2.astype(ndt), n1, n2, e)
    # FP32 sums over 2^e terms of unit-size products: error ~ 1e-7 sqrt(2^e)
    tol = 1e-12 if dtype == "c128" else 2e-6 * max(1.0, np.sqrt(1 << e))
    assert np.abs(got - ref).max() <= tol * max(1.0, np.abs(ref).max())
    assert orc.rel_l2(got, ref) <= (1e-13 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("s1,s2", [(1e-6, 1.0), (1.0, 3e5), (1e-15, 1e-12), (1e10, 1e-10)])
def test_contract_split_accuracy_independent_of_scale(s1, s2):
    """The split-fp16 form scales each tensor from its own largest component:
    tensors of very different sizes keep single-precision accuracy (no fp16
    overflow or underflow)."""
    torch = _torch()
    n1, n2, e = 7, 8, 6
    rng = np.random.default_rng(31)
    t1 = (_rand((1 << e) << n1, rng) * s1).astype(np.complex64)
    t2 = (_rand((1 << e) << n2, rng) * s2).astype(np.complex64)
    g1 = torch.from_numpy(t1).cuda()
    g2 = torch.from_numpy(t2).cuda()
    out = torch.zeros(1 << (n1 + n2), dtype=torch.complex64, device="cuda")
    sv.contract(g1.data_ptr(), g2.data_ptr(), out.data_ptr(), n1, n2, e, "c64",
                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    ref = D.contract_matrix(t1, t2, n1, n2, e)
    assert np.all(np.isfinite(got))
    assert orc.rel_l2(got, ref) <= 1e-5


def test_contract_rejects_bad_arguments():
    torch = _torch()
    a = torch.zeros(1 << 10, dtype=torch.complex64, device="cuda")
    b = torch.zeros(1 << 10, dtype=torch.complex64, device="cuda")
    o = torch.zeros(1 << 12, dtype=torch.complex64, device="cuda")
    with pytest.raises(sv.SVError):
        sv.contract(0, b.data_ptr(), o.data_ptr(), 6, 6, 4, "c64")
    with pytest.raises(sv.SVError):
        sv.contract(a.data_ptr() + 8, b.data_ptr(), o.data_ptr(), 6, 6, 4, "c64")     # misaligned
    with pytest.raises(sv.SVError):
        sv.contract(a.data_ptr(), b.data_ptr(), a.data_ptr(), 6, 6, 4, "c64")         # overlap
    with pytest.raises(sv.SVError):
        sv.contract(a.data_ptr(), b.data_ptr(), o.data_ptr(), 30, 20, 4, "c64")       # too large
    with pytest.raises(sv.SVError):
        sv.contract(a.data_ptr(), b.data_ptr(), o.data_ptr(), 6, 6, -1, "c64")
    with pytest.raises(sv.SVError):
        sv.contract(a.data_ptr(), b.data_ptr(), o.data_ptr(), 2, 2, 31, "c64")       # e above 30


@pytest.mark.parametrize("n,depth,ncycles", [(16, 8, 2), (16, 6, 4), (20, 8, 3)])
def test_deferred_pipeline_equals_simulation(n, depth, ncycles):
    """Two tensors (left and right halves of the grid) with EI / E2Q for the
    bridging gates of the first cycles, the contraction, then the rest of
    the circuit on the joint state: every amplitude equals the plain
    simulation."""
    _torch()
    c = W.sycamore_circuit(n, depth, seed=400 + n + ncycles)
    bits = np.arange(1 << n, dtype=np.uint64)
    res = runner.simulate_deferred(c, bits, deferral.grid_halves(n), ncycles)
    assert res["split"].n_bridging >= 2
    ref = orc.simulate(c)
    assert orc.rel_l2(res["amps"], ref) <= 1e-5
    assert abs(res["norm"] - 1.0) <= 1e-5
