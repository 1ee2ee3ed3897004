"""pmg_vcycle_noalloc (work memory in the library's static device array) against
pmg_vcycle (the problem's own work buffers): the same kernels in the same order, so the
results agree to rounding-free equality, checked as the FP64 V-cycle tolerance of the
parity tests (1e-11 relative) and FP32 (2e-4).  Two calls in a row, the second on a
smaller problem, so that the second runs on memory the first left behind; then a problem
whose cycle needs more work memory than the array holds is rejected before anything runs.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2512_02577_amd import pmg  # noqa: E402
from paper_2512_02577_amd.inputs import rhs_vector  # noqa: E402

DEV = "cuda:0"


def relerr(x, ref):
    return float((x - ref).abs().max() / ref.abs().max())


def _check(dim, n, p, seed):
    print(f"case noalloc vcycle dim {dim} n {n} p {p}", flush=True)
    pr = pmg.make_problem(dim, n, p)
    r = torch.as_tensor(rhs_vector(dim, n, p, seed), dtype=torch.float64, device=DEV)
    for prec, tol in ((pmg.FP64, 1e-11), (pmg.FP32, 2e-4)):
        z_ref = torch.empty_like(r)
        pmg.vcycle(pr, r, z_ref, prec)
        z = torch.full_like(r, float("nan"))
        pmg.vcycle_noalloc(pr, r, z, prec)
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
        assert relerr(z, z_ref) <= tol, (prec, relerr(z, z_ref))
        # the FP64 cycle is bit-identical (same kernels, same order)
        if prec == pmg.FP64:
            assert torch.equal(z, z_ref)


def test_noalloc_vcycle_two_calls_second_smaller():
    _check(3, 32, 4, 61)   # 2.1M nodes: the largest 3D Q4 mesh whose work set fits
    _check(3, 8, 3, 62)    # smaller: runs on what the first call left in the array
    _check(2, 16, 5, 63)


def test_noalloc_vcycle_rejects_work_beyond_the_array():
    pr = pmg.make_problem(3, 48, 4)
    r = torch.as_tensor(rhs_vector(3, 48, 4, 64), dtype=torch.float64, device=DEV)
    z = torch.zeros_like(r)
    with pytest.raises(pmg.PmgError) as e:
        pmg.vcycle_noalloc(pr, r, z, pmg.FP64)
    assert e.value.status == pmg.ERR_INVALID_ARG and "scratch array" in str(e.value)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(z)) == 0  # nothing was enqueued
