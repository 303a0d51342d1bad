"""fstat_compute_noalloc: the entry point for callers that cannot allocate
keeps all its device scratch in the library's static array.  Through the
C-ABI it must give what fstat_compute gives on the same plan and inputs (the
same kernels: 2F bit for bit, and the oracle's values within 1e-4, or 5e-3
with FP16 coefficients), on two calls in a row of which the second has a
smaller work unit (the array keeps the first call's contents), with and
without a toplist; a work unit too large for the array is refused before
anything runs."""
import sys

import numpy as np
import pytest

from synth.device import to_device, alloc_output
from tests._helpers import small_workload, twoF_error

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _units():
    big = small_workload(900, n_det=2, slots=23, keep=0.85, n_sky=3, n_fd=9, n_f=700, dterms=8,
                         injections=((1, 5, 333, 15.0),))
    small = small_workload(901, n_det=1, slots=10, keep=1.0, n_sky=2, n_fd=3, n_f=150, dterms=16,
                           injections=((0, 1, 70, 12.0),))
    return big, small


@pytest.mark.parametrize("kernel,coef,tol", [("interp", "f32", 1e-4), ("interp", "f16", 5e-3), ("direct", "f32", 1e-4)])
def test_noalloc_matches_compute_twice(torch_cuda, oracle_lib, kernel, coef, tol):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    big, small = _units()
    with P.Plan(max_sft=big.n_sft, max_bins=max(big.n_bins, small.n_bins), max_sky=3, max_fd=9, max_f=700,
                max_dterms=16, kernel=kernel, coef=coef) as p:
        for k, w in enumerate((big, small)):
            top_k = 0 if k == 0 else 40
            _say(f"noalloc {kernel}/{coef} call {k}: n_sft={w.n_sft} n_bins={w.n_bins} templates={w.n_templates} "
                 f"top_k={top_k}")
            wu, _ = to_device(w)
            ref_out = alloc_output(w, fafb=True, top_k=top_k, threshold=8.0)
            out = alloc_output(w, fafb=True, top_k=top_k, threshold=8.0)
            p.compute(wu, ref_out)
            p.compute_noalloc(wu, out)
            torch.cuda.synchronize()
            a, b = out.twoF.cpu().numpy(), ref_out.twoF.cpu().numpy()
            assert np.array_equal(a, b), np.max(np.abs(a - b))
            assert np.array_equal(out.fa.cpu().numpy(), ref_out.fa.cpu().numpy())
            e = twoF_error(a.ravel(), oracle_lib.fstat(w)["twoF"])
            _say(f"  max_e={e.max():.2e}")
            assert e.max() <= tol
            if top_k:
                t1, t2 = P.toplist(out), P.toplist(ref_out)
                assert t1[4] == t2[4] and t1[4] > 0
                for x, y in zip(t1[:4], t2[:4]):
                    assert np.array_equal(x, y)


def test_noalloc_refuses_a_unit_larger_than_the_array(torch_cuda):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    # 2000 SFTs x ~1100 bins: 64 B of coefficients per (SFT, bin) is over 128 MiB
    w = small_workload(902, n_det=2, slots=1000, keep=1.0, n_sky=1, n_fd=1, n_f=1000, dterms=8, injections=(),
                       fdot_lo=0.0)
    need = w.n_sft * w.n_bins * 64
    assert need > P.NOALLOC_SCRATCH_BYTES
    _say(f"noalloc size check: n_sft={w.n_sft} n_bins={w.n_bins} coefficient bytes={need}")
    wu, _ = to_device(w)
    out = alloc_output(w)
    with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=1, max_fd=1, max_f=w.n_f, max_dterms=8) as p:
        with pytest.raises(P.FstatError) as e:
            p.compute_noalloc(wu, out)
        assert e.value.code == P.FSTAT_E_SIZE and "static array" in p.last_error()
        p.compute(wu, out)                    # the allocating entry point takes it
        torch.cuda.synchronize()
