"""Precision forms on the work-unit-shaped inputs (2 detectors x 1000 SFTs,
2000 sky x 8 spindowns x 3600 frequencies, D = 8): the phase in FP64 versus
double-FP32 split products, and SFT storage in BF16 / FP16 with a per-SFT
scale, each against the FP64 oracle, with the 2F error reported per template
block (one sky point x 8 spindowns x 3600 frequencies)."""
import math
import sys

import numpy as np
import pytest

import synth
from synth.device import to_device, alloc_output
from tests._helpers import small_workload, twoF_error

pytestmark = pytest.mark.gpu

SKY_SAMPLE = list(range(0, 2000, 200))            # 10 blocks


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def cfg1():
    return synth.make_config(1)


def _plan(w, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                  max_dterms=16, **kw)


def _gpu(torch, w, storage="c64", phase="fp64"):
    wu, deq = to_device(w, storage)
    out = alloc_output(w)
    with _plan(w, storage=storage, phase=phase) as p:
        p.compute(wu, out)
        torch.cuda.synchronize()
    tw = out.twoF.cpu().numpy()
    del wu, out
    torch.cuda.empty_cache()
    return tw, deq


def _block_stats(e, n_blocks):
    e = e.reshape(n_blocks, -1)
    return e.max(axis=1), np.sqrt(np.mean(e * e, axis=1)), np.quantile(e, 0.9999, axis=1)


def test_split_phase_bins_and_phase_error(torch_cuda, oracle_lib, cfg1):
    torch = torch_cuda
    w = cfg1
    rng = np.random.default_rng(2)
    n = 50000
    idx = [rng.integers(0, m, n).astype(np.int32) for m in (w.n_sky, w.n_fd, w.n_f, w.n_sft)]
    wu, _ = to_device(w)
    dev = [torch.from_numpy(x).cuda() for x in idx]
    k = torch.empty(n, dtype=torch.int64, device="cuda")
    kap = torch.empty(n, dtype=torch.float64, device="cuda")
    ph = torch.empty(n, dtype=torch.float64, device="cuda")
    with _plan(w, phase="split") as p:
        p.bins(wu, *dev, k, kap, ph)
        torch.cuda.synchronize()
    k_ref, kap_ref, ph_ref, _ = oracle_lib.bins(w, tuple(idx[:3]))
    r = np.arange(n)
    assert np.array_equal(k.cpu().numpy(), k_ref[r, idx[3]])          # k* stays FP64
    assert np.array_equal(kap.cpu().numpy(), kap_ref[r, idx[3]])
    d = np.abs(ph.cpu().numpy() - ph_ref[r, idx[3]])
    d = np.minimum(d, 1.0 - d)
    _say(f"split-FP32 phase vs FP64: max |dphi| = {d.max():.2e} cycles, rms {math.sqrt(np.mean(d * d)):.2e}")
    # 1e-5 cycles (6e-5 rad) per SFT keeps the 2F error well inside the 1e-4 bound
    assert d.max() < 1e-5


def test_precision_forms_per_block(torch_cuda, oracle_lib, cfg1):
    torch = torch_cuda
    w = cfg1
    s, i, j = oracle_lib.all_templates(w, SKY_SAMPLE)
    nb = len(SKY_SAMPLE)
    ref = oracle_lib.fstat(w, (s, i, j))["twoF"]
    inj = np.zeros(len(s), dtype=bool)
    for x in w.injections:
        inj |= (s == x.sky_index) & (i == x.fdot_index) & (j == x.f_index)
    cand = (ref >= 20.0) | inj
    rows = []
    results = {}
    for name, storage, phase in [("c64/fp64", "c64", "fp64"), ("c64/split", "c64", "split"),
                                 ("bf16/fp64", "bf16", "fp64"), ("fp16/fp64", "fp16", "fp64")]:
        tw, deq = _gpu(torch, w, storage, phase)
        g = tw[s, i, j].astype(np.float64)
        assert np.all(np.isfinite(g))
        if deq is None:
            e_arith = twoF_error(g, ref)
        else:
            ref_q = oracle_lib.fstat(w, (s, i, j), sft=deq)["twoF"]
            e_arith = twoF_error(g, ref_q)
        e_store = twoF_error(g, ref)
        mx, rms, p9999 = _block_stats(e_arith, nb)
        smx, srms, _ = _block_stats(e_store, nb)
        rows.append(f"{name:10s} arith max {mx.max():.2e} rms {rms.max():.2e} p99.99 {p9999.max():.2e} | "
                    f"vs complex64 rms {srms.max():.2e} max {smx.max():.2e} candidates max "
                    f"{e_store[cand].max() if cand.any() else 0.0:.2e}")
        results[name] = (mx.max(), srms.max(), e_store[cand].max() if cand.any() else 0.0)
    _say("per-block 2F error (worst block), e = |2F - 2F_ref| / max(2F_ref, 4):")
    for r in rows:
        _say("  " + r)
    assert results["c64/fp64"][0] <= 1e-4
    assert results["c64/split"][0] <= 1e-4
    for name in ("bf16/fp64", "fp16/fp64"):
        assert results[name][0] <= 1e-4            # arithmetic parity on the stored values
        assert results[name][1] <= 5e-3            # storage error, rms per block
        assert results[name][2] <= 5e-3            # storage error on candidates


def test_split_phase_small_parity(torch_cuda, oracle_lib):
    torch = torch_cuda
    w = small_workload(500, n_det=2, slots=30, keep=0.9, n_sky=4, n_fd=5, n_f=600, dterms=16,
                       injections=((1, 3, 200, 15.0),))
    tw, _ = _gpu(torch, w, "c64", "split")
    ref = oracle_lib.fstat(w)["twoF"]
    e = twoF_error(tw.ravel(), ref)
    assert e.max() <= 1e-4, e.max()


def test_split_phase_with_direct_kernel_is_unsupported(torch_cuda):
    import paper_0904_1826_amd as P
    w = small_workload(501, n_sky=1, n_fd=1, n_f=10, injections=())
    with pytest.raises(P.FstatError) as e:
        _plan(w, phase="split", kernel="direct")
    assert e.value.code == P.FSTAT_E_UNSUPPORTED
