"""The Dirichlet offset's edges on the GPU: work units where every (template,
SFT) pair has kappa = 0 exactly, or kappa = 1 - 2^-34 (Dphi just below an
integer), through the direct kernel (bounded central weights), the interp
kernel with FP32 and with FP16 coefficients, and the batched form, each
against the FP64 oracle over every template.  At kappa = 0 the window keeps
the bin k* alone; as kappa -> 1 it keeps bin k* + 1 alone (Listing 1,
Section 2, per-SFT body read as the Dirichlet demodulation)."""
import sys

import numpy as np
import pytest

from synth.device import to_device, alloc_output
from tests._helpers import kappa_edge_workload, twoF_error

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


def _plan(ws, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                  max_sky=max(w.n_sky for w in ws), max_fd=max(w.n_fd for w in ws), max_f=max(w.n_f for w in ws),
                  max_dterms=16, **kw)


FORMS = [("direct", "f32", 1e-4), ("interp", "f32", 1e-4), ("interp", "f16", 5e-3)]


@pytest.mark.parametrize("kernel,coef,tol", FORMS, ids=[f"{k}-{c}" for k, c, _ in FORMS])
@pytest.mark.parametrize("edge", ["zero", "one"])
def test_kappa_edge_single(torch_cuda, oracle_lib, edge, kernel, coef, tol):
    torch = torch_cuda
    w = kappa_edge_workload(edge)
    _say(f"kappa {edge} {kernel} {coef}: n_sft={w.n_sft} n_bins={w.n_bins} templates={w.n_templates}")
    wu, _ = to_device(w)
    out = alloc_output(w, fafb=True)
    with _plan([w], kernel=kernel, coef=coef) as p:
        p.compute(wu, out)
        torch.cuda.synchronize()
    r = oracle_lib.fstat(w)
    g = out.twoF.cpu().numpy().ravel().astype(np.float64)
    e = twoF_error(g, r["twoF"])
    _say(f"  max_e={e.max():.2e} mean 2F={r['twoF'].mean():.2f}")
    assert np.all(np.isfinite(g))
    assert e.max() <= tol, e.max()
    # every spindown is 0 here: the 9 spindown rows of a sky point are equal
    tw = out.twoF.cpu().numpy()
    assert np.array_equal(tw[:, :1, :].repeat(w.n_fd, axis=1), tw)


@pytest.mark.parametrize("coef,tol", [("f32", 1e-4), ("f16", 5e-3)])
def test_kappa_edges_batched(torch_cuda, oracle_lib, coef, tol):
    torch = torch_cuda
    ws = [kappa_edge_workload("zero"), kappa_edge_workload("one", seed=821)]
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w) for w in ws]
    with _plan(ws, coef=coef) as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
    for w, o in zip(ws, outs):
        e = twoF_error(o.twoF.cpu().numpy().ravel(), oracle_lib.fstat(w)["twoF"])
        _say(f"  batched {w.name} {coef}: max_e={e.max():.2e}")
        assert e.max() <= tol
