"""Runtime behaviour of the library on the GPU: forced allocation and launch
failures (from the host, through FSTAT_FAULT), plan reuse after errors,
the autotuner and its on-disk cache, and non-default streams."""
import numpy as np
import pytest

import synth
from synth.device import to_device, alloc_output
from tests._helpers import small_workload, twoF_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(w, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                  max_dterms=16, **kw)


@pytest.fixture(scope="module")
def wl():
    return small_workload(600, n_det=2, slots=20, keep=0.9, n_sky=3, n_fd=4, n_f=400, dterms=8,
                          injections=((1, 2, 100, 15.0),))


@pytest.mark.parametrize("kernel,nth", [("interp", 1), ("interp", 2), ("interp", 3), ("interp", 4), ("direct", 1),
                                        ("direct", 2)])
def test_injected_allocation_failure_then_recovery(torch_cuda, oracle_lib, wl, monkeypatch, kernel, nth):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    monkeypatch.setenv("FSTAT_FAULT", f"malloc:{nth}")
    wu, _ = to_device(wl)
    out = alloc_output(wl)
    with _plan(wl, kernel=kernel) as p:
        with pytest.raises(P.FstatError) as e:
            p.compute(wu, out)
        assert e.value.code == P.FSTAT_E_NOMEM
        assert "injected" in p.last_error()
        p.compute(wu, out)                                  # the plan is still usable
        torch.cuda.synchronize()
        assert p.last_error() == ""
    ref = oracle_lib.fstat(wl)["twoF"]
    assert twoF_error(out.twoF.cpu().numpy().ravel(), ref).max() <= 1e-4


@pytest.mark.parametrize("nth", [1, 2, 3])
def test_injected_launch_failure_then_recovery(torch_cuda, wl, monkeypatch, nth):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    monkeypatch.setenv("FSTAT_FAULT", f"launch:{nth}")
    wu, _ = to_device(wl)
    out = alloc_output(wl)
    with _plan(wl) as p:
        with pytest.raises(P.FstatError) as e:
            p.compute(wu, out)
        assert e.value.code == P.FSTAT_E_DEVICE
        p.compute(wu, out)
        torch.cuda.synchronize()


def test_injected_failure_in_batch(torch_cuda, monkeypatch):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=3, scale=0.05, seed=21)
    monkeypatch.setenv("FSTAT_FAULT", "malloc:1")
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w) for w in ws]
    with P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                max_sky=max(w.n_sky for w in ws), max_fd=16, max_f=max(w.n_f for w in ws), max_dterms=16) as p:
        with pytest.raises(P.FstatError) as e:
            p.batch_compute(devs, outs)
        assert e.value.code == P.FSTAT_E_NOMEM
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()


def test_host_side_argument_errors(torch_cuda, wl):
    import paper_0904_1826_amd as P
    wu, _ = to_device(wl)
    out = alloc_output(wl)
    with _plan(wl) as p:
        import dataclasses
        n = wl.n_sft
        bad = [dict(dterms=0), dict(dterms=17), dict(a=None), dict(t_start=None), dict(f0=-1.0), dict(df=0.0),
               dict(t_sft=float("nan")), dict(n_f=wl.n_f + 1), dict(det_offset=np.array([1, 5, n])),
               dict(det_offset=np.array([0, 5, n - 1])), dict(det_offset=np.array([0, n + 2, n]))]
        for kw in bad:
            w2 = dataclasses.replace(wu, **kw)
            o2 = alloc_output(dataclasses.replace(wl, n_f=w2.n_f))      # outputs sized for the unit
            with pytest.raises(P.FstatError) as e:
                p.compute(w2, o2)
            assert e.value.code in (P.FSTAT_E_ARG, P.FSTAT_E_SIZE), kw
        for off in ([0, n // 2, n], [0, n, n], [0, 0, n]):      # consistent detector blocks are accepted
            p.compute(dataclasses.replace(wu, det_offset=np.array(off)), out)
        torch_sync = __import__("torch").cuda.synchronize
        torch_sync()
        # arrays that do not match the unit's sizes are refused by the binding
        with pytest.raises(ValueError, match="elements"):
            p.compute(dataclasses.replace(wu, n_f=wl.n_f - 1), out)
        with pytest.raises(P.FstatError):
            p.compute(wu, P.Output(twoF=None))


def test_autotune_and_cache(torch_cuda, oracle_lib, wl, tmp_path):
    torch = torch_cuda
    cache = str(tmp_path / "tiles.txt")
    wu, _ = to_device(wl)
    out = alloc_output(wl)
    with _plan(wl) as p:
        p.autotune(wu, out, cache_path=cache)
        p.compute(wu, out)
        torch.cuda.synchronize()
    lines = [l.split() for l in open(cache).read().splitlines()]
    # one line for the single-unit class, one for the plan's batch class
    assert len(lines) == 2 and all(len(l) == 5 for l in lines)
    assert lines[0][0].startswith("s0_d8_k") and lines[1][0] == "batch_s0_c0"
    ref = oracle_lib.fstat(wl)["twoF"]
    assert twoF_error(out.twoF.cpu().numpy().ravel(), ref).max() <= 1e-4
    # a cache entry chosen by hand is taken as is: one spindown per thread and
    # the SFT loop split into launches of 5 SFTs (running sums in between)
    key = lines[0][0]
    with open(cache, "w") as f:
        f.write(f"{key} 1 3 5 256\n{' '.join(lines[1])}\n")
    out2 = alloc_output(wl)
    with _plan(wl) as p:
        p.autotune(wu, out2, cache_path=cache)
        p.compute(wu, out2)
        torch.cuda.synchronize()
    assert twoF_error(out2.twoF.cpu().numpy().ravel(), ref).max() <= 1e-4


def test_non_default_stream(torch_cuda, oracle_lib, wl):
    torch = torch_cuda
    wu, _ = to_device(wl)
    out = alloc_output(wl)
    s = torch.cuda.Stream()
    with _plan(wl) as p:
        with torch.cuda.stream(s):
            p.compute(wu, out, stream=s)
        s.synchronize()
        assert p.last_kernel_ms() > 0
    ref = oracle_lib.fstat(wl)["twoF"]
    assert twoF_error(out.twoF.cpu().numpy().ravel(), ref).max() <= 1e-4


def test_forced_narrow_slice_is_reported_not_silent(torch_cuda, wl, monkeypatch):
    """With the slice forced narrower than the tile's windows (fault injection
    from the host: the variant without the global-memory path at 64 bins),
    every tile meets SFTs it cannot evaluate: its outputs are NaN, never a
    2F with terms missing, and the next call on the plan returns
    FSTAT_E_DEVICE saying so; the call after that runs (and drops) again."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    monkeypatch.setenv("FSTAT_FAULT", "narrow:64")
    wu, _ = to_device(wl)
    out = alloc_output(wl)
    with _plan(wl, kernel="interp") as p:
        p.compute(wu, out)
        torch.cuda.synchronize()
        assert np.all(np.isnan(out.twoF.cpu().numpy()))      # both frequency tiles span > 64 bins
        with pytest.raises(P.FstatError) as e:
            p.compute(wu, out)
        assert e.value.code == P.FSTAT_E_DEVICE and "outside the LDS slice" in p.last_error()
        p.compute(wu, out)                                  # runs (and drops) again
        torch.cuda.synchronize()


def test_forced_narrow_slice_in_batch(torch_cuda, monkeypatch):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=3, scale=0.05, seed=22)
    devs = [to_device(w)[0] for w in ws]
    ref = [alloc_output(w) for w in ws]
    outs = [alloc_output(w) for w in ws]
    mk = lambda: P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                        max_sky=max(w.n_sky for w in ws), max_fd=16, max_f=max(w.n_f for w in ws), max_dterms=16)
    with mk() as p:
        p.batch_compute(devs, ref)
    monkeypatch.setenv("FSTAT_FAULT", "narrow:64")
    with mk() as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            # tiles of up to 64 frequencies fit the narrow slice and are
            # evaluated as usual; every other output is NaN
            a, b = o.twoF.cpu().numpy(), r.twoF.cpu().numpy()
            assert np.all(np.isnan(a) | (a == b)) and np.isnan(a).mean() > 0.5
        with pytest.raises(P.FstatError) as e:
            p.batch_compute(devs, outs)
        assert e.value.code == P.FSTAT_E_DEVICE and "work unit" in p.last_error()
