"""The two many-work-unit cases at full size, in the batched launch
configuration, checked against the FP64 oracle on sampled outputs:

- 64 work units with U{200..2000} SFTs, U{900..7200}-bin bands,
  U{500..4000} sky points x U{4..16} spindowns, Dterms 8 or 16, one injected
  signal each (complex64 storage);
- 256 work units with 2 x U{1000..4000} SFTs, 14400-bin bands, 10000 sky
  points x 32 spindowns in total, Dterms 16, BF16 storage of device-drawn
  noise (arithmetic parity against the oracle run on the stored values)."""
import os
import sys
import time

import numpy as np
import pytest

import synth
from synth.device import to_device, alloc_output, draw_noise_16bit, host_values
from tests._helpers import twoF_error

pytestmark = pytest.mark.gpu
WORKERS = min(16, os.cpu_count() or 1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan_for(ws, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                  max_sky=max(w.n_sky for w in ws), max_fd=max(w.n_fd for w in ws), max_f=max(w.n_f for w in ws),
                  max_dterms=16, **kw)


def test_batch_64_work_units_full_size(torch_cuda, oracle_lib):
    torch = torch_cuda
    t0 = time.time()
    ws = synth.make_batch(3, workers=WORKERS)
    pairs = sum(w.n_templates * w.n_sft for w in ws)
    _say(f"64-unit batch: generated in {time.time() - t0:.1f} s, {pairs:.3e} template*SFT pairs")
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w) for w in ws]
    torch.cuda.synchronize()
    with _plan_for(ws) as p:
        p.batch_compute(devs, outs)                      # capture + first run
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.batch_compute(devs, outs)                      # graph replay
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    _say(f"  batched call {el * 1e3:.0f} ms -> {pairs / el:.3e} template*SFT/s")
    worst = 0.0
    for k, w in enumerate(ws):
        x = w.injections[0]
        j = np.unique(np.concatenate([np.arange(0, w.n_f, 16), [x.f_index]]))
        s_, i_, j_ = np.meshgrid([x.sky_index], np.arange(w.n_fd), j, indexing="ij")
        s_, i_, j_ = (a.ravel().astype(np.int32) for a in (s_, i_, j_))
        ref = oracle_lib.fstat(w, (s_, i_, j_))["twoF"]
        got = outs[k].twoF[x.sky_index].cpu().numpy()[i_, j_].astype(np.float64)
        e = twoF_error(got, ref)
        worst = max(worst, e.max())
        assert e.max() <= 1e-4, (k, e.max())
        assert outs[k].twoF[x.sky_index, x.fdot_index, x.f_index].item() > 0.4 * x.snr ** 2
    _say(f"  sampled max 2F error over 64 units: {worst:.2e}")
    # the units the persistent queues serve last (fewest SFTs) and units whose
    # spindowns split into blocks of several sizes (the tables after the
    # first): every template of their last sky point
    # (every spindown, every frequency including the ragged last tile)
    by_sft = sorted(range(len(ws)), key=lambda k: ws[k].n_sft)
    rem4 = [k for k in range(len(ws)) if 1 <= ws[k].n_fd % 8 <= 4 and ws[k].n_fd > 8][:3]
    for k in sorted(set(by_sft[:3] + rem4)):
        w = ws[k]
        s_, i_, j_ = oracle_lib.all_templates(w, [w.n_sky - 1])
        ref = oracle_lib.fstat(w, (s_, i_, j_))["twoF"]
        got = outs[k].twoF[w.n_sky - 1].cpu().numpy().ravel().astype(np.float64)
        e = twoF_error(got, ref)
        _say(f"  unit {k}: {w.n_sft} SFTs, {w.n_fd} spindowns, last sky point: max 2F error {e.max():.2e}")
        assert e.max() <= 1e-4, (k, e.max())
    # the FP16-coefficient form (outside the metric's 1e-4; its own bound) on the same inputs
    with _plan_for(ws, coef="f16") as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        el16 = time.perf_counter() - t0
    _say(f"  FP16 coefficients: batched call {el16 * 1e3:.0f} ms -> {pairs / el16:.3e} template*SFT/s "
         f"({el / el16:.2f}x the plain form)")
    worst = 0.0
    for k in range(0, 64, 9):
        w = ws[k]
        x = w.injections[0]
        j = np.arange(0, w.n_f, 16)
        s_, i_, j_ = np.meshgrid([x.sky_index], np.arange(w.n_fd), j, indexing="ij")
        s_, i_, j_ = (a.ravel().astype(np.int32) for a in (s_, i_, j_))
        ref = oracle_lib.fstat(w, (s_, i_, j_))["twoF"]
        got = outs[k].twoF[x.sky_index].cpu().numpy()[i_, j_].astype(np.float64)
        worst = max(worst, twoF_error(got, ref).max())
    _say(f"  FP16 coefficients: sampled max 2F error {worst:.2e}")
    assert worst <= 5e-3


def test_batch_256_work_units_bf16_full_size(torch_cuda, oracle_lib):
    torch = torch_cuda
    ws = synth.make_batch(4, workers=WORKERS)
    pairs = sum(w.n_templates * w.n_sft for w in ws)
    t0 = time.time()
    devs = [draw_noise_16bit(w, "bf16", seed=7000 + k) for k, w in enumerate(ws)]
    outs = [alloc_output(w) for w in ws]
    torch.cuda.synchronize()
    _say(f"256-unit BF16 batch: inputs drawn in {time.time() - t0:.1f} s, {pairs:.3e} template*SFT pairs, "
         f"{sum(d.sft.numel() * 2 for d in devs) / 1e9:.1f} GB of SFTs")
    with _plan_for(ws, storage="bf16") as p:
        t0 = time.perf_counter()
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    _say(f"  batched call {el:.1f} s -> {pairs / el:.3e} template*SFT/s")
    for k in (0, 101, 255):
        w = ws[k]
        vals = host_values(devs[k], "bf16")
        j = np.arange(0, w.n_f, 8)
        s_, i_, j_ = np.meshgrid([0], np.arange(w.n_fd), j, indexing="ij")
        s_, i_, j_ = (a.ravel().astype(np.int32) for a in (s_, i_, j_))
        ref = oracle_lib.fstat(w, (s_, i_, j_), sft=vals)["twoF"]
        got = outs[k].twoF[0].cpu().numpy()[i_, j_].astype(np.float64)
        e = twoF_error(got, ref)
        _say(f"  unit {k}: {w.n_sft} SFTs x {w.n_bins} bins, sampled max 2F error {e.max():.2e}")
        assert e.max() <= 1e-4, (k, e.max())
        del vals
    # the units served last (fewest SFTs): their last sky point, first and
    # last spindown, every frequency
    by_sft = sorted(range(len(ws)), key=lambda k: ws[k].n_sft)
    for k in by_sft[:2]:
        w = ws[k]
        vals = host_values(devs[k], "bf16")
        s_, i_, j_ = np.meshgrid([w.n_sky - 1], [0, w.n_fd - 1], np.arange(w.n_f), indexing="ij")
        s_, i_, j_ = (a.ravel().astype(np.int32) for a in (s_, i_, j_))
        ref = oracle_lib.fstat(w, (s_, i_, j_), sft=vals)["twoF"]
        got = outs[k].twoF[w.n_sky - 1].cpu().numpy()[i_, j_].astype(np.float64)
        e = twoF_error(got, ref)
        _say(f"  unit {k} (served last): {w.n_sft} SFTs, last sky point: max 2F error {e.max():.2e}")
        assert e.max() <= 1e-4, (k, e.max())
        del vals
    # BF16 storage with FP16 polynomial coefficients (outside the metric's 1e-4; its own bound)
    with _plan_for(ws, storage="bf16", coef="f16") as p:
        t0 = time.perf_counter()
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        el16 = time.perf_counter() - t0
    _say(f"  FP16 coefficients: batched call {el16:.1f} s -> {pairs / el16:.3e} template*SFT/s "
         f"({el / el16:.2f}x the BF16-storage form)")
    for k in (0, 255):
        w = ws[k]
        vals = host_values(devs[k], "bf16")
        j = np.arange(0, w.n_f, 8)
        s_, i_, j_ = np.meshgrid([0], np.arange(w.n_fd), j, indexing="ij")
        s_, i_, j_ = (a.ravel().astype(np.int32) for a in (s_, i_, j_))
        ref = oracle_lib.fstat(w, (s_, i_, j_), sft=vals)["twoF"]
        e = twoF_error(outs[k].twoF[0].cpu().numpy()[i_, j_].astype(np.float64), ref)
        _say(f"  FP16 coefficients, unit {k}: sampled max 2F error {e.max():.2e}")
        assert e.max() <= 5e-3, (k, e.max())
        del vals
