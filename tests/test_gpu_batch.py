"""Batched form: many work units with uneven SFT counts, bands, grids and
Dterms in one persistent launch (replayed from a captured hipGraph), checked
against single-work-unit calls and against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import synth
from synth.device import to_device, alloc_output
from tests._helpers import small_workload, replace, twoF_error, slice_edge_workload, sft_block_workloads

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


def _plan_for(ws, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                  max_sky=max(w.n_sky for w in ws), max_fd=max(w.n_fd for w in ws), max_f=max(w.n_f for w in ws),
                  max_dterms=max(max(w.dterms for w in ws), 16), **kw)


def _batch(torch, ws, storage="c64", **kw):
    devs = [to_device(w, storage) for w in ws]
    outs = [alloc_output(w) for w in ws]
    with _plan_for(ws, storage=storage, **kw) as p:
        p.batch_compute([d[0] for d in devs], outs)
        torch.cuda.synchronize()
    return outs, devs


def test_batch_matches_single_and_oracle(torch_cuda, oracle_lib):
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=6, scale=0.1)
    _say("batch shapes:", [(w.n_sft, w.n_bins, w.n_sky, w.n_fd, w.n_f, w.dterms) for w in ws])
    outs, devs = _batch(torch, ws)
    for k, w in enumerate(ws):
        single = alloc_output(w)
        with _plan_for([w]) as p:
            p.compute(devs[k][0], single)
            torch.cuda.synchronize()
        a = outs[k].twoF.cpu().numpy()
        b = single.twoF.cpu().numpy()
        assert np.array_equal(a, b), (k, np.max(np.abs(a - b)))
        s, i, j = oracle_lib.all_templates(w, [0, w.n_sky - 1])
        ref = oracle_lib.fstat(w, (s, i, j))["twoF"]
        e = twoF_error(a[s, i, j], ref)
        _say(f"  wu {k}: D={w.dterms} n_fd={w.n_fd} max_e={e.max():.2e}")
        assert e.max() <= 1e-4


@pytest.mark.parametrize("coef", ["f32", "f16"])
def test_batch_spindown_ranges(torch_cuda, oracle_lib, coef):
    """Spindown counts with every remainder modulo 8 and the splits they take
    in the batched tables (blocks of 4 to 8 per thread with FP32
    coefficients, and 16 where its slice fits, e.g. 9 = 5 + 4, 12 = 6 + 6,
    20 = 16 + 4, 33 = 16 + 16 + 1 in a block of 4; blocks of 8
    and 4 with FP16 ones, partial blocks included); every template against
    the oracle and against the single-unit call."""
    torch = torch_cuda
    n_fds = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 20, 21, 23, 30, 32, 33, 49, 50]
    ws = [small_workload(300 + k, n_sky=3, n_fd=nfd, n_f=300, slots=12, fdot_lo=-1e-9, injections=())
          for k, nfd in enumerate(n_fds)]
    outs, devs = _batch(torch, ws, coef=coef)
    tol = 5e-3 if coef == "f16" else 1e-4
    for k, w in enumerate(ws):
        a = outs[k].twoF.cpu().numpy()
        ref = oracle_lib.fstat(w)["twoF"].reshape(a.shape)
        e = twoF_error(a, ref)
        single = alloc_output(w)
        with _plan_for([w], coef=coef) as p:
            p.compute(devs[k][0], single)
            torch.cuda.synchronize()
        b = single.twoF.cpu().numpy()
        d = np.max(np.abs(a - b) / np.maximum(np.abs(b), 4.0))
        _say(f"  n_fd={w.n_fd}: max e vs oracle {e.max():.2e}, vs single call {d:.1e}")
        assert e.max() <= tol, (w.n_fd, e.max())
        assert d <= 1e-6, (w.n_fd, d)


def test_batch_graph_replay_follows_new_contents(torch_cuda, oracle_lib):
    """The second call replays the captured graph; the work-unit table lives in
    device memory, so new data (and new buffers) of the same shapes are used."""
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=4, scale=0.06, seed=77)
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w) for w in ws]
    with _plan_for(ws) as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        first = [o.twoF.clone() for o in outs]
        p.batch_compute(devs, outs)                  # replay, same inputs
        torch.cuda.synchronize()
        for a, b in zip(first, outs):
            assert torch.equal(a, b.twoF)
        for d in devs:
            d.sft.mul_(2.0)                            # 2F scales by 4 exactly (powers of two)
        outs2 = [alloc_output(w) for w in ws]          # new output buffers
        p.batch_compute(devs, outs2)
        torch.cuda.synchronize()
        for a, b in zip(first, outs2):
            assert torch.allclose(b.twoF, 4.0 * a, rtol=1e-6, atol=1e-5)
        for d in devs:
            d.sft.mul_(0.5)
        # different shapes: a new graph
        ws2 = ws[:3]
        outs3 = [alloc_output(w) for w in ws2]
        p.batch_compute(devs[:3], outs3)
        torch.cuda.synchronize()
        for a, b in zip(first[:3], outs3):
            assert torch.equal(a, b.twoF)


def test_batch_without_graph_is_identical(torch_cuda):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=3, scale=0.05, seed=5)
    a, _ = _batch(torch, ws)
    b, _ = _batch(torch, ws, flags=P.FSTAT_FLAG_NO_GRAPH)
    for x, y in zip(a, b):
        assert torch.equal(x.twoF, y.twoF)


def test_batch_band_error_names_the_work_unit(torch_cuda, oracle_lib):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=3, scale=0.05, seed=9)
    w = ws[1]
    s, i, j = oracle_lib.all_templates(w)
    k, _, _, _ = oracle_lib.bins(w, (s, i, j))
    lo = int(k.min()) - w.dterms + 2                   # one bin short at the bottom
    c0 = lo - w.k_first
    ws[1] = replace(w, sft=np.ascontiguousarray(w.sft[:, c0:]), k_first=lo)
    outs = [alloc_output(x) for x in ws]
    for o in outs:
        o.twoF.fill_(-7.0)
    with _plan_for(ws) as p:
        with pytest.raises(P.FstatError) as e:
            p.batch_compute([to_device(x)[0] for x in ws], outs)
        assert e.value.code == P.FSTAT_E_BAND
        assert "work unit 1" in str(e.value)
    torch.cuda.synchronize()
    for o in outs:                                    # nothing was demodulated
        assert bool((o.twoF == -7.0).all())


def test_batch_groups_under_a_small_scratch_budget(torch_cuda, monkeypatch):
    """With a tiny scratch budget every work unit forms its own group (its own
    table slice and graph); results are unchanged."""
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=4, scale=0.05, seed=11)
    a, _ = _batch(torch, ws)
    monkeypatch.setenv("FSTAT_BATCH_SCRATCH_GB", "0.000001")
    b, _ = _batch(torch, ws)
    for x, y in zip(a, b):
        assert torch.equal(x.twoF, y.twoF)


@pytest.mark.parametrize("storage", ["bf16", "fp16"])
def test_batch_16bit_storage(torch_cuda, oracle_lib, storage):
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=3, scale=0.06, seed=13)
    outs, devs = _batch(torch, ws, storage=storage)
    for k, w in enumerate(ws):
        s, i, j = oracle_lib.all_templates(w, [0])
        ref = oracle_lib.fstat(w, (s, i, j), sft=devs[k][1])["twoF"]
        e = twoF_error(outs[k].twoF.cpu().numpy()[s, i, j], ref)
        assert e.max() <= 1e-4, (k, e.max())


@pytest.mark.parametrize("mix", ["in", "in+out"])
@pytest.mark.parametrize("coef", ["f32", "f16"])
def test_batch_slice_capacity_edge(torch_cuda, oracle_lib, coef, mix):
    """Work units whose slice bound sits just inside the LDS slice's capacity
    (a batch of them runs the kernel without the global-memory path) or just
    beyond it (a batch holding one runs the kernel with that path, and the
    entries that fit take the LDS path in it); every template against the
    oracle."""
    torch = torch_cuda
    ws = [slice_edge_workload(coef, side) for side in mix.split("+")]
    _say(f"batch slice edge {coef} {mix}:", [(w.n_sft, w.n_bins, w.dfdot) for w in ws])
    outs, _ = _batch(torch, ws, coef=coef)
    for k, w in enumerate(ws):
        r = oracle_lib.fstat(w)
        s, i, j = r["templates"]
        e = twoF_error(outs[k].twoF.cpu().numpy()[s, i, j], r["twoF"])
        _say(f"  wu {k}: max_e={e.max():.2e}")
        assert e.max() <= (1e-4 if coef == "f32" else 5e-3)


@pytest.mark.parametrize("coef", ["f32", "f16"])
def test_batch_sft_blocks(torch_cuda, oracle_lib, coef):
    """Units of about 1100, 600 and 300 SFTs: the batched SFT loop runs in
    launches of 256 SFTs, Fa and Fb carried between them, and each launch
    serves only the units with SFTs left.  Every template against the oracle,
    and bit for bit against single-unit calls (the carried sums are exact
    FP32 values, so the split changes no rounding)."""
    torch = torch_cuda
    ws = sft_block_workloads()
    _say("sft blocks:", [w.n_sft for w in ws])
    assert ws[0].n_sft > 1024 and 512 < ws[1].n_sft <= 1024 and ws[2].n_sft <= 512
    outs, devs = _batch(torch, ws, coef=coef)
    for k, w in enumerate(ws):
        single = alloc_output(w)
        with _plan_for([w], coef=coef) as p:
            p.compute(devs[k][0], single)
            torch.cuda.synchronize()
        a = outs[k].twoF.cpu().numpy()
        assert np.array_equal(a, single.twoF.cpu().numpy()), k
        r = oracle_lib.fstat(w)
        s, i, j = r["templates"]
        e = twoF_error(a[s, i, j], r["twoF"])
        _say(f"  wu {k}: n_sft={w.n_sft} max_e={e.max():.2e}")
        assert e.max() <= (1e-4 if coef == "f32" else 5e-3)


def test_batch_sft_blocks_toplists(torch_cuda):
    """Toplists of units that span 3, 2 and 1 SFT blocks: candidates are
    taken in each unit's last block only, and equal the single-unit calls'."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = sft_block_workloads()
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w, top_k=30, threshold=8.0, full=False) for w in ws]
    with _plan_for(ws) as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
    for k, w in enumerate(ws):
        single = alloc_output(w, top_k=30, threshold=8.0, full=False)
        with _plan_for([w]) as p:
            p.compute(devs[k], single)
            torch.cuda.synchronize()
        a, b = P.toplist(outs[k]), P.toplist(single)
        _say(f"  wu {k}: n_sft={w.n_sft} n_above {a[4]} / {b[4]}")
        assert a[4] == b[4] > 30
        for x, y in zip(a[:4], b[:4]):
            assert np.array_equal(x, y)


BATCH_TILES = [("c0", "4 64 256 256"), ("c0", "8 1 100 256"), ("c1", "4 1024 1024 256"), ("c1", "8 7 384 256")]


@pytest.mark.parametrize("cls,shape", BATCH_TILES, ids=[f"{c}-{s.replace(' ', '_')}" for c, s in BATCH_TILES])
def test_batch_tile_from_the_autotune_cache(torch_cuda, oracle_lib, tmp_path, cls, shape):
    """Batched launch shapes forced through the autotune cache (spindowns in
    blocks of 4 only, or split by lane cost into blocks of 16 and 4 to 8 (8
    and 4 with FP16 coefficients), tiles per chunk of the
    per-XCD queues, SFTs per launch): every unit bit for bit equal to its
    single-unit call with the default tile, and every template within the
    oracle's tolerance."""
    torch = torch_cuda
    coef = "f16" if cls == "c1" else "f32"
    ws = sft_block_workloads() + [small_workload(720 + k, n_sky=3, n_fd=nfd, n_f=290, slots=40, fdot_lo=-1e-9,
                                                 injections=()) for k, nfd in enumerate([3, 12, 13])]
    cache = tmp_path / "tiles.txt"
    # the single-unit class of the first unit keeps its default tile; the
    # batch class gets the forced shape
    c16 = 1 if coef == "f16" else 0
    cache.write_text(f"s0_d8_k0_c{c16} 8 {5 if c16 else 4} 512 256\nbatch_s0_{cls} {shape}\n")
    devs = [to_device(w) for w in ws]
    outs = [alloc_output(w) for w in ws]
    with _plan_for(ws, coef=coef) as p:
        p.autotune(devs[0][0], outs[0], cache_path=str(cache))
        p.batch_compute([d[0] for d in devs], outs)
        torch.cuda.synchronize()
    tol = 1e-4 if coef == "f32" else 5e-3
    for k, w in enumerate(ws):
        single = alloc_output(w)
        with _plan_for([w], coef=coef) as p:
            p.compute(devs[k][0], single)
            torch.cuda.synchronize()
        a = outs[k].twoF.cpu().numpy()
        assert np.array_equal(a, single.twoF.cpu().numpy()), k
        r = oracle_lib.fstat(w)
        s, i, j = r["templates"]
        e = twoF_error(a[s, i, j], r["twoF"])
        _say(f"  {shape} wu {k}: n_sft={w.n_sft} n_fd={w.n_fd} max_e={e.max():.2e}")
        assert e.max() <= tol


def test_batch_autotune_writes_both_classes(torch_cuda, oracle_lib, tmp_path):
    """fstat_autotune on one unit tunes the single-unit tile and the batched
    launch shape and appends both to the cache; a batch then runs with the
    tuned shape and matches the oracle."""
    torch = torch_cuda
    ws = sft_block_workloads()[1:]
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w) for w in ws]
    cache = tmp_path / "tiles.txt"
    with _plan_for(ws) as p:
        p.autotune(devs[0], outs[0], cache_path=str(cache))
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
    lines = [l.split() for l in cache.read_text().splitlines()]
    assert [l[0] for l in lines] == ["s0_d8_k0_c0", "batch_s0_c0"] and all(len(l) == 5 for l in lines)
    _say("tuned:", lines)
    for w, o in zip(ws, outs):
        e = twoF_error(o.twoF.cpu().numpy().ravel(), oracle_lib.fstat(w)["twoF"])
        assert e.max() <= 1e-4
