"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the
same seeded inputs.  Bin selection must match bit for bit; 2F must agree to
e = |2F_gpu - 2F_ref| / max(2F_ref, 4) <= 1e-4 (FP32 window sums)."""
import math
import sys

import numpy as np
import pytest

import synth
from synth.device import to_device, alloc_output
from tests._helpers import small_workload, replace, twoF_error, slice_edge_workload

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(w, storage="c64", kernel="auto", max_dterms=None, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                  max_dterms=max_dterms or max(w.dterms, 16), storage=storage, kernel=kernel, **kw)


def _run(torch, w, storage="c64", kernel="auto", fafb=True, tile=None):
    wu, deq = to_device(w, storage)
    out = alloc_output(w, fafb=fafb)
    with _plan(w, storage, kernel) as p:
        p.compute(wu, out)
        torch.cuda.synchronize()
    return out, deq


def _compare(oracle, w, out, templates=None, sft=None, tol=TOL):
    r = oracle.fstat(w, templates, sft=sft)
    s, i, j = r["templates"]
    gpu = out.twoF.cpu().numpy()[s, i, j].astype(np.float64)
    e = twoF_error(gpu, r["twoF"])
    _say(f"  templates={len(s)} max_e={e.max():.3e} rms_e={math.sqrt(np.mean(e * e)):.3e} "
         f"max2F_ref={r['twoF'].max():.2f}")
    assert np.all(np.isfinite(gpu))
    assert e.max() <= tol, (e.max(), int(np.argmax(e)))
    if out.fa is not None:
        fa = out.fa.cpu().numpy()[s, i, j]
        fa = fa[..., 0] + 1j * fa[..., 1]
        scale = np.sqrt(np.maximum(np.abs(r["Fa"]) ** 2 + np.abs(r["Fb"]) ** 2, 1.0 * len(w.t_start)))
        assert np.max(np.abs(fa - r["Fa"]) / scale) < 1e-4
    return e


def test_bins_bit_exact(torch_cuda, oracle_lib):
    torch = torch_cuda
    w = synth.make_config(1, slots_per_det=200, n_sky=64, injections=(), noise=False)
    _say(f"bins: n_sft={w.n_sft} n_bins={w.n_bins}")
    rng = np.random.default_rng(5)
    n = 20000
    ts = rng.integers(0, w.n_sky, n).astype(np.int32)
    ti = rng.integers(0, w.n_fd, n).astype(np.int32)
    tj = rng.integers(0, w.n_f, n).astype(np.int32)
    ta = rng.integers(0, w.n_sft, n).astype(np.int32)
    wu, _ = to_device(w)
    dev = lambda x: torch.from_numpy(x).cuda()
    k = torch.empty(n, dtype=torch.int64, device="cuda")
    kap = torch.empty(n, dtype=torch.float64, device="cuda")
    ph = torch.empty(n, dtype=torch.float64, device="cuda")
    with _plan(w) as p:
        p.bins(wu, dev(ts), dev(ti), dev(tj), dev(ta), k, kap, ph)
        torch.cuda.synchronize()
    k_ref, kap_ref, ph_ref, _ = oracle_lib.bins(w, (ts, ti, tj))
    k_ref = k_ref[np.arange(n), ta]
    kap_ref = kap_ref[np.arange(n), ta]
    ph_ref = ph_ref[np.arange(n), ta]
    assert np.array_equal(k.cpu().numpy(), k_ref)
    assert np.array_equal(kap.cpu().numpy().view(np.int64), kap_ref.view(np.int64))   # bit-identical
    d = np.abs(ph.cpu().numpy() - ph_ref)
    assert np.max(np.minimum(d, 1 - d)) < 1e-9


KERNELS = ["direct", "interp"]


@pytest.mark.parametrize("kernel", KERNELS)
def test_parity_config0(torch_cuda, oracle_lib, kernel):
    w = synth.make_config(0)
    _say(f"config0 {kernel}: {w.name} n_sft={w.n_sft} n_bins={w.n_bins} D={w.dterms}")
    out, _ = _run(torch_cuda, w, kernel=kernel)
    _compare(oracle_lib, w, out)
    # the injected template stands out
    assert out.twoF.cpu().numpy()[0, 0, 128] > 60


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dterms", [1, 3, 8, 16, 33, 64])
def test_parity_ragged_tiles(torch_cuda, oracle_lib, dterms, kernel):
    """Several frequency tiles with a ragged tail, an SFT count that is not a
    multiple of the LDS chunk, two detectors, several sky points and spindowns."""
    w = small_workload(100 + dterms, n_det=2, slots=23, keep=0.8, n_sky=3, n_fd=3, n_f=700, dterms=dterms,
                       injections=((1, 2, 333, 15.0),))
    _say(f"ragged {kernel} D={dterms}: n_sft={w.n_sft} n_bins={w.n_bins} templates={w.n_templates}")
    out, _ = _run(torch_cuda, w, kernel=kernel)
    _compare(oracle_lib, w, out)


@pytest.mark.parametrize("kernel", KERNELS)
def test_parity_four_detectors(torch_cuda, oracle_lib, kernel):
    """Four detectors (the two synthetic sites twice, each with its own SFT
    times and gaps), the largest detector count of the workloads, summed
    coherently: every template against the oracle; the detector offsets pass
    the library's check."""
    w = small_workload(150, n_det=4, slots=11, keep=0.8, n_sky=5, n_fd=3, n_f=300, dterms=8,
                       injections=((2, 1, 150, 15.0),))
    assert len(w.det_offset) == 5
    _say(f"four detectors {kernel}: n_sft={w.n_sft} offsets={[int(x) for x in w.det_offset]} templates={w.n_templates}")
    out, _ = _run(torch_cuda, w, kernel=kernel)
    _compare(oracle_lib, w, out)


INTERP_TILES = [(8, 4, 0, 256), (8, 4, 7, 256), (8, 3, 0, 256), (8, 2, 0, 256), (8, 3, 7, 256), (4, 3, 0, 256),
                (4, 2, 7, 256), (2, 3, 0, 256), (1, 3, 7, 256), (8, 3, 0, 64), (8, 2, 7, 64), (4, 3, 0, 64)]


@pytest.mark.parametrize("side", ["in", "out"])
@pytest.mark.parametrize("coef", ["f32", "f16"])
def test_slice_capacity_edge(torch_cuda, oracle_lib, coef, side):
    """Parity of every template where the slice bound is tightest, for the
    8-spindown blocks (16 spindowns as 8 + 8 with FP32 coefficients; 12 as
    8 + 4 with FP16 ones)."""
    torch = torch_cuda
    w = slice_edge_workload(coef, side)
    _say(f"slice edge {coef} {side}: n_sft={w.n_sft} n_bins={w.n_bins} dfdot={w.dfdot:.4e}")
    wu, _ = to_device(w)
    out = alloc_output(w)
    with _plan(w, kernel="interp", max_dterms=8, coef=coef) as p:
        p.compute(wu, out)
        torch.cuda.synchronize()
        shape = p.last_tile()
    # one range at 8 per thread (FP32: 16 spindowns as two 8-blocks), or 8 + 4
    assert shape["nf_reg"] == 8 and shape["pair_seg"] == 0
    assert shape["split"] == ({} if coef == "f32" else {8: 8, 4: 4}), shape
    _compare(oracle_lib, w, out, tol=TOL if coef == "f32" else 5e-3)


@pytest.mark.parametrize("tile", INTERP_TILES, ids=lambda t: "nf%d_w%d_sb%d_t%d" % t)
def test_interp_tile_variants(torch_cuda, oracle_lib, tile, tmp_path):
    """Every interp tile shape (spindowns per thread, waves per SIMD, SFTs
    per launch, work-group size), forced through the tile cache, on ragged
    frequency, spindown and SFT counts; a wide spindown range makes some
    windows fall outside the staged slice (global-memory path)."""
    torch = torch_cuda
    w = small_workload(300, n_det=2, slots=23, keep=0.85, n_sky=3, n_fd=9, n_f=700, dterms=8,
                       fdot_lo=-2.4e-6, injections=((1, 5, 333, 15.0),))
    cache = tmp_path / "tiles.txt"
    cache.write_text("s0_d8_k2_c0 %d %d %d %d\n" % tile)
    _say(f"tile {tile}: n_sft={w.n_sft} n_bins={w.n_bins} templates={w.n_templates}")
    wu, _ = to_device(w)
    out = alloc_output(w)
    with _plan(w, kernel="interp", max_dterms=8) as p:
        p.autotune(wu, out, cache_path=str(cache))
        p.compute(wu, out)
        torch.cuda.synchronize()
    _compare(oracle_lib, w, out)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("storage", ["bf16", "fp16"])
def test_parity_16bit_storage(torch_cuda, oracle_lib, storage, kernel):
    """Arithmetic parity against the oracle run on the exactly dequantised
    stored values (1e-4), and the storage error against complex64 input."""
    w = small_workload(200, n_det=2, slots=30, keep=0.9, n_sky=4, n_fd=2, n_f=600, dterms=8,
                       injections=((0, 1, 300, 20.0),))
    _say(f"16-bit {storage} {kernel}: n_sft={w.n_sft} n_bins={w.n_bins}")
    out, deq = _run(torch_cuda, w, storage, kernel=kernel)
    _compare(oracle_lib, w, out, sft=deq)
    ref = oracle_lib.fstat(w)
    e = twoF_error(out.twoF.cpu().numpy().ravel(), ref["twoF"])
    _say(f"  storage error vs complex64: max {e.max():.2e} rms {math.sqrt(np.mean(e * e)):.2e}")
    assert math.sqrt(np.mean(e * e)) < 5e-3


@pytest.mark.parametrize("kernel", KERNELS)
def test_parity_config1_sampled(torch_cuda, oracle_lib, kernel):
    """The work-unit-shaped case at full size, in the launch configuration the
    benchmark times; the oracle checks two whole sky points (8 x 3600
    templates each, all 2000 SFTs) and every injected template."""
    torch = torch_cuda
    w = synth.make_config(1)
    _say(f"config1 {kernel}: n_sft={w.n_sft} n_bins={w.n_bins} templates={w.n_templates}")
    out, _ = _run(torch, w, kernel=kernel, fafb=False)
    sk = [0, 1234]
    s, i, j = oracle_lib.all_templates(w, sk)
    inj = [(x.sky_index, x.fdot_index, x.f_index) for x in w.injections]
    s = np.concatenate([s, [x[0] for x in inj]]).astype(np.int32)
    i = np.concatenate([i, [x[1] for x in inj]]).astype(np.int32)
    j = np.concatenate([j, [x[2] for x in inj]]).astype(np.int32)
    _compare(oracle_lib, w, out, (s, i, j))
    tw = out.twoF.cpu().numpy()
    assert np.all(np.isfinite(tw))
    for (a, b, c), x in zip(inj, w.injections):
        assert tw[a, b, c] > 0.5 * x.snr ** 2


def test_band_error_on_gpu(torch_cuda, oracle_lib):
    import paper_0904_1826_amd as P
    w = small_workload(300, injections=())
    s, i, j = oracle_lib.all_templates(w)
    k, _, _, _ = oracle_lib.bins(w, (s, i, j))
    lo, hi = int(k.min()) - w.dterms + 1, int(k.max()) + w.dterms
    c0, c1 = lo - w.k_first, hi - w.k_first + 1
    tight = replace(w, sft=np.ascontiguousarray(w.sft[:, c0:c1]), k_first=lo)
    for kernel in KERNELS:
        out, _ = _run(torch_cuda, tight, kernel=kernel, fafb=False)     # exactly enough bins: accepted
        _compare(oracle_lib, tight, out)
    cut = replace(w, sft=np.ascontiguousarray(w.sft[:, c0 + 1:c1]), k_first=lo + 1)
    with pytest.raises(P.FstatError) as e:
        _run(torch_cuda, cut, fafb=False)
    assert e.value.code == P.FSTAT_E_BAND


@pytest.mark.parametrize("kernel", KERNELS)
def test_edge_single_frequency_two_sfts(torch_cuda, oracle_lib, kernel):
    w = small_workload(400, n_det=1, slots=2, keep=1.0, n_sky=1, n_fd=1, n_f=1, injections=())
    out, _ = _run(torch_cuda, w, kernel=kernel)
    _compare(oracle_lib, w, out)


def test_singular_antenna_matrix_is_an_error(torch_cuda):
    import paper_0904_1826_amd as P
    w = small_workload(401, n_det=1, slots=1, keep=1.0, n_sky=1, n_fd=1, n_f=4, injections=())
    with pytest.raises(P.FstatError) as e:
        _run(torch_cuda, w, fafb=False)
    assert e.value.code == P.FSTAT_E_ARG
