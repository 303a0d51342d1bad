"""Semi-coherent combination on the GPU (fstat_semicoherent): the sum over
time segments of each segment's coherent 2F, and the toplist of that sum,
against the FP64 oracle's sum; every output at small sizes (both kernels,
16-bit storage, FP16 coefficients, uneven segments), sampled outputs at the
size of the work-unit-shaped case split into 20 segments, and the argument
errors."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from synth.device import to_device, alloc_output, host_values
from tests._helpers import twoF_error, replace

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
                  max_dterms=max(max(w.dterms for w in ws), 16), **kw)


def _segments(n_seg=3, seed=71, **kw):
    p = dict(n_det=2, seg_slots=14, keep_frac=0.8, jitter=60.0, t_sft=1800.0, f0=400.0, n_f=300, n_sky=5, n_fd=3,
             fdot_lo=-2e-9, fdot_hi=0.0, dterms=8, injections=[(2, 1, 120, 6.0), (4, 2, 250, 5.0)])
    p.update(kw)
    return synth.make_segments(n_seg, seed=seed, **p)


@pytest.mark.parametrize("form", ["interp", "direct", "interp-coef16"])
def test_semicoherent_every_output(torch_cuda, form):
    segs = _segments()
    kernel, _, extra = form.partition("-")
    kw = dict(kernel=kernel, coef="f16" if extra == "coef16" else "f32")
    devs = [to_device(w)[0] for w in segs]
    out = alloc_output(segs[0])
    with _plan(segs, **kw) as p:
        p.semicoherent(devs, out)
        torch_cuda.cuda.synchronize()
        ms = p.last_kernel_ms()
    got = out.twoF.cpu().numpy().ravel().astype(np.float64)
    ref = oracle.semicoherent(segs)["twoF"]
    e = twoF_error(got, ref)
    tol = 5e-3 if extra == "coef16" else 1e-4
    _say(f"{form}: {len(segs)} segments of {[w.n_sft for w in segs]} SFTs, max 2F-sum error {e.max():.2e}, "
         f"demodulation {ms:.3f} ms")
    assert e.max() <= tol
    assert ms > 0
    # the injected templates stand out in the sum
    for x in segs[0].injections:
        o = (x.sky_index * segs[0].n_fd + x.fdot_index) * segs[0].n_f + x.f_index
        assert got[o] > 4 * len(segs) + 0.5 * len(segs) * x.snr ** 2


def test_semicoherent_uneven_segments_bf16(torch_cuda):
    """Segments of different length (22, 22 and 48 SFTs), BF16 storage:
    arithmetic parity against the oracle run on the stored values."""
    segs = _segments(2, 72)
    # a third, longer segment after the first two, on the same grid and t_ref
    segs.append(synth.make_workload("long", seed=73, n_det=2, slots_per_det=30, keep_frac=0.8, jitter=60.0,
                                    t_sft=1800.0, f0=400.0, n_f=300, n_sky=5, n_fd=3, fdot_lo=-2e-9, fdot_hi=0.0,
                                    dterms=8, epoch=synth.EPOCH + 28 * 1800.0, t_ref=synth.EPOCH))
    devs = [to_device(w, "bf16")[0] for w in segs]
    vals = [host_values(d, "bf16") for d in devs]
    out = alloc_output(segs[0])
    with _plan(segs, storage="bf16") as p:
        p.semicoherent(devs, out)
        torch_cuda.cuda.synchronize()
    got = out.twoF.cpu().numpy().ravel().astype(np.float64)
    ref = oracle.semicoherent(segs, sfts=vals)["twoF"]
    e = twoF_error(got, ref)
    _say(f"bf16, segments of {[w.n_sft for w in segs]} SFTs: max 2F-sum error {e.max():.2e}")
    assert e.max() <= 1e-4


def test_semicoherent_toplist(torch_cuda):
    import paper_0904_1826_amd as P
    segs = _segments(4, 74)
    devs = [to_device(w)[0] for w in segs]
    top_k, thr = 30, 24.0
    full = alloc_output(segs[0])
    both = alloc_output(segs[0], top_k=top_k, threshold=thr)
    with _plan(segs) as p:
        p.semicoherent(devs, full)
        p.semicoherent(devs, both)
        torch_cuda.cuda.synchronize()
    f = full.twoF.cpu().numpy().ravel()
    assert np.array_equal(both.twoF.cpu().numpy().ravel(), f)        # the sum is deterministic
    tf, s, i, j, n_above = P.toplist(both)
    # the selection of the GPU's own sum: identical indices, order and values
    idx, n = oracle.toplist(f.astype(np.float64), thr, top_k)
    got = (s.astype(np.int64) * segs[0].n_fd + i) * segs[0].n_f + j
    _say(f"toplist of the sum: n_above {n_above}, top {tf[:3]}")
    assert n_above == n and n > top_k
    assert np.array_equal(got, idx)
    assert np.array_equal(tf, f[idx])
    # against the oracle's sum: the same set except near the cut
    ref = oracle.semicoherent(segs)["twoF"]
    ridx, rn = oracle.toplist(ref, thr, top_k)
    cut = ref[ridx[-1]]
    differ = set(got.tolist()) ^ set(ridx.tolist())
    assert all(abs(ref[o] - cut) <= 1e-4 * max(cut, 4.0) * 4 for o in differ)
    assert abs(n_above - rn) <= 2


@pytest.mark.parametrize("fault", ["band", "singular"])
def test_semicoherent_segment_error_names_the_segment(torch_cuda, oracle_lib, fault):
    """Every segment is checked before any is demodulated: a middle segment
    whose stored band is one bin short of its lowest window (FSTAT_E_BAND),
    or whose antenna patterns make A B - C^2 vanish for a sky point (a = b:
    FSTAT_E_ARG), fails naming it, the output is left untouched, and the
    plan then sums the intact segments (against the oracle)."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    segs = _segments(3, 77, n_f=64, injections=[(2, 1, 30, 6.0)])
    w = segs[1]
    if fault == "band":
        k, _, _, _ = oracle_lib.bins(w, oracle_lib.all_templates(w))
        lo = int(k.min()) - w.dterms + 1
        bad1 = replace(w, sft=np.ascontiguousarray(w.sft[:, lo - w.k_first + 1:]), k_first=lo + 1)
        code = P.FSTAT_E_BAND
    else:
        b = w.b.copy()
        b[3] = w.a[3]
        bad1 = replace(w, b=b)
        code = P.FSTAT_E_ARG
    bad = [segs[0], bad1, segs[2]]
    out = alloc_output(segs[0])
    out.twoF.fill_(-1.0)
    with _plan(bad) as p:
        with pytest.raises(P.FstatError) as ei:
            p.semicoherent([to_device(x)[0] for x in bad], out)
        _say(f"  {p.last_error()}")
        assert ei.value.code == code and "segment 1" in p.last_error()
        torch.cuda.synchronize()
        assert bool((out.twoF == -1.0).all())           # nothing was demodulated
        p.semicoherent([to_device(x)[0] for x in segs], out)
        torch.cuda.synchronize()
        assert p.last_kernel_ms() > 0.0
    r = oracle_lib.semicoherent(segs)
    s_, i_, j_ = r["templates"]
    e = twoF_error(out.twoF.cpu().numpy()[s_, i_, j_], r["twoF"])
    _say(f"  intact segments after the error: max e {e.max():.2e}")
    assert e.max() <= 1e-4


def test_semicoherent_argument_errors(torch_cuda):
    import paper_0904_1826_amd as P
    segs = _segments(2, 75, n_f=64, n_sky=2, injections=[])
    devs = [to_device(w)[0] for w in segs]
    with _plan(segs) as p:
        with pytest.raises(P.FstatError) as ei:
            p.semicoherent([], alloc_output(segs[0]))
        assert ei.value.code == P.FSTAT_E_ARG
        with pytest.raises(P.FstatError) as ei:
            p.semicoherent(devs, alloc_output(segs[0], fafb=True))
        assert ei.value.code == P.FSTAT_E_UNSUPPORTED
        bad = synth.make_segments(1, seed=76, n_det=2, seg_slots=14, keep_frac=0.8, jitter=60.0, t_sft=1800.0,
                                  f0=400.5, n_f=64, n_sky=2, n_fd=3, fdot_lo=-2e-9, fdot_hi=0.0, dterms=8)
        with pytest.raises(P.FstatError) as ei:
            p.semicoherent(devs + [to_device(bad[0])[0]], alloc_output(segs[0]))
        assert ei.value.code == P.FSTAT_E_ARG and "segment 2" in p.last_error()
        out = alloc_output(segs[0], top_k=4, threshold=0.0, full=False)
        with pytest.raises(P.FstatError) as ei:
            p.semicoherent(devs, out)
        assert ei.value.code == P.FSTAT_E_ARG
        # still usable afterwards
        good = alloc_output(segs[0])
        p.semicoherent(devs, good)
        torch_cuda.cuda.synchronize()
        assert np.all(np.isfinite(good.twoF.cpu().numpy()))


@pytest.mark.parametrize("coef", ["f32", "f16"])
def test_semicoherent_full_size_20_segments(torch_cuda, coef):
    """The work-unit-shaped case split into 20 segments of about 100 SFTs
    (2000 sky points x 8 spindowns x 3600 frequencies, Dterms 8): sampled
    sums against the oracle, all spindowns and every 16th frequency at the
    injected sky points."""
    t0 = time.time()
    segs = synth.make_segment_config(20)
    pairs = segs[0].n_templates * sum(w.n_sft for w in segs)
    _say(f"{segs[0].name}: generated in {time.time() - t0:.1f} s, {pairs:.3e} template*SFT pairs")
    devs = [to_device(w)[0] for w in segs]
    out = alloc_output(segs[0])
    torch_cuda.cuda.synchronize()
    with _plan(segs, coef=coef) as p:
        p.semicoherent(devs, out)
        torch_cuda.cuda.synchronize()
        t0 = time.perf_counter()
        p.semicoherent(devs, out)
        torch_cuda.cuda.synchronize()
        el = time.perf_counter() - t0
        kms = p.last_kernel_ms()
    _say(f"  coef {coef}: {el * 1e3:.1f} ms per call ({kms:.1f} ms in demodulation kernels) -> "
         f"{pairs / el:.3e} template*SFT/s")
    w0 = segs[0]
    worst = 0.0
    for x in w0.injections:
        j = np.unique(np.concatenate([np.arange(0, w0.n_f, 16), [x.f_index]]))
        s_, i_, j_ = np.meshgrid([x.sky_index], np.arange(w0.n_fd), j, indexing="ij")
        s_, i_, j_ = (a.ravel().astype(np.int32) for a in (s_, i_, j_))
        ref = oracle.semicoherent(segs, (s_, i_, j_))["twoF"]
        got = out.twoF[x.sky_index].cpu().numpy()[i_, j_].astype(np.float64)
        worst = max(worst, twoF_error(got, ref).max())
        peak = out.twoF[x.sky_index, x.fdot_index, x.f_index].item()
        assert peak > 80 + 0.5 * 20 * x.snr ** 2, (x, peak)
    _say(f"  sampled max 2F-sum error {worst:.2e}")
    assert worst <= (5e-3 if coef == "f16" else 1e-4)


def test_semicoherent_from_device_detector_inputs(torch_cuda):
    """The whole chain on the device: each segment's detector positions,
    velocities and antenna patterns from fstat_detector_inputs (orbit model
    with the diurnal term), then the semi-coherent sum; against the oracle's
    detector inputs and the oracle's sum on them."""
    import math
    import synth.workloads as sw
    import paper_0904_1826_amd as P
    torch = torch_cuda
    earth = dict(t0=sw.EPOCH, orbit_radius=sw.ORBIT_R, orbit_rate=sw.ORBIT_OMEGA, orbit_phase=0.3,
                 obliquity=sw.OBLIQUITY, earth_radius=6378137.0 / 299792458.0, sidereal_rate=sw.SIDEREAL_OMEGA,
                 sidereal_phase=0.7)
    sites = [tuple(math.radians(x) for x in (lat, lon, az)) + (math.radians(az + 90.0),) for lat, lon, az in sw.SITES]
    segs = _segments(3, 77, injections=[])
    dev = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).cuda()
    segs2, segs_ref = [], []
    with P.Plan(max_sft=max(w.n_sft for w in segs), max_bins=max(w.n_bins for w in segs), max_sky=segs[0].n_sky,
                max_fd=segs[0].n_fd, max_f=segs[0].n_f) as p:
        for w in segs:
            t_mid = w.t_start + 0.5 * w.t_sft
            idx = np.zeros(w.n_sft, np.int32)
            idx[w.det_offset[1]:] = 1
            pos = torch.empty((w.n_sft, 3), dtype=torch.float64, device="cuda")
            vel = torch.empty_like(pos)
            a = torch.empty((w.n_sky, w.n_sft), dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            p.detector_inputs(earth, sites, dev(t_mid, np.float64), dev(idx, np.int32), dev(w.sky, np.float64),
                              pos, vel, a, b)
            torch.cuda.synchronize()
            segs2.append(replace(w, pos=pos.cpu().numpy(), vel=vel.cpu().numpy(), a=a.cpu().numpy(),
                                 b=b.cpu().numpy()))
            rp, rv, ra, rb = oracle.detector_inputs(earth, sites, t_mid, idx, w.sky)
            segs_ref.append(replace(w, pos=rp, vel=rv, a=ra.astype(np.float32), b=rb.astype(np.float32)))
        devs = [to_device(w)[0] for w in segs2]
        out = alloc_output(segs2[0])
        p.semicoherent(devs, out)
        torch.cuda.synchronize()
    got = out.twoF.cpu().numpy().ravel().astype(np.float64)
    e = twoF_error(got, oracle.semicoherent(segs2)["twoF"])
    e_ref = twoF_error(got, oracle.semicoherent(segs_ref)["twoF"])
    _say(f"device detector inputs + semi-coherent sum: max error {e.max():.2e} (oracle inputs: {e_ref.max():.2e})")
    assert e.max() <= 1e-4 and e_ref.max() <= 1e-4
