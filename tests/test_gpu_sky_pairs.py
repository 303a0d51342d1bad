"""Tiles of two sky points (interp kernels, ranges of at most 8 spindowns
per thread, single-unit and batched): the library pairs neighbouring sky
points so that one staged coefficient slice serves both.  The slice must hold
both points' windows, so a point with no partner near enough runs as a tile
of its own, and a grid too sparse for pairing keeps one sky point per tile.
Every case must be bit for bit equal to one-sky-point tiles (the same work
unit cut to one sky point, which is never paired: same arithmetic per
template and SFT) and within the oracle's tolerance; fstat_last_tile reports
which shape the single-unit call ran."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import synth
from synth.device import to_device, alloc_output
from tests._helpers import twoF_error

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


def _unit(seed, sky, n_f=300, f0=400.0, n_fd=8):
    sky = np.asarray(sky, dtype=np.float64)
    return synth.make_workload(f"pairs-{seed}", seed=seed, n_det=2, slots_per_det=20, keep_frac=0.9, jitter=60.0,
                               t_sft=1800.0, f0=f0, n_f=n_f, n_sky=len(sky), n_fd=n_fd, fdot_lo=-2e-9, fdot_hi=0.0,
                               dterms=8, injections=((1, 3, 100, 15.0),), sky_override=sky)


def _unit_vec(theta, phi):
    return [math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)]


# three tight pairs (0.01 rad apart) and one isolated point: 7 points, 4 sky tiles
CLUSTERED = [_unit_vec(0.7, 0.3), _unit_vec(0.71, 0.3), _unit_vec(1.9, 2.0), _unit_vec(1.9, 2.01),
             _unit_vec(2.6, -1.2), _unit_vec(2.61, -1.2), _unit_vec(1.3, -2.6)]
# four points about 1.9 rad apart: too sparse to pair
SPARSE = [_unit_vec(0.0, 0.0), _unit_vec(1.91, 0.0), _unit_vec(1.91, 2.094), _unit_vec(1.91, -2.094)]
# both poles twice (longitude undefined, pair distance 0) and a close pair on the equator: 3 sky tiles
POLES = [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [0.0, 0.0, 1.0], _unit_vec(math.pi / 2, 0.4), [0.0, 0.0, -1.0],
         _unit_vec(math.pi / 2 + 0.01, 0.4)]


def _one_sky(wu, s):
    """The work unit cut to sky point s (its row of the antenna patterns)."""
    return dataclasses.replace(wu, sky=wu.sky[s:s + 1], a=wu.a[s:s + 1], b=wu.b[s:s + 1])


def _run(torch, w, skies, nfd_split=None):
    import paper_0904_1826_amd as P
    wu, _ = to_device(w)
    single, batched = alloc_output(w), alloc_output(w)
    one = alloc_output(dataclasses.replace(w, sky=w.sky[:1]))
    ref = {}
    with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                max_dterms=8) as p:
        p.compute(wu, single)
        torch.cuda.synchronize()
        shape = p.last_tile()
        p.batch_compute([wu], [batched])
        torch.cuda.synchronize()
        for s in skies:                                  # one sky point per tile
            p.compute(_one_sky(wu, s), one)
            torch.cuda.synchronize()
            assert p.last_tile()["pair_seg"] == 0
            ref[s] = one.twoF.cpu().numpy()[0].copy()
    return single.twoF.cpu().numpy(), batched.twoF.cpu().numpy(), shape, ref


@pytest.mark.parametrize("case", ["clustered", "sparse", "poles", "fibonacci200"])
def test_paired_tiles_match_single_sky_tiles_and_oracle(torch_cuda, oracle_lib, case):
    torch = torch_cuda
    if case == "clustered":
        w = _unit(901, CLUSTERED)
    elif case == "sparse":
        w = _unit(902, SPARSE)
    elif case == "poles":
        w = _unit(905, POLES)
    else:
        w = synth.make_workload("pairs-903", seed=903, n_det=2, slots_per_det=20, keep_frac=0.9, jitter=60.0,
                                t_sft=1800.0, f0=400.0, n_f=300, n_sky=200, n_fd=8, fdot_lo=-2e-9, fdot_hi=0.0,
                                dterms=8, injections=((17, 3, 100, 15.0),))
    skies = list(range(w.n_sky)) if w.n_sky < 10 else list(range(0, w.n_sky, 23)) + [w.n_sky - 1]
    a, b, shape, ref = _run(torch, w, skies)
    _say(f"  {case}: n_sky={w.n_sky} shape={shape}")
    if case == "clustered":
        assert shape["pair_seg"] > 0 and shape["sky_tiles"] == 4
    elif case == "sparse":
        assert shape["pair_seg"] == 0 and shape["sky_tiles"] == w.n_sky
    elif case == "poles":
        assert shape["pair_seg"] > 0 and shape["sky_tiles"] == 3
        assert np.array_equal(a[0], a[2]) and np.array_equal(a[1], a[4])     # a sky point paired with its copy
    else:
        assert shape["pair_seg"] > 0 and w.n_sky // 2 <= shape["sky_tiles"] < 3 * w.n_sky // 4
    assert np.array_equal(a, b)
    for s_, r1 in ref.items():
        assert np.array_equal(a[s_], r1), s_
    r = oracle_lib.fstat(w)
    s, i, j = r["templates"]
    e = twoF_error(a[s, i, j], r["twoF"])
    _say(f"  {case}: max e vs oracle {e.max():.2e}")
    assert e.max() <= 1e-4


def test_paired_tiles_with_sft_blocks_and_outputs(torch_cuda, oracle_lib, tmp_path):
    """Pairs with the SFT loop split into launches (Fa, Fb carried between
    them) and Fa, Fb written out: equal to the batched path's (one launch)."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    w = _unit(904, CLUSTERED, n_f=260)
    wu, _ = to_device(w)
    cache = tmp_path / "tiles.txt"
    cache.write_text("s0_d8_k0_c0 8 4 16 256\nbatch_s0_c0 8 256 256 256\n")      # 16 SFTs per launch
    outs = []
    for batched in (False, True):
        o = alloc_output(w, fafb=True)
        with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                    max_dterms=8) as p:
            p.autotune(wu, o, cache_path=str(cache))
            if batched:
                p.batch_compute([wu], [o])
            else:
                p.compute(wu, o)
                shape = p.last_tile()
            torch.cuda.synchronize()
        outs.append(o)
    _say(f"  shape {shape}")
    assert shape["pair_seg"] > 0 and shape["sblock"] == 16
    for name in ("twoF", "fa", "fb"):
        assert torch.equal(getattr(outs[0], name), getattr(outs[1], name)), name
    r = oracle_lib.fstat(w)
    s, i, j = r["templates"]
    assert twoF_error(outs[0].twoF.cpu().numpy()[s, i, j], r["twoF"]).max() <= 1e-4


def test_batch_mixes_paired_and_single_sky_tables(torch_cuda, oracle_lib):
    """One batch with units that pair (clustered and Fibonacci skies, spindown
    counts split into blocks of 16 and 4 to 8, of which the blocks of at most
    8 run paired) and a unit too sparse to pair: every unit bit for bit equal
    to its sky points computed one at a time, and within the oracle's
    tolerance."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = [_unit(911, CLUSTERED, n_f=270, n_fd=12),
          synth.make_workload("pairs-912", seed=912, n_det=2, slots_per_det=16, keep_frac=0.9, jitter=60.0,
                              t_sft=1800.0, f0=300.0, n_f=280, n_sky=60, n_fd=20, fdot_lo=-2e-9, fdot_hi=0.0,
                              dterms=8, injections=((5, 11, 90, 15.0),)),
          _unit(913, SPARSE, n_f=250),
          synth.make_workload("pairs-914", seed=914, n_det=2, slots_per_det=12, keep_frac=0.9, jitter=60.0,
                              t_sft=1800.0, f0=500.0, n_f=300, n_sky=40, n_fd=5, fdot_lo=-2e-9, fdot_hi=0.0,
                              dterms=8, injections=())]
    devs = [to_device(w)[0] for w in ws]
    outs = [alloc_output(w) for w in ws]
    mk = lambda: P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                        max_sky=max(w.n_sky for w in ws), max_fd=max(w.n_fd for w in ws),
                        max_f=max(w.n_f for w in ws), max_dterms=8)
    with mk() as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        for k, (w, wu) in enumerate(zip(ws, devs)):
            a = outs[k].twoF.cpu().numpy()
            one = alloc_output(dataclasses.replace(w, sky=w.sky[:1]))
            for s_ in sorted({0, 1, w.n_sky // 2, w.n_sky - 1}):
                p.compute(_one_sky(wu, s_), one)
                torch.cuda.synchronize()
                assert np.array_equal(a[s_], one.twoF.cpu().numpy()[0]), (k, s_)
            r = oracle_lib.fstat(w)
            s, i, j = r["templates"]
            e = twoF_error(a[s, i, j], r["twoF"])
            _say(f"  wu {k}: n_sky={w.n_sky} n_fd={w.n_fd} max e {e.max():.2e}")
            assert e.max() <= 1e-4


def test_pairing_follows_sky_vectors_changed_in_place(torch_cuda):
    """The host copies the sky vectors back on the geometry pass's wait and
    keeps the band order of the last grid it paired while the vectors are
    unchanged.  A grid changed in place between calls (the same device array,
    its points reversed) must be copied and paired afresh: the second call
    equals a fresh plan's bit for bit, with no tile dropped."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    w = _unit(906, CLUSTERED)
    wu, _ = to_device(w)
    a, b = alloc_output(w), alloc_output(w)
    mk = lambda: P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                        max_dterms=8)
    with mk() as p:
        p.compute(wu, a)
        torch.cuda.synchronize()
        before = a.twoF.clone()
        wu.sky.copy_(torch.flip(wu.sky, dims=[0]))
        p.compute(wu, a)
        torch.cuda.synchronize()
        assert p.last_tile()["pair_seg"] > 0
        p.compute(wu, a)                             # a dropped tile would be reported here
        torch.cuda.synchronize()
    with mk() as p:
        p.compute(wu, b)
        torch.cuda.synchronize()
    _say(f"  in-place sky change: max |2F| {float(a.twoF.abs().max()):.3g}")
    assert torch.isfinite(a.twoF).all()
    assert torch.equal(a.twoF, b.twoF)
    assert not torch.equal(a.twoF, before)
