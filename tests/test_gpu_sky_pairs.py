"""Tiles of two sky points (single-unit interp kernel, 8 spindowns per
thread): the library pairs neighbouring sky points so that one staged
coefficient slice serves both.  The slice must hold both points' windows, so
a point with no partner near enough runs as a tile of its own, and a grid too
sparse for pairing keeps one sky point per tile.  Every case must be bit for
bit equal to the one-sky-point tiles of the batched path (same arithmetic per
template and SFT) and within the oracle's tolerance; fstat_last_tile reports
which shape ran."""
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


def _unit(seed, sky, n_f=300, f0=400.0):
    sky = np.asarray(sky, dtype=np.float64)
    return synth.make_workload(f"pairs-{seed}", seed=seed, n_det=2, slots_per_det=20, keep_frac=0.9, jitter=60.0,
                               t_sft=1800.0, f0=f0, n_f=n_f, n_sky=len(sky), n_fd=8, fdot_lo=-2e-9, fdot_hi=0.0,
                               dterms=8, injections=((1, 3, 100, 15.0),), sky_override=sky)


def _unit_vec(theta, phi):
    return [math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)]


# three tight pairs (0.01 rad apart) and one isolated point: 7 points, 4 sky tiles
CLUSTERED = [_unit_vec(0.7, 0.3), _unit_vec(0.71, 0.3), _unit_vec(1.9, 2.0), _unit_vec(1.9, 2.01),
             _unit_vec(2.6, -1.2), _unit_vec(2.61, -1.2), _unit_vec(1.3, -2.6)]
# four points about 1.9 rad apart: too sparse to pair
SPARSE = [_unit_vec(0.0, 0.0), _unit_vec(1.91, 0.0), _unit_vec(1.91, 2.094), _unit_vec(1.91, -2.094)]


def _run(torch, w):
    import paper_0904_1826_amd as P
    wu, _ = to_device(w)
    single, batched = alloc_output(w), alloc_output(w)
    with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                max_dterms=8) as p:
        p.compute(wu, single)
        torch.cuda.synchronize()
        shape = p.last_tile()
        p.batch_compute([wu], [batched])                 # one sky point per tile
        torch.cuda.synchronize()
    return single.twoF.cpu().numpy(), batched.twoF.cpu().numpy(), shape


@pytest.mark.parametrize("case", ["clustered", "sparse", "fibonacci200"])
def test_paired_tiles_match_single_sky_tiles_and_oracle(torch_cuda, oracle_lib, case):
    torch = torch_cuda
    if case == "clustered":
        w = _unit(901, CLUSTERED)
    elif case == "sparse":
        w = _unit(902, SPARSE)
    else:
        w = synth.make_workload("pairs-903", seed=903, n_det=2, slots_per_det=20, keep_frac=0.9, jitter=60.0,
                                t_sft=1800.0, f0=400.0, n_f=300, n_sky=200, n_fd=8, fdot_lo=-2e-9, fdot_hi=0.0,
                                dterms=8, injections=((17, 3, 100, 15.0),))
    a, b, shape = _run(torch, w)
    _say(f"  {case}: n_sky={w.n_sky} shape={shape}")
    if case == "clustered":
        assert shape["pair_seg"] > 0 and shape["sky_tiles"] == 4
    elif case == "sparse":
        assert shape["pair_seg"] == 0 and shape["sky_tiles"] == w.n_sky
    else:
        assert shape["pair_seg"] > 0 and w.n_sky // 2 <= shape["sky_tiles"] < 3 * w.n_sky // 4
    assert np.array_equal(a, b)
    r = oracle_lib.fstat(w)
    s, i, j = r["templates"]
    e = twoF_error(a[s, i, j], r["twoF"])
    _say(f"  {case}: max e vs oracle {e.max():.2e}")
    assert e.max() <= 1e-4


def test_paired_tiles_with_sft_blocks_and_outputs(torch_cuda, oracle_lib, tmp_path):
    """Pairs with the SFT loop split into launches (Fa, Fb carried between
    them) and Fa, Fb written out: equal to the batched path's."""
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
