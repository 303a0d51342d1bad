"""Detector inputs computed on the device (fstat_detector_inputs) against the
FP64 oracle's, at the work-unit shape, plus edge cases, and end to end: a
work unit whose positions, velocities and antenna patterns come from the
device gives the oracle's 2F on those inputs."""
import math
import sys
import time

import numpy as np
import pytest

import oracle
import synth
import synth.workloads as sw
from synth.device import to_device, alloc_output
from tests._helpers import small_workload, replace, twoF_error

pytestmark = pytest.mark.gpu

EARTH = dict(t0=sw.EPOCH, orbit_radius=sw.ORBIT_R, orbit_rate=sw.ORBIT_OMEGA, orbit_phase=0.3,
             obliquity=sw.OBLIQUITY, earth_radius=6378137.0 / 299792458.0, sidereal_rate=sw.SIDEREAL_OMEGA,
             sidereal_phase=0.7)
SITES = [tuple(math.radians(x) for x in (lat, lon, az)) + (math.radians(az + 90.0),) for lat, lon, az in sw.SITES]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan():
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=4, max_bins=64, max_sky=1, max_fd=1, max_f=1)


def _device(torch, earth, t_mid, site_of_sft, sky, sites=SITES):
    n_sft, n_sky = len(t_mid), len(sky)
    dev = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).cuda()
    t, idx, n = dev(t_mid, np.float64), dev(site_of_sft, np.int32), dev(sky, np.float64)
    pos = torch.empty((n_sft, 3), dtype=torch.float64, device="cuda")
    vel = torch.empty_like(pos)
    a = torch.empty((n_sky, n_sft), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    with _plan() as p:
        p.detector_inputs(earth, sites, t, idx, n, pos, vel, a, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.detector_inputs(earth, sites, t, idx, n, pos, vel, a, b)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    return pos.cpu().numpy(), vel.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy(), el


def test_detector_inputs_work_unit_shape(torch_cuda):
    """2 sites x 1000 SFTs over a year, 2000 sky points, with the diurnal term."""
    rng = np.random.default_rng(4)
    t = np.sort(sw.EPOCH + rng.uniform(0, 3.0e7, 2000))
    idx = np.repeat([0, 1], 1000).astype(np.int32)
    sky = sw.sky_grid(2000)
    pos, vel, a, b, el = _device(torch_cuda, EARTH, t, idx, sky)
    rp, rv, ra, rb = oracle.detector_inputs(EARTH, SITES, t, idx, sky)
    _say(f"detector inputs for 2000 SFTs x 2000 sky points: {el * 1e3:.3f} ms")
    assert np.max(np.abs(pos - rp)) < 1e-11                 # light-s, |r| ~ 500
    assert np.max(np.abs(vel - rv)) < 1e-17                 # units of c, |v| ~ 1e-4
    assert np.max(np.abs(a - ra)) < 3e-7 and np.max(np.abs(b - rb)) < 3e-7   # FP32 outputs


def test_detector_inputs_edges(torch_cuda):
    """Poles and the equator, a site index out of range (NaN for that SFT)."""
    sky = np.array([[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [0, 1.0, 0]])
    t = sw.EPOCH + np.array([0.0, 1000.0, 5e6])
    idx = np.array([0, 1, 0], np.int32)
    pos, vel, a, b, _ = _device(torch_cuda, EARTH, t, idx, sky)
    rp, rv, ra, rb = oracle.detector_inputs(EARTH, SITES, t, idx, sky)
    assert np.max(np.abs(a - ra)) < 3e-7 and np.max(np.abs(b - rb)) < 3e-7
    pos, vel, a, b, _ = _device(torch_cuda, EARTH, t, np.array([0, 5, 1], np.int32), sky)
    assert np.all(np.isnan(pos[1])) and np.all(np.isnan(a[:, 1])) and np.all(np.isfinite(a[:, [0, 2]]))


def test_work_unit_from_device_detector_inputs(torch_cuda):
    """A work unit whose r, v, a, b come from the device: 2F matches the
    oracle run on those inputs, and (without the diurnal term, the
    generator's model) the generator's own work unit."""
    torch = torch_cuda
    import paper_0904_1826_amd as P
    w = small_workload(990, n_det=2, slots=30, keep=0.9, n_sky=4, n_fd=3, n_f=400, dterms=8,
                       injections=((2, 1, 200, 15.0),))
    t_mid = w.t_start + 0.5 * w.t_sft
    # detector of each SFT: the generator fills detector blocks in order
    idx = np.zeros(w.n_sft, np.int32)
    idx[w.det_offset[1]:] = 1
    e0 = dict(EARTH, earth_radius=0.0, sidereal_phase=0.0)
    pos, vel, a, b, _ = _device(torch, e0, t_mid, idx, w.sky)
    w2 = replace(w, pos=pos, vel=vel, a=a, b=b)
    wu, _ = to_device(w2)
    out = alloc_output(w2)
    with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f) as p:
        p.compute(wu, out)
        torch.cuda.synchronize()
    g = out.twoF.cpu().numpy().ravel()
    e = twoF_error(g, oracle.fstat(w2)["twoF"])
    _say(f"device detector inputs: max 2F error vs oracle {e.max():.2e}")
    assert e.max() <= 1e-4
    e_gen = twoF_error(g, oracle.fstat(w)["twoF"])
    _say(f"  against the generator's inputs: max {e_gen.max():.2e}")
    assert e_gen.max() <= 1e-4
