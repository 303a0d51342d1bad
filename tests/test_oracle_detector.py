"""Pins of the oracle's detector inputs (positions, velocities, antenna
patterns) against closed forms and independent constructions."""
import math

import numpy as np

import oracle
import synth.workloads as sw

EARTH = dict(t0=8.0e8, orbit_radius=499.005, orbit_rate=2 * math.pi / (365.25636 * 86400.0), orbit_phase=0.3,
             obliquity=math.radians(23.4393), earth_radius=6378137.0 / 299792458.0,
             sidereal_rate=2 * math.pi / 86164.0905, sidereal_phase=1.1)
SITE = (math.radians(46.5), math.radians(-119.4), math.radians(126.0), math.radians(216.0))


def _vertical(site, t):
    th = site[1] + EARTH["sidereal_phase"] + EARTH["sidereal_rate"] * (t - EARTH["t0"])
    return np.array([math.cos(site[0]) * math.cos(th), math.cos(site[0]) * math.sin(th), math.sin(site[0])])


def test_zenith_response_is_sin_of_arm_angle():
    """A source overhead sees |F|^2 = a^2 + b^2 = sin^2 of the angle between the arms."""
    for zeta in (90.0, 60.0, 120.0):
        site = (SITE[0], SITE[1], SITE[2], SITE[2] + math.radians(zeta))
        for t in (8.0e8, 8.0e8 + 12345.6, 8.1e8):
            n = _vertical(site, t)
            _, _, a, b = oracle.detector_inputs(EARTH, [site], [t], [0], n[None, :])
            assert abs(a[0, 0] ** 2 + b[0, 0] ** 2 - math.sin(math.radians(zeta)) ** 2) < 1e-12


def test_sky_average_is_two_fifths_sin2():
    """Averaged over isotropic directions, a^2 + b^2 = (2/5) sin^2 zeta."""
    n = sw.sky_grid(200000)
    for zeta in (90.0, 50.0):
        site = (SITE[0], SITE[1], SITE[2], SITE[2] + math.radians(zeta))
        _, _, a, b = oracle.detector_inputs(EARTH, [site], [8.0e8 + 777.0], [0], n)
        avg = float(np.mean(a ** 2 + b ** 2))
        assert abs(avg - 0.4 * math.sin(math.radians(zeta)) ** 2) < 2e-4, avg


def test_against_arm_projections():
    """a, b from the arms' projections on the wave frame, with the local frame
    built from the vertical by cross products (a different construction)."""
    rng = np.random.default_rng(3)
    n = rng.normal(size=(40, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    t = 8.0e8 + rng.uniform(0, 3e7, 25)
    _, _, a, b = oracle.detector_inputs(EARTH, [SITE], t, np.zeros(len(t), np.int32), n)
    for k, tk in enumerate(t):
        up = _vertical(SITE, tk)
        east = np.cross([0.0, 0.0, 1.0], up)
        east /= np.linalg.norm(east)
        north = np.cross(up, east)
        u = math.cos(SITE[2]) * north + math.sin(SITE[2]) * east
        w = math.cos(SITE[3]) * north + math.sin(SITE[3]) * east
        for s in range(len(n)):
            al, dl = math.atan2(n[s, 1], n[s, 0]), math.asin(n[s, 2])
            X = np.array([math.sin(al), -math.cos(al), 0.0])
            Y = np.array([-math.sin(dl) * math.cos(al), -math.sin(dl) * math.sin(al), math.cos(dl)])
            fp = 0.5 * ((u @ X) ** 2 - (u @ Y) ** 2 - (w @ X) ** 2 + (w @ Y) ** 2)
            fc = (u @ X) * (u @ Y) - (w @ X) * (w @ Y)
            assert abs(a[s, k] - fp) < 1e-13 and abs(b[s, k] - fc) < 1e-13


def test_orbit_geometry_and_velocity_is_derivative():
    t = 8.0e8 + np.linspace(0, 3.1e7, 37)
    e0 = dict(EARTH, earth_radius=0.0)
    pos, vel, _, _ = oracle.detector_inputs(e0, [SITE], t, np.zeros(len(t), np.int32), np.eye(3))
    R, W = e0["orbit_radius"], e0["orbit_rate"]
    assert np.allclose(np.linalg.norm(pos, axis=1), R, rtol=1e-14)
    assert np.allclose(np.linalg.norm(vel, axis=1), R * W, rtol=1e-13)
    assert np.max(np.abs(np.sum(pos * vel, axis=1))) < 1e-12 * R * R * W
    # the orbit lies in the ecliptic: normal (0, -sin eps, cos eps)
    nrm = np.array([0.0, -math.sin(e0["obliquity"]), math.cos(e0["obliquity"])])
    assert np.max(np.abs(pos @ nrm)) < 1e-12 * R
    # with the Earth's rotation: v = dr/dt by a central difference
    h = 5.0
    pp, vv, _, _ = oracle.detector_inputs(EARTH, [SITE], np.concatenate([t + h, t - h, t]),
                                          np.zeros(3 * len(t), np.int32), np.eye(3))
    fd = (pp[: len(t)] - pp[len(t): 2 * len(t)]) / (2 * h)
    assert np.max(np.abs(fd - vv[2 * len(t):])) < 1e-12   # truncation (h W)^2 / 6 and rounding of r / 2h
    # the site is R_e from the Earth's centre
    assert np.allclose(np.linalg.norm(pp[2 * len(t):] - pos, axis=1), EARTH["earth_radius"], rtol=1e-9)


def test_patterns_repeat_every_sidereal_day():
    n = sw.sky_grid(50)
    t = np.array([8.0e8 + 1234.5])
    day = 2 * math.pi / EARTH["sidereal_rate"]
    _, _, a0, b0 = oracle.detector_inputs(EARTH, [SITE], t, [0], n)
    _, _, a1, b1 = oracle.detector_inputs(EARTH, [SITE], t + 50 * day, [0], n)
    assert np.max(np.abs(a1 - a0)) < 1e-9 and np.max(np.abs(b1 - b0)) < 1e-9


def test_reduces_to_the_workload_generator_model():
    """Without the diurnal term and with the generator's constants, the
    oracle reproduces the synthetic inputs (orbit and antenna patterns)."""
    e = dict(t0=sw.EPOCH, orbit_radius=sw.ORBIT_R, orbit_rate=sw.ORBIT_OMEGA, orbit_phase=0.3,
             obliquity=sw.OBLIQUITY, earth_radius=0.0, sidereal_rate=sw.SIDEREAL_OMEGA, sidereal_phase=0.0)
    lat, lon, az = (math.radians(x) for x in sw.SITES[0])
    t = sw.EPOCH + np.linspace(900.0, 2.9e7, 64)
    n = sw.sky_grid(30)
    pos, vel, a, b = oracle.detector_inputs(e, [(lat, lon, az, az + math.pi / 2)], t, np.zeros(64, np.int32), n)
    p2, v2 = sw.orbit(t)
    a2, b2 = sw.antenna_patterns(sw.SITES[0], n, t)
    assert np.max(np.abs(pos - p2)) < 1e-10 and np.max(np.abs(vel - v2)) < 1e-16
    assert np.max(np.abs(a.astype(np.float32) - a2)) <= 1.2e-7 and np.max(np.abs(b.astype(np.float32) - b2)) <= 1.2e-7
