"""The sky pairing of the interp kernels (fstat_sky_pairs, a host function of
the library) against brute force: a tile of two sky points stages one slice
per SFT, starting one bin below the lowest k* of the tile's corners over both
points, and the kernel variant without a global-memory path relies on every
k* of both points lying in it.  For synthetic geometry (the generator's
orbit, Fibonacci skies) the k* of both points of every pair are evaluated
from the canonical FP64 D-hat-phi = f P + (fdot tau) P at the corners of
random tiles (256 frequencies x min(n_fd, 8) spindowns) for every SFT, and
at every template of the tile for a sample of pairs and SFTs; the pairing
must also place every sky point in exactly one tile, and leave few points
without a partner."""
import dataclasses

import numpy as np
import pytest

import paper_0904_1826_amd as P
import synth

T_SFT = 1800.0


def _unit(seed, f0, n_sky, slots, n_fd=8, n_f=3600):
    return synth.make_workload(f"pairs-bound-{seed}", seed=seed, n_det=2, slots_per_det=slots, keep_frac=0.6,
                               jitter=0.0, t_sft=T_SFT, f0=f0, n_f=n_f, n_sky=n_sky, n_fd=n_fd, fdot_lo=-1e-9,
                               fdot_hi=0.0, dterms=8, injections=(), noise=False)


def _geometry(w):
    tau = (w.t_start + 0.5 * w.t_sft - w.t_ref)[None, :] + w.sky @ w.pos.T
    p = (1.0 + w.sky @ w.vel.T) * w.t_sft
    vmax = float(np.sqrt((w.vel ** 2).sum(axis=1)).max())
    rmax = float(np.sqrt((w.pos ** 2).sum(axis=1)).max())
    return tau, p, float(np.abs(tau).max()), float(p.max()), vmax, rmax


def _kstar(f, fd, tau, p):
    # floor of f P + (fdot tau) P; the sum in extended precision is within an
    # ulp of the library's fused multiply-add, far below the slice's slack
    q = (fd * tau) * p
    return np.floor(np.longdouble(f) * np.longdouble(p) + np.longdouble(q))


def _pairs(w, g):
    _, _, max_tau, max_p, vmax, rmax = g
    return P.fstat_sky_pairs(w.sky, w.f0, w.df, w.n_f, w.fdot0, w.dfdot, w.n_fd, w.t_sft, max_tau, max_p, vmax, rmax)


@pytest.mark.parametrize("seed,f0,n_sky,slots", [(1, 1000.0, 2000, 1667), (2, 250.0, 400, 400), (3, 1450.0, 1200, 900)])
def test_pair_slices_hold_both_points_windows(seed, f0, n_sky, slots):
    w = _unit(seed, f0, n_sky, slots)
    g = _geometry(w)
    tau, p = g[0], g[1]
    width, tiles = _pairs(w, g)
    assert width > 0 and width % 4 == 0 and width <= 296
    # every sky point in exactly one tile (a point without a partner appears twice in its own)
    members = np.concatenate([np.unique(t) for t in tiles])
    assert np.array_equal(np.sort(members), np.arange(w.n_sky))
    real = tiles[tiles[:, 0] != tiles[:, 1]]
    assert 2 * 2 * len(real) >= w.n_sky                      # at least half the points pair
    # the points left alone by consecutive pairing (band ends) are paired among
    # themselves where they fit: few tiles of one point remain on these grids
    assert len(tiles) - len(real) <= (w.n_sky // 100 if f0 < 1200 else w.n_sky // 10)
    a, b = real[:, 0], real[:, 1]
    rng = np.random.default_rng(seed)
    nfd = min(w.n_fd, 8)
    worst = 0
    for _ in range(4):
        j0 = int(rng.integers(0, w.n_f - 255))
        i0 = int(rng.integers(0, w.n_fd - nfd + 1))
        f_lo, f_hi = w.f0 + j0 * w.df, w.f0 + (j0 + 255) * w.df
        fd = [w.fdot0 + i0 * w.dfdot, w.fdot0 + (i0 + nfd - 1) * w.dfdot]
        # corners of both points of every pair, every SFT: [pairs, SFTs]
        ks = [_kstar(f, d, tau[s], p[s]) for s in (a, b) for f in (f_lo, f_hi) for d in fd]
        lo = np.minimum.reduce(ks) - 1
        hi = np.maximum.reduce(ks)
        span = (hi - lo + 1).astype(np.int64)
        worst = max(worst, int(span.max()))
        assert span.max() <= width, (span.max(), width)
        # every template of the tile for a few pairs and SFTs
        for x in rng.choice(len(a), size=3, replace=False):
            al = rng.choice(w.n_sft, size=40, replace=False)
            f = (w.f0 + (j0 + np.arange(256)) * w.df)[:, None, None]
            d = (w.fdot0 + (i0 + np.arange(nfd)) * w.dfdot)[None, :, None]
            for s in (a[x], b[x]):
                k = _kstar(f, d, tau[s, al][None, None, :], p[s, al][None, None, :])
                assert np.all(k >= lo[x, al]) and np.all(k <= lo[x, al] + width - 1)
    assert worst <= width


def test_poles_and_duplicate_points_pair_with_their_copies():
    """Both poles twice (their longitude is undefined) and a close pair on the
    equator: three tiles of two points, each point in exactly one."""
    w = _unit(6, 400.0, 6, 100)
    sky = np.array([[0, 0, 1.0], [0, 0, -1.0], [0, 0, 1.0], [np.cos(0.4), np.sin(0.4), 0.0], [0, 0, -1.0],
                    [np.cos(0.4) * np.cos(0.01), np.sin(0.4) * np.cos(0.01), -np.sin(0.01)]])
    w = dataclasses.replace(w, sky=sky)
    width, tiles = _pairs(w, _geometry(w))
    assert width > 0 and len(tiles) == 3
    assert sorted(map(sorted, tiles.tolist())) == [[0, 2], [1, 4], [3, 5]]


def test_sparse_sky_keeps_one_point_per_tile():
    w = _unit(4, 1500.0, 30, 200)
    width, tiles = _pairs(w, _geometry(w))
    assert width == 0 and len(tiles) == 0


def test_tiny_sky_and_bad_arguments():
    w = _unit(5, 300.0, 3, 40)
    width, tiles = _pairs(w, _geometry(w))
    assert width == 0 and len(tiles) == 0                  # fewer than 4 points: never paired
    lib = P.load_library()
    assert lib.fstat_sky_pairs(0, None, 1.0, 1.0, 1, 0.0, 0.0, 1, 1800.0, 1.0, 1800.0, 1e-4, 500.0, None,
                               None) == P.FSTAT_E_ARG
