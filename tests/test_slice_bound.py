"""The interp kernel's LDS slice width (fstat_interp_slice, a host function of
the library) against brute force: for random geometry and random tiles of
frequency templates x spindowns, every template's bin k* must fall inside the
slice the kernel stages, [lo, lo + W), with lo one bin below the lowest k* of
the tile's corners, whenever the library reports that the slice fits (the
kernel variant without a global-memory path then relies on it).  k* is the
floor of the canonical FP64 D-hat-phi = f P + (fdot tau) P, evaluated here
for every template of the tile, not only the corners."""
import numpy as np
import pytest

import paper_0904_1826_amd as P

T_SFT = 1800.0


def _dphi(f, fd, tau, p):
    # f P + q with q = (fdot tau) P rounded; the sum in extended precision is
    # within an ulp of the fused multiply-add the library uses, far below the
    # bin of slack the slice has
    q = (fd * tau) * p
    return (np.longdouble(f) * np.longdouble(p) + np.longdouble(q)).astype(np.float64)


def _check_tiles(rng, W, nt, nfd, df, dfdot, max_tau, max_p, n_tiles):
    worst = 0
    for _ in range(n_tiles):
        f0 = rng.uniform(50.0, 1500.0)
        f = f0 + np.arange(nt) * df
        fd0 = -rng.uniform(0.0, 1e-8)
        fd = fd0 + np.arange(nfd) * dfdot
        # corners of the (tau, P) box are where the spread is widest
        tau = rng.choice([-max_tau, max_tau, rng.uniform(-max_tau, max_tau)])
        p = rng.choice([max_p, rng.uniform(T_SFT * (1 - 1e-4), max_p)])
        d = _dphi(f[:, None], fd[None, :], tau, p)
        k = np.floor(d)
        d1, d2 = _dphi(f[0], fd[0], tau, p), _dphi(f[0], fd[-1], tau, p)
        d3, d4 = _dphi(f[-1], fd[0], tau, p), _dphi(f[-1], fd[-1], tau, p)
        kmin, kmax = np.floor(min(d1, d2)), np.floor(max(d3, d4))
        assert k.min() == kmin and k.max() == kmax        # D-hat-phi is monotone in f and in fdot
        lo = kmin - 1                                     # the kernel's slice start (band far from 0)
        assert k.min() >= lo and k.max() <= lo + W - 1, (W, k.min() - lo, k.max() - lo)
        worst = max(worst, int(k.max() - lo) + 1)
    return worst


@pytest.mark.parametrize("threads,coef16", [(256, False), (256, True), (64, False)])
@pytest.mark.parametrize("nfd", [8, 4, 2, 1])
def test_slice_holds_every_window_when_it_fits(threads, coef16, nfd):
    rng = np.random.default_rng(1000 * nfd + threads + coef16)
    cap = (threads + threads // 8 + 8) if not coef16 else 3 * threads // 2
    n_fit = 0
    for trial in range(40):
        max_tau = rng.choice([5e2, 3e6, 1.2e7]) * rng.uniform(0.5, 1.0)
        max_p = T_SFT * (1.0 + rng.uniform(0.0, 1e-4))
        df = rng.choice([1.0 / T_SFT, 0.5 / T_SFT, 1.0 / 1024.0])
        dfdot = 10 ** rng.uniform(-13, -8.5)
        W, fits = P.fstat_interp_slice(df, dfdot, nfd, threads, coef16, max_tau, max_p)
        assert W % 4 == 0 and 8 <= W <= cap
        if not fits:
            continue
        n_fit += 1
        worst = _check_tiles(rng, W, threads, nfd, df, dfdot, max_tau, max_p, 60)
        assert worst <= W
    assert n_fit >= 10


@pytest.mark.parametrize("coef16", [False, True])
def test_slice_at_capacity_edge(coef16):
    """Spindown steps that put the spread within a few bins of the slice's
    capacity: reported fits must hold there, and one bin more must not fit."""
    rng = np.random.default_rng(7 + coef16)
    nt, nfd = 256, 8
    cap = 296 if not coef16 else 384
    max_tau, max_p = 1.2e7, T_SFT * (1.0 + 1e-4)
    df = 1.0 / T_SFT
    seen = set()
    for target in np.linspace(cap - 12.0, cap - 2.0, 41):
        dfdot = (target - (nt - 1) * df * max_p) / ((nfd - 1) * max_tau * max_p)
        W, fits = P.fstat_interp_slice(df, dfdot, nfd, nt, coef16, max_tau, max_p)
        seen.add(fits)
        if fits:
            assert _check_tiles(rng, W, nt, nfd, df, dfdot, max_tau, max_p, 80) <= W
    assert seen == {True, False}
