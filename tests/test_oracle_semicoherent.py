"""Pins of the oracle's semi-coherent statistic (the sum over time segments
of each segment's coherent 2F) against facts that do not come from the
oracle: the chi-square law with 4 N degrees of freedom of a sum of N
independent noise-only 2F values (its mean catches a dropped or doubled
segment, its variance a segment counted in place of another), and the
recovery of N rho^2 from a phase-continuous signal synthesised in the time
domain with SNR rho in each segment."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import synth
from tests._helpers import kernel_power_loss


def _segments(n_seg, seed, **kw):
    p = dict(n_det=2, seg_slots=12, keep_frac=1.0, jitter=60.0, t_sft=1800.0, f0=200.0, n_f=500, n_sky=24, n_fd=2,
             fdot_lo=-2e-9, fdot_hi=0.0, dterms=8)
    p.update(kw)
    return synth.make_segments(n_seg, seed=seed, **p)


def test_segments_share_the_template_grid():
    segs = _segments(3, 31, n_sky=3, n_f=40)
    g = segs[0]
    for w in segs[1:]:
        assert (w.f0, w.df, w.n_f, w.fdot0, w.dfdot, w.n_fd, w.t_ref) == (g.f0, g.df, g.n_f, g.fdot0, g.dfdot,
                                                                         g.n_fd, g.t_ref)
        assert np.array_equal(w.sky, g.sky)
        assert w.t_start.min() > segs[0].t_start.max()          # disjoint, consecutive spans
    assert g.t_ref == synth.EPOCH


def test_noise_only_sum_is_chi2_4N(oracle_lib):
    n_seg = 4
    segs = _segments(n_seg, 41)
    r = oracle_lib.semicoherent(segs)
    tf = r["twoF"]
    s, i, j = r["templates"]
    wbar = integrate.quad(lambda k: 1.0 - kernel_power_loss(k, 8), 0.0, 1.0)[0]
    assert len(tf) == 24 * 2 * 500
    # chi^2 with 4 N degrees of freedom, scaled by the mean window power wbar
    assert abs(tf.mean() / (4.0 * n_seg * wbar) - 1.0) < 0.02, (tf.mean(), wbar)
    assert abs(tf.var() / (8.0 * n_seg * wbar ** 2) - 1.0) < 0.08, tf.var()
    pick = (j % 3 == 0) & (s % 2 == 0)
    ks = stats.kstest(tf[pick] / wbar, stats.chi2(4 * n_seg).cdf).statistic
    assert ks < 0.03, ks
    # the same data as one segment repeated would give variance 8 N^2 wbar^2
    rep = oracle_lib.semicoherent([segs[0]] * n_seg)["twoF"]
    assert rep.var() > 2.5 * tf.var()


@pytest.mark.parametrize("n_seg", [1, 3])
def test_time_domain_signal_sums_segment_snr(oracle_lib, n_seg):
    """Noiseless phase-continuous signal with SNR 10 in each segment: the sum
    at the injected template approaches n_seg * 100 within the window loss
    of Dterms = 64; off-template frequencies see almost nothing."""
    segs = _segments(n_seg, 51, seg_slots=10, f0=300.0, n_f=64, n_sky=4, fdot_lo=-3e-9, dterms=64, noise=False,
                     injections=[(1, 1, 31, 10.0)])
    r = oracle_lib.semicoherent(segs, ([1], [1], [31]))
    ratio = r["twoF"][0] / (100.0 * n_seg)
    assert 0.993 <= ratio <= 1.002, ratio
    off = oracle_lib.semicoherent(segs, ([1, 1], [1, 1], [27, 35]))
    assert np.all(off["twoF"] < 0.05 * r["twoF"][0])


def test_sum_is_order_free_and_reduces_to_coherent(oracle_lib):
    segs = _segments(3, 61, n_sky=3, n_f=60, injections=[(2, 0, 30, 8.0)])
    a = oracle_lib.semicoherent(segs)["twoF"]
    b = oracle_lib.semicoherent(segs[::-1])["twoF"]
    assert np.allclose(a, b, rtol=1e-13, atol=0)
    one = oracle_lib.semicoherent(segs[:1])["twoF"]
    assert np.array_equal(one, oracle_lib.fstat(segs[0])["twoF"])
    assert math.isclose(a.sum(), sum(oracle_lib.fstat(w)["twoF"].sum() for w in segs), rel_tol=1e-12)
