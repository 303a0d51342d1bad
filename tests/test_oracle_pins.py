"""Pins of the FP64 oracle against facts fixed by mathematics, not by the
oracle itself: Dirichlet-kernel identities, a closed-form noiseless
injection, time-domain demodulation, chi^2_4 noise statistics, an
independent bin-index evaluation, exact rational phase, invariances and a
hand-derived single-term case."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from tests._helpers import small_workload, replace, kernel_power_loss

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- kernel ---
@pytest.mark.parametrize("kappa", [0.0, 1e-12, 0.013, 0.25, 0.5, 0.77, 0.999999])
def test_dirichlet_partition_of_unity(oracle_lib, kappa):
    """sum_m sinc(kappa+m) = 1 and sum_m sinc^2(kappa+m) = 1 over all m."""
    D = 200000
    w = oracle_lib.window_weights(kappa, D)
    assert abs(w.sum() - 1.0) < 1e-5
    # the squared tail beyond the window is sin^2/pi^2 (psi1(kappa+D) + psi1(D+1-kappa)) ~ 1e-6
    assert abs((w * w).sum() - (1.0 - kernel_power_loss(kappa, D))) < 1e-11


@pytest.mark.parametrize("dterms", [1, 4, 8, 16, 64])
def test_window_power_closed_form(oracle_lib, dterms):
    """Truncated kernel power equals 1 - trigamma tail, and the loss stays
    under 2/(pi^2 D) (0.0253 at D=8, 0.0127 at D=16)."""
    for kappa in np.linspace(0.0, 0.999, 37):
        w = oracle_lib.window_weights(kappa, dterms)
        loss = 1.0 - np.sum(w * w)
        assert abs(loss - kernel_power_loss(kappa, dterms)) < 1e-13
        assert loss <= 2.0 / (math.pi ** 2 * (dterms - 0.5)) + 1e-15


def test_sinc_values(oracle_lib):
    assert oracle_lib.sinc(0.0) == 1.0
    assert abs(oracle_lib.sinc(0.5) - 2.0 / math.pi) < 1e-16
    for n in range(1, 6):
        assert abs(oracle_lib.sinc(float(n))) < 1e-15


# ------------------------------------------------- P1: closed-form signal ---
def _ideal_injection(w, s_idx, fd_idx, f_idx, amp_a, amp_b):
    """SFT bins of a noiseless signal whose phase is exactly linear across each
    SFT: X[k] = s * exp(2 pi i phi) (-1)^k sinc(Dphi - k) over the whole band.
    Returns the data and the per-SFT complex amplitudes s."""
    n = w.sky[s_idx]
    f = w.f0 + float(f_idx) * w.df
    fd = w.fdot0 + float(fd_idx) * w.dfdot
    t_mid = w.t_start + 0.5 * w.t_sft
    rn = (w.pos[:, 0] * n[0] + w.pos[:, 1] * n[1]) + w.pos[:, 2] * n[2]
    vn = (w.vel[:, 0] * n[0] + w.vel[:, 1] * n[1]) + w.vel[:, 2] * n[2]
    tau = (t_mid - w.t_ref) + rn
    dphi = ((f + fd * tau) * (1.0 + vn)) * w.t_sft
    phi = tau * (f + (0.5 * fd) * tau)
    phi = phi - np.floor(phi)
    s = w.a[s_idx].astype(np.float64) * amp_a + w.b[s_idx].astype(np.float64) * amp_b
    k = w.k_first + np.arange(w.n_bins)
    x = (s[:, None] * np.exp(2j * np.pi * phi)[:, None] * np.where(k % 2 == 0, 1.0, -1.0)[None, :]
         * np.sinc(dphi[:, None] - k[None, :]))
    return x, s, dphi


def _closed_form_2F(w, s_idx, s, dphi, dterms):
    kappa = dphi - np.floor(dphi)
    W = 1.0 - kernel_power_loss(kappa, dterms)
    a = w.a[s_idx].astype(np.float64)
    b = w.b[s_idx].astype(np.float64)
    y = np.array([np.sum(a * s * W), np.sum(b * s * W)])
    M = np.array([[a @ a, a @ b], [a @ b, b @ b]])
    return 2.0 * np.real(np.conj(y) @ np.linalg.solve(M, y)), y


@pytest.mark.parametrize("dterms", [4, 8, 16])
def test_closed_form_noiseless_injection(oracle_lib, dterms):
    w = small_workload(11, dterms=32, noise=False, injections=())
    w = replace(w, dterms=dterms)
    amp_a, amp_b = 0.8 - 0.3j, -0.2 + 0.9j
    x, s, dphi = _ideal_injection(w, 3, 1, 77, amp_a, amp_b)
    expect, y = _closed_form_2F(w, 3, s, dphi, dterms)
    r = oracle_lib.fstat(w, ([3], [1], [77]), sft=x)
    assert abs(r["twoF"][0] - expect) < 1e-9 * expect
    assert abs(r["Fa"][0] - y[0]) < 1e-9 * abs(y[0])
    assert abs(r["Fb"][0] - y[1]) < 1e-9 * abs(y[1])
    rho2 = 2.0 * np.sum(np.abs(s) ** 2)
    # truncation loss of the window: at most 2/(pi^2 (D - 1/2)) of the power
    assert rho2 * (1 - 2.0 / (math.pi ** 2 * (dterms - 0.5))) ** 2 <= r["twoF"][0] <= rho2 * (1 + 1e-12)


# --------------------------------------- P4: time-domain synthesised data ---
@pytest.mark.parametrize("dterms,lo", [(8, 0.95), (16, 0.975), (64, 0.993)])
def test_time_domain_injection_recovers_snr(oracle_lib, dterms, lo):
    """SFTs are DFTs of the sampled waveform (exact per-sample Doppler and
    spindown phase); the demodulated 2F of the injected template approaches
    rho^2 as the window widens, within the kernel truncation loss."""
    w = synth.make_workload("td", seed=5, n_det=2, slots_per_det=20, keep_frac=1.0, jitter=30.0, t_sft=1800.0,
                            f0=300.0, n_f=64, n_sky=4, n_fd=2, fdot_lo=-3e-9, fdot_hi=0.0, dterms=64,
                            injections=[(1, 1, 31, 10.0)], noise=False)
    w = replace(w, dterms=dterms)
    r = oracle_lib.fstat(w, ([1], [1], [31]))
    ratio = r["twoF"][0] / 100.0
    assert lo <= ratio <= 1.002, ratio
    # off-template frequencies see almost nothing of the signal
    r2 = oracle_lib.fstat(w, ([1, 1], [1, 1], [27, 35]))
    assert np.all(r2["twoF"] < 0.05 * r["twoF"][0])


def test_time_domain_matched_filter_agreement(oracle_lib):
    """Fa from the SFT-domain window sum agrees with a direct time-domain sum
    of data x(t) exp(-2 pi i Phi_lin(t)) over each SFT as the window grows."""
    nb = 128
    w = synth.make_workload("tdmf", seed=9, n_det=1, slots_per_det=6, keep_frac=1.0, jitter=20.0, t_sft=60.0,
                            f0=20.0, n_f=8, n_sky=2, n_fd=1, fdot_lo=0.0, fdot_hi=0.0, dterms=40,
                            injections=(), noise=False)
    rng = np.random.default_rng(3)
    # time-domain data: noise plus a tone near the template, band-limited to the stored band
    n_b = w.n_bins
    td = (rng.standard_normal((w.n_sft, n_b)) + 1j * rng.standard_normal((w.n_sft, n_b))) / math.sqrt(2)
    x = np.fft.fft(td, axis=1) / n_b
    s_i, j_i = 1, 4
    errs = []
    n = w.sky[s_i]
    f = w.f0 + j_i * w.df
    t_mid = w.t_start + 0.5 * w.t_sft
    tau = (t_mid - w.t_ref) + w.pos @ n
    tdot = 1.0 + w.vel @ n
    finst = f * tdot                      # fdot = 0
    phi = tau * f
    # time-domain matched filter of the heterodyned samples with the linear phase
    j = np.arange(n_b)
    fa_td = 0.0
    for al in range(w.n_sft):
        t_rel = j * (w.t_sft / n_b) - 0.5 * w.t_sft
        cyc = phi[al] + finst[al] * t_rel - (w.k_first * j) / n_b
        fa_td += w.a[s_i, al] * np.mean(td[al] * np.exp(-2j * np.pi * cyc))
    for dterms in (8, 16, 40):
        r = oracle_lib.fstat(replace(w, dterms=dterms), ([s_i], [0], [j_i]), sft=x)
        errs.append(abs(r["Fa"][0] - fa_td) / abs(fa_td))
    assert errs[2] < errs[0]
    assert errs[0] < 0.08 and errs[2] < 0.03, errs


def test_time_domain_discrete_kernel_identity_and_convergence(oracle_lib):
    """The survey's time-domain pin, at 4096 samples per SFT: (1) the
    time-domain matched filter of each SFT's samples with the SFT-linear phase
    equals the sum over all N bins of the SFT's DFT weighted by the discrete
    Dirichlet kernel (1/N) sum_j exp(-2 pi i kappa j / N), to rounding (an
    identity of the DFT, which checks this test's own conventions); (2) the
    oracle's Fa, which keeps the 2D bins nearest the instantaneous frequency
    and uses the continuous kernel sinc, approaches the time-domain Fa as D
    grows, to 2.5e-4 at D = 256 (the rest is the continuous kernel standing
    in for the discrete one, of order (D / N)^2)."""
    N = 4096
    w = synth.make_workload("tdmf4096", seed=9, n_det=1, slots_per_det=6, keep_frac=1.0, jitter=20.0, t_sft=60.0,
                            f0=20.0, n_f=8, n_sky=2, n_fd=1, fdot_lo=0.0, fdot_hi=0.0, dterms=8,
                            injections=(), noise=False)
    k_first = w.k_first + w.n_bins // 2 - N // 2       # a band of N bins around the templates
    w = replace(w, k_first=k_first, sft=np.zeros((w.n_sft, N), dtype=np.complex64))
    rng = np.random.default_rng(3)
    j = np.arange(N)
    s_i, j_i = 1, 4
    f = w.f0 + j_i * w.df
    # noise plus a tone 0.3 bins from the template's frequency (heterodyned samples)
    td = (rng.standard_normal((w.n_sft, N)) + 1j * rng.standard_normal((w.n_sft, N))) / math.sqrt(2)
    td += 3.0 * np.exp(2j * np.pi * (f * w.t_sft - k_first + 0.3) * j / N)
    X = np.fft.fft(td, axis=1) / N                    # column q is bin k_first + q
    # the discrete kernel by its geometric-series closed form, checked against the plain sum
    def kdisc(kap):
        e1 = np.exp(-2j * np.pi * kap)
        eN = np.exp(-2j * np.pi * kap / N)
        return (1.0 - e1) / (N * (1.0 - eN))
    for kap in rng.uniform(-50.0, 50.0, 8):
        assert abs(kdisc(kap) - np.mean(np.exp(-2j * np.pi * kap * j / N))) < 1e-12
    n = w.sky[s_i]
    tau = (w.t_start + 0.5 * w.t_sft - w.t_ref) + w.pos @ n
    finst = f * (1.0 + w.vel @ n)                     # fdot = 0
    phi = tau * f
    fa_td = 0.0
    for al in range(w.n_sft):
        t_rel = j * (w.t_sft / N) - 0.5 * w.t_sft
        cyc = phi[al] + finst[al] * t_rel - (w.k_first * j) / N
        z_td = np.mean(td[al] * np.exp(-2j * np.pi * cyc))
        dphi = finst[al] * w.t_sft
        kap = dphi - (k_first + np.arange(N))
        z_disc = np.exp(-2j * np.pi * (phi[al] - dphi / 2.0)) * np.sum(X[al] * kdisc(kap))
        assert abs(z_disc - z_td) <= 1e-10 * abs(z_td), (al, abs(z_disc - z_td) / abs(z_td))
        fa_td += w.a[s_i, al] * z_td
    errs = {}
    for dterms in (8, 64, 256):
        r = oracle_lib.fstat(replace(w, dterms=dterms), ([s_i], [0], [j_i]), sft=X)
        errs[dterms] = abs(r["Fa"][0] - fa_td) / abs(fa_td)
    assert errs[8] > errs[64] > errs[256], errs
    assert errs[256] < 5e-4 and errs[8] < 0.05, errs


# ------------------------------------------------- P2: noise statistics ---
def test_noise_only_chi2_4(oracle_lib):
    from scipy import stats, integrate
    w = small_workload(21, n_det=2, slots=30, keep=1.0, n_sky=40, n_fd=4, n_f=600, f0=200.0,
                       injections=(), dterms=8)
    s, i, j = oracle_lib.all_templates(w)
    r = oracle_lib.fstat(w, (s, i, j))
    tf = r["twoF"]
    wbar = integrate.quad(lambda k: 1.0 - kernel_power_loss(k, 8), 0.0, 1.0)[0]
    assert len(tf) >= 90000
    assert abs(tf.mean() / (4.0 * wbar) - 1.0) < 0.02, (tf.mean(), wbar)
    assert abs(tf.var() / (8.0 * wbar ** 2) - 1.0) < 0.06, tf.var()
    pick = (j % 3 == 0) & (s % 4 == 0)
    ks = stats.kstest(tf[pick] / wbar, stats.chi2(4).cdf).statistic
    assert ks < 0.02, ks


# ------------------------------------ P5: independent bin-index evaluation ---
def _py_bins(w, s, i, j, al):
    n = [float(v) for v in w.sky[s]]
    r = [float(v) for v in w.pos[al]]
    v = [float(x) for x in w.vel[al]]
    T = float(w.t_sft)
    t_mid = float(w.t_start[al]) + 0.5 * T
    rn = (r[0] * n[0] + r[1] * n[1]) + r[2] * n[2]
    vn = (v[0] * n[0] + v[1] * n[1]) + v[2] * n[2]
    tau = (t_mid - float(w.t_ref)) + rn
    tdot = 1.0 + vn
    f = float(w.f0) + float(j) * float(w.df)
    fd = float(w.fdot0) + float(i) * float(w.dfdot)
    P = tdot * T
    q = (fd * tau) * P
    dphi = _fma(f, P, q)
    k = math.floor(dphi)
    return k, dphi - k, tau, f, fd


def _fma(a, b, c):
    """a * b + c rounded once: exact rational sum, then Python's correctly
    rounded integer division."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_bin_index_bit_exact_vs_python(oracle_lib):
    w = synth.make_config(1, slots_per_det=40, n_sky=50, n_f=3600, injections=(), noise=False)
    rng = np.random.default_rng(0)
    n = 400
    ts = rng.integers(0, w.n_sky, n).astype(np.int32)
    ti = rng.integers(0, w.n_fd, n).astype(np.int32)
    tj = rng.integers(0, w.n_f, n).astype(np.int32)
    k, kap, ph, dp = oracle_lib.bins(w, (ts, ti, tj))
    for t in range(n):
        for al in range(0, w.n_sft, 7):
            kp, kapp, _, _, _ = _py_bins(w, ts[t], ti[t], tj[t], al)
            assert k[t, al] == kp
            assert kap[t, al] == kapp          # bit-identical


def test_bin_index_exact_integer_case(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "single_term_kappa0.json")))
    w = _golden_workload(g)
    k, kap, ph, dp = oracle_lib.bins(w, ([0], [0], [0]))
    assert list(k[0]) == [g["kstar"]] * 2
    assert list(kap[0]) == [0.0, 0.0]
    assert list(ph[0]) == [0.0, 0.0]


# ------------------------------------------------ P6: exact rational phase ---
def test_phase_vs_exact_rational(oracle_lib):
    w = synth.make_config(1, slots_per_det=1667, keep_frac=0.02, n_sky=8, injections=(), noise=False)
    k, kap, ph, dp = oracle_lib.bins(w, ([0, 3, 7], [0, 4, 7], [0, 1800, 3599]))
    for t, (s, i, j) in enumerate([(0, 0, 0), (3, 4, 1800), (7, 7, 3599)]):
        for al in range(w.n_sft):
            _, _, tau, f, fd = _py_bins(w, s, i, j, al)
            exact = Fraction(tau) * (Fraction(f) + Fraction(fd) / 2 * Fraction(tau))
            frac_exact = exact - math.floor(exact)
            d = abs(Fraction(ph[t, al]) - frac_exact)
            d = min(d, 1 - d)
            ulp = math.ulp(abs(f * tau))
            assert float(d) <= 4 * ulp, (float(d), ulp)


# ------------------------------------------------------ P7: invariances ---
def test_invariances(oracle_lib):
    w = small_workload(31)
    tmpl = oracle_lib.all_templates(w, [0, 2, 5])
    ref = oracle_lib.fstat(w, tmpl)["twoF"]
    rng = np.random.default_rng(1)
    perm = rng.permutation(w.n_sft)
    wp = replace(w, sft=w.sft[perm], t_start=w.t_start[perm], pos=w.pos[perm], vel=w.vel[perm],
                 a=w.a[:, perm], b=w.b[:, perm])
    assert np.allclose(oracle_lib.fstat(wp, tmpl)["twoF"], ref, rtol=1e-11, atol=1e-11)
    # detector order: swap the two detectors' blocks
    o = w.det_offset
    idx = np.concatenate([np.arange(o[1], o[2]), np.arange(o[0], o[1])])
    wd = replace(w, sft=w.sft[idx], t_start=w.t_start[idx], pos=w.pos[idx], vel=w.vel[idx],
                 a=w.a[:, idx], b=w.b[:, idx])
    assert np.allclose(oracle_lib.fstat(wd, tmpl)["twoF"], ref, rtol=1e-11, atol=1e-11)
    # common scaling of the antenna patterns
    ws = replace(w, a=(w.a.astype(np.float64) * 3.0), b=(w.b.astype(np.float64) * 3.0))
    assert np.allclose(oracle_lib.fstat(ws, tmpl)["twoF"], ref, rtol=1e-11, atol=1e-11)
    # a global phase rotation of every SFT
    rot = w.sft.astype(np.complex128) * np.exp(1j * 0.7)
    assert np.allclose(oracle_lib.fstat(w, tmpl, sft=rot)["twoF"], ref, rtol=1e-11, atol=1e-11)


# ------------------------------------------- P8: hand-derived single term ---
def _golden_workload(g):
    t = np.asarray(g["t_start"], dtype=np.float64)
    n_bins = 64
    k_first = g["kstar"] - 32
    rng = np.random.default_rng(2)
    sft = (rng.standard_normal((2, n_bins)) + 1j * rng.standard_normal((2, n_bins))).astype(np.complex64)
    for al in range(2):
        sft[al, g["kstar"] - k_first] = complex(*g["x_kstar"][al])
    return synth.Workload(name="golden", sft=sft, k_first=k_first, t_sft=g["t_sft"], t_start=t,
                          pos=np.zeros((2, 3)), vel=np.zeros((2, 3)), det_offset=np.array([0, 2], dtype=np.int32),
                          a=np.array([g["a"]], dtype=np.float32), b=np.array([g["b"]], dtype=np.float32),
                          sky=np.array([[0.0, 0.0, 1.0]]), f0=g["f0"], df=1.0 / g["t_sft"], n_f=1, fdot0=0.0,
                          dfdot=0.0, n_fd=1, t_ref=g["t_ref"], dterms=g["dterms"])


def test_golden_single_term(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "single_term_kappa0.json")))
    w = _golden_workload(g)
    r = oracle_lib.fstat(w, ([0], [0], [0]))
    assert r["twoF"][0] == pytest.approx(g["expected"]["twoF"], rel=1e-14)
    assert r["Fa"][0] == pytest.approx(complex(*g["expected"]["Fa"]), rel=1e-14)
    assert r["Fb"][0] == pytest.approx(complex(*g["expected"]["Fb"]), rel=1e-14)


def test_band_error(oracle_lib):
    """Exactly the bins [min k* - D + 1, max k* + D] suffice; one bin fewer on
    either side is a band error."""
    w = small_workload(41, injections=())
    s, i, j = oracle_lib.all_templates(w)
    k, _, _, _ = oracle_lib.bins(w, (s, i, j))
    lo, hi = int(k.min()) - w.dterms + 1, int(k.max()) + w.dterms
    c0, c1 = lo - w.k_first, hi - w.k_first + 1
    tight = replace(w, sft=w.sft[:, c0:c1], k_first=lo)
    oracle_lib.fstat(tight, (s, i, j))
    for cut in (replace(w, sft=w.sft[:, c0 + 1:c1], k_first=lo + 1), replace(w, sft=w.sft[:, c0:c1 - 1], k_first=lo)):
        with pytest.raises(ValueError, match="band"):
            oracle_lib.fstat(cut, (s, i, j))


# ------------------------------------------------ P9: toplist selection ---
def test_toplist_selection_definition():
    """Threshold, order by 2F descending, ties by smaller index, truncation."""
    import oracle
    v = np.array([5.0, 7.0, 7.0, 3.0, 9.0, 4.0, 7.0])
    idx, n = oracle.toplist(v, 4.0, 3)
    assert n == 6                                   # 5, 7, 7, 9, 4, 7 are >= 4
    assert list(idx) == [4, 1, 2]                   # 9, then the first two 7s by index
    idx, n = oracle.toplist(v, 7.5, 10)
    assert n == 1 and list(idx) == [4]              # fewer than k pass
    idx, n = oracle.toplist(v, 100.0, 3)
    assert n == 0 and len(idx) == 0


def test_toplist_brute_force_random():
    """Against a pairwise-comparison ranking on random arrays with ties."""
    import oracle
    rng = np.random.default_rng(11)
    for _ in range(20):
        v = rng.integers(0, 12, 40).astype(np.float64)
        thr, k = float(rng.integers(0, 12)), int(rng.integers(1, 15))
        idx, n = oracle.toplist(v, thr, k)
        cand = [t for t in range(len(v)) if v[t] >= thr]
        rank = {t: sum(1 for u in cand if v[u] > v[t] or (v[u] == v[t] and u < t)) for t in cand}
        expect = sorted(cand, key=lambda t: rank[t])[:k]
        assert n == len(cand) and list(idx) == expect
