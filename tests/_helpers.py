"""Helpers shared by the tests: small custom workloads and the 2F error metric."""
import dataclasses
import math

import numpy as np

import synth


def small_workload(seed=7, *, n_det=2, slots=24, keep=0.75, n_sky=6, n_fd=3, n_f=200, f0=400.0,
                   dterms=8, fdot_lo=-2e-9, fdot_hi=0.0, injections=((2, 1, 90, 12.0),), noise=True,
                   jitter=60.0):
    return synth.make_workload(f"small-{seed}", seed=seed, n_det=n_det, slots_per_det=slots, keep_frac=keep,
                               jitter=jitter, t_sft=1800.0, f0=f0, n_f=n_f, n_sky=n_sky, n_fd=n_fd,
                               fdot_lo=fdot_lo, fdot_hi=fdot_hi, dterms=dterms, injections=injections,
                               noise=noise)


def replace(w, **kw):
    return dataclasses.replace(w, **kw)


def twoF_error(gpu, ref, floor=4.0):
    """Normalised 2F error |2F_gpu - 2F_ref| / max(2F_ref, floor)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(gpu - ref) / np.maximum(ref, floor)


def kernel_power_loss(kappa, dterms):
    """1 - sum_{m=-D}^{D-1} sinc^2(kappa + m) in closed form via the trigamma
    function: sum over all m of 1/(kappa+m)^2 is pi^2 / sin^2(pi kappa)."""
    from scipy.special import polygamma
    kappa = np.asarray(kappa, dtype=np.float64)
    s2 = np.sin(np.pi * kappa) ** 2 / np.pi ** 2
    return s2 * (polygamma(1, kappa + dterms) + polygamma(1, dterms + 1.0 - kappa))


def slice_edge_workload(coef, side):
    """A spindown step chosen so that the bound on how far D-hat-phi moves
    across a tile of 256 frequencies x 8 spindowns sits at the LDS slice's
    capacity (296 bins with FP32 coefficients, 384 with FP16): `in` about 5
    bins inside, where the kernel without the global-memory path runs and
    every window must still be in its slice; `out` half a bin beyond, where
    the kernel with that path runs and almost every SFT still takes the LDS
    path.  tau and Tdot follow their definitions (arrival-time offset and its
    derivative at the SFT midpoints).  Spindowns: 12 with FP16 coefficients
    (blocks of 8 and 4), 16 with FP32 ones, which run as two blocks of 8 (a
    block of 16 would need a slice twice as wide as the edge)."""
    n_fd = 12 if coef == "f16" else 16
    base = dict(n_det=2, slots=23, keep=0.85, n_sky=3, n_f=700, dterms=8, injections=((1, 5, 333, 15.0),))
    w = small_workload(310, n_fd=n_fd, fdot_lo=-1e-9, **base)
    tau = (w.t_start + 0.5 * w.t_sft - w.t_ref)[None, :] + w.sky @ w.pos.T
    p = (1.0 + w.sky @ w.vel.T) * w.t_sft
    max_tau, max_p = float(np.abs(tau).max()), float(p.max())
    cap = 384 if coef == "f16" else 296
    spread = cap - 9 + 0.01 if side == "in" else cap - 7 + 0.5
    dfdot = (spread / max_p - 255 * w.df) / (7 * max_tau)
    assert dfdot > 0
    w = small_workload(310, n_fd=n_fd, fdot_lo=-(n_fd - 1) * dfdot, **base)
    assert math.isclose(w.dfdot, dfdot, rel_tol=1e-9)
    width = 262 + math.ceil(spread - 255)
    assert (width <= cap) == (side == "in")
    return w


def sft_block_workloads():
    """Three units of 1100, 600 and 300 SFTs (5, 3 and 2 launches of the
    batched form's default 256 SFTs; 3, 2 and 1 of 512) with 9 spindowns
    (blocks of two sizes: 5 + 4 with FP32 coefficients, 8 + 4 with FP16)."""
    return [small_workload(700 + k, n_det=2, slots=s, keep=1.0, n_sky=2, n_fd=9, n_f=300, dterms=8,
                           injections=((1, 4, 150, 12.0),)) for k, s in enumerate([550, 300, 150])]


def kappa_edge_workload(edge, seed=820, n_fd=9):
    """A work unit whose every (template, SFT) pair sits at an edge of the
    Dirichlet offset: kappa = 0 exactly (edge "zero") or kappa = 1 - 2^-34
    (edge "one").  T_sft = 1024 s and df = 1/1024 Hz are powers of two, the
    detector velocity is zero (Tdot = 1, so P = T exactly) and every spindown
    is 0 (q = 0), so Dphi = 1024 f0 + j exactly: f0 = 400 Hz makes it an
    integer, and f0 one ulp of 400 below 400 (2^-44 Hz) puts it 2^-34 below
    one.  The positions stay on the orbit (the phase is generic)."""
    f0 = 400.0 if edge == "zero" else 400.0 - 2.0 ** -44
    w = synth.make_workload(f"kappa-{edge}", seed=seed, n_det=2, slots_per_det=12, keep_frac=1.0, jitter=60.0,
                            t_sft=1024.0, f0=f0, n_f=300, n_sky=3, n_fd=n_fd, fdot_lo=0.0, fdot_hi=0.0, dterms=8,
                            injections=())
    return replace(w, vel=np.zeros_like(w.vel))
