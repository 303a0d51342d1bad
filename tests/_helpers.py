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
