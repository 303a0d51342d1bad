"""Seeded synthetic inputs for the F-statistic demodulation.

This module makes the detector-side data that both the FP64 oracle and the
GPU library consume: SFT timestamps, a circular Earth orbit (positions and
velocities at SFT midpoints), antenna-pattern factors a(t), b(t) for fixed
synthetic detector sites, a Fibonacci sky grid, complex Gaussian noise SFTs
and continuous-wave signals injected by time-domain synthesis followed by a
DFT.  It holds none of the demodulation arithmetic (no bin selection, no
Dirichlet weights, no Fa/Fb/2F): the signal model is the physical phase
Phi(t) = f*tau + fdot*tau^2/2 with tau = t - t_ref + r(t).n, evaluated at
every sample, and each SFT is the discrete Fourier transform of the samples.

The paper describes the F-statistic loop over a frequency band, detectors
and SFTs (Listing 1, Section 2) and times two Einstein@Home workloads
(Section 3) whose contents are not published; the recipes here stand in for
them with the shapes stated in `CONFIGS`.
"""
from .workloads import (  # noqa: F401
    Workload, Injection, CONFIG_NAMES, make_config, make_workload, orbit, sky_grid,
    antenna_patterns, SITES, band_limits, quantise_time, dequantise_16bit,
    quantise_sfts, EPOCH, make_batch, BATCH_NAMES, make_segments, make_segment_config, SEGMENT_NAMES,
)
