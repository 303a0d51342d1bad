"""Workload recipes and physical input models (no demodulation arithmetic).

Units: times in GPS seconds, positions in light-seconds, velocities in units
of c, frequencies in Hz, SFT bin k <-> frequency k / T_sft.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

EPOCH = 8.0e8                       # GPS start of every synthetic data set
ORBIT_R = 499.005                   # light-seconds, 1 AU
ORBIT_OMEGA = 2.0 * math.pi / (365.25636 * 86400.0)
OBLIQUITY = math.radians(23.4393)
SIDEREAL_OMEGA = 2.0 * math.pi / 86164.0905

# Two synthetic interferometer sites: latitude, longitude, azimuth of arm 1
# (from north towards east), in degrees.  The second arm is 90 degrees on.
SITES = (
    (46.5, -119.4, 126.0),
    (30.6, -90.8, 198.0),
)


def quantise_time(t):
    """Round times to 2**-10 s so that sums and midpoints stay exact in FP64."""
    return np.round(np.asarray(t, dtype=np.float64) * 1024.0) / 1024.0


def orbit(t):
    """Circular orbit in equatorial coordinates: positions [n,3] (light-s) and
    velocities [n,3] (units of c) at GPS times t."""
    t = np.asarray(t, dtype=np.float64)
    th = ORBIT_OMEGA * (t - EPOCH) + 0.3
    ce, se = math.cos(OBLIQUITY), math.sin(OBLIQUITY)
    c, s = np.cos(th), np.sin(th)
    pos = ORBIT_R * np.stack([c, s * ce, s * se], axis=-1)
    vel = (ORBIT_R * ORBIT_OMEGA) * np.stack([-s, c * ce, c * se], axis=-1)
    return pos, vel


def sky_grid(n: int, *, offset: float = 0.5):
    """Fibonacci lattice of n unit vectors [n,3] (FP64), near-isotropic."""
    i = np.arange(n, dtype=np.float64) + offset
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ga = math.pi * (3.0 - math.sqrt(5.0))
    phi = ga * i
    v = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=-1)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _wave_frame(sky):
    """Two unit vectors xi, eta orthogonal to each sky direction."""
    n = np.asarray(sky, dtype=np.float64)
    alpha = np.arctan2(n[:, 1], n[:, 0])
    delta = np.arcsin(np.clip(n[:, 2], -1.0, 1.0))
    xi = np.stack([np.sin(alpha), -np.cos(alpha), np.zeros_like(alpha)], axis=-1)
    eta = np.stack([-np.sin(delta) * np.cos(alpha), -np.sin(delta) * np.sin(alpha), np.cos(delta)], axis=-1)
    return xi, eta


def antenna_patterns(site, sky, t_mid):
    """a, b [n_sky, n_sft] (float32) for a detector at `site` (latitude,
    longitude, arm azimuth in degrees) rotating with the Earth.  The detector
    tensor is d = (u u^T - v v^T)/2 with u, v the arm directions; a and b are
    its projections on the plus and cross polarisation tensors of the wave
    frame."""
    lat, lon, az = (math.radians(x) for x in site)
    ang = lon + SIDEREAL_OMEGA * (np.asarray(t_mid, dtype=np.float64) - EPOCH)   # [n_sft]
    east = np.stack([-np.sin(ang), np.cos(ang), np.zeros_like(ang)], axis=-1)
    north = np.stack([-math.sin(lat) * np.cos(ang), -math.sin(lat) * np.sin(ang),
                      np.full_like(ang, math.cos(lat))], axis=-1)
    u = math.cos(az) * north + math.sin(az) * east
    v = -math.sin(az) * north + math.cos(az) * east
    d = 0.5 * (u[:, :, None] * u[:, None, :] - v[:, :, None] * v[:, None, :])   # [n_sft,3,3]
    xi, eta = _wave_frame(sky)                                                   # [n_sky,3]
    dxi = np.einsum("tij,sj->sti", d, xi)
    deta = np.einsum("tij,sj->sti", d, eta)
    a = np.einsum("si,sti->st", xi, dxi) - np.einsum("si,sti->st", eta, deta)
    b = 2.0 * np.einsum("si,sti->st", xi, deta)
    return a.astype(np.float32), b.astype(np.float32)


def quantise_sfts(sft: np.ndarray, storage: str):
    """16-bit storage of complex64 SFTs with a per-SFT FP32 scale.

    Returns (stored, scale): `stored` is uint16 [n_sft, n_bins, 2] holding
    bfloat16 or float16 bit patterns of sft/scale, and x = scale * stored is
    the dequantised value.  scale = max|re,im| / 256 keeps float16 far from
    overflow and subnormals."""
    assert storage in ("bf16", "fp16")
    x = np.ascontiguousarray(sft).view(np.float32).reshape(sft.shape[0], sft.shape[1], 2)
    m = np.max(np.abs(x), axis=(1, 2)).astype(np.float32)
    scale = np.where(m > 0, m / np.float32(256.0), np.float32(1.0)).astype(np.float32)
    y = (x / scale[:, None, None]).astype(np.float32)
    if storage == "fp16":
        stored = y.astype(np.float16).view(np.uint16)
    else:
        u = y.view(np.uint32).astype(np.uint64)
        # round to nearest even on the upper 16 bits (inputs are finite)
        r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        stored = r.astype(np.uint16)
    return np.ascontiguousarray(stored), scale


def dequantise_16bit(stored: np.ndarray, scale: np.ndarray, storage: str) -> np.ndarray:
    """Exact FP64 values scale * stored of 16-bit SFT storage, as complex128."""
    if storage == "fp16":
        y = stored.view(np.float16).astype(np.float64)
    else:
        y = (stored.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    y = y * scale.astype(np.float64)[:, None, None]
    return y[..., 0] + 1j * y[..., 1]


@dataclasses.dataclass
class Injection:
    sky_index: int
    fdot_index: int
    f_index: int
    snr: float
    cos_iota: float
    psi: float
    phi0: float


@dataclasses.dataclass
class Workload:
    """One work unit: an SFT band of every detector plus a template grid."""
    name: str
    sft: Optional[np.ndarray]  # complex64 [n_sft, n_bins], or None when drawn on the device
    k_first: int               # absolute bin index of column 0
    t_sft: float
    t_start: np.ndarray        # float64 [n_sft]
    pos: np.ndarray            # float64 [n_sft, 3], light-s, at SFT midpoints
    vel: np.ndarray            # float64 [n_sft, 3], units of c
    det_offset: np.ndarray     # int32 [n_det + 1]
    a: np.ndarray              # float32 [n_sky, n_sft]
    b: np.ndarray              # float32 [n_sky, n_sft]
    sky: np.ndarray            # float64 [n_sky, 3]
    f0: float
    df: float
    n_f: int
    fdot0: float
    dfdot: float
    n_fd: int
    t_ref: float
    dterms: int
    injections: List[Injection] = dataclasses.field(default_factory=list)
    shape: Optional[tuple] = None  # (n_sft, n_bins) when `sft` is None (drawn on the device)

    @property
    def n_sft(self):
        return self.sft.shape[0] if self.sft is not None else self.shape[0]

    @property
    def n_bins(self):
        return self.sft.shape[1] if self.sft is not None else self.shape[1]

    @property
    def n_sky(self):
        return self.sky.shape[0]

    @property
    def n_det(self):
        return len(self.det_offset) - 1

    @property
    def n_templates(self):
        return self.n_sky * self.n_fd * self.n_f


def band_limits(f_lo, f_hi, fd_lo, fd_hi, t_mid, t_ref, rmax, vmax, t_sft, dterms, guard=2):
    """Bin range [k_first, k_last] that holds every frequency the signal model
    can reach: (f + fdot*tau)(1 + v.n) * T_sft for |r.n| <= rmax, |v.n| <= vmax,
    widened by the 2*Dterms window and a guard of a few bins."""
    taus = [float(np.min(t_mid)) - t_ref - rmax, float(np.max(t_mid)) - t_ref + rmax]
    vals = []
    for f in (f_lo, f_hi):
        for fd in (fd_lo, fd_hi):
            for tau in taus:
                for v in (-vmax, vmax):
                    vals.append((f + fd * tau) * (1.0 + v) * t_sft)
    k_first = int(math.floor(min(vals))) - dterms + 1 - guard
    k_last = int(math.floor(max(vals))) + dterms + guard
    return k_first, k_last


def _amplitudes(inj: Injection):
    ap = 0.5 * (1.0 + inj.cos_iota ** 2)
    ax = inj.cos_iota
    c2, s2 = math.cos(2 * inj.psi), math.sin(2 * inj.psi)
    e = complex(math.cos(inj.phi0), math.sin(inj.phi0))
    return e * complex(ap * c2, -ax * s2), e * complex(ap * s2, ax * c2)


def _inject(w: Workload, inj: Injection, sft: np.ndarray, rng_unused=None):
    """Add one CW signal to `sft` by sampling its complex (positive-frequency)
    waveform at n_bins points per SFT, heterodyned by k_first, and taking the
    DFT.  The per-SFT complex amplitude a*A + b*B is scaled so that
    2 * sum |a*A + b*B|^2 equals snr^2 for unit-variance noise bins."""
    n = w.sky[inj.sky_index]
    f = w.f0 + inj.f_index * w.df
    fd = w.fdot0 + inj.fdot_index * w.dfdot
    amp_a, amp_b = _amplitudes(inj)
    s = w.a[inj.sky_index].astype(np.float64) * amp_a + w.b[inj.sky_index].astype(np.float64) * amp_b
    rho2 = 2.0 * np.sum(np.abs(s) ** 2)
    s *= inj.snr / math.sqrt(rho2)
    nb = w.n_bins
    j = np.arange(nb, dtype=np.int64)
    het = ((w.k_first % nb) * j) % nb                       # exact k_first*j mod nb
    chunk = max(1, (1 << 22) // nb)                          # SFTs per vectorised block
    for a0 in range(0, w.n_sft, chunk):
        a1 = min(w.n_sft, a0 + chunk)
        tj = w.t_start[a0:a1, None] + j[None, :] * (w.t_sft / nb)
        r, _ = orbit(tj)
        tau = (tj - w.t_ref) + r @ n
        cyc = f * tau + 0.5 * fd * tau * tau
        cyc = cyc - np.floor(cyc) - het[None, :] / nb
        x = s[a0:a1, None] * np.exp(2j * np.pi * cyc)
        sft[a0:a1] += (np.fft.fft(x, axis=1) / nb).astype(np.complex64)


CONFIG_NAMES = {
    0: "plain-1det-32sft-256f-D16",
    1: "workunit-2det-1000sft-2000sky-8fd-3600f-D8",
}


def make_workload(name, *, seed, n_det, slots_per_det, keep_frac, jitter, t_sft, f0, n_f,
                  n_sky, n_fd, fdot_lo, fdot_hi, dterms, injections=(), sky_override=None,
                  noise=True, sites=SITES, epoch=EPOCH, t_ref=None):
    """General recipe.  Each detector has `slots_per_det` consecutive T_sft
    slots starting at `epoch`; a random `keep_frac` of them is kept (all if 1),
    and each kept start is jittered by U[0, jitter) s and quantised.  The
    reference time is the first SFT start unless `t_ref` is given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t_all, det_offset = [], [0]
    for d in range(n_det):
        slots = np.arange(slots_per_det)
        if keep_frac < 1.0:
            n_keep = int(round(keep_frac * slots_per_det))
            slots = np.sort(rng.choice(slots_per_det, size=n_keep, replace=False))
        t = epoch + slots * t_sft + rng.uniform(0.0, jitter, size=len(slots))
        t_all.append(quantise_time(t))
        det_offset.append(det_offset[-1] + len(slots))
    t_start = np.concatenate(t_all)
    t_mid = t_start + 0.5 * t_sft
    pos, vel = orbit(t_mid)
    sky = sky_grid(n_sky) if sky_override is None else np.asarray(sky_override, dtype=np.float64)
    a = np.empty((sky.shape[0], len(t_start)), dtype=np.float32)
    b = np.empty_like(a)
    for d in range(n_det):
        lo, hi = det_offset[d], det_offset[d + 1]
        a[:, lo:hi], b[:, lo:hi] = antenna_patterns(sites[d % len(sites)], sky, t_mid[lo:hi])
    df = 1.0 / t_sft
    dfdot = (fdot_hi - fdot_lo) / (n_fd - 1) if n_fd > 1 else 0.0
    t_ref = float(t_start.min()) if t_ref is None else float(t_ref)
    rmax = float(np.max(np.linalg.norm(pos, axis=1)))
    vmax = float(np.max(np.linalg.norm(vel, axis=1)))
    f_hi = f0 + (n_f - 1) * df
    k_first, k_last = band_limits(f0, f_hi, fdot_lo, fdot_lo + (n_fd - 1) * dfdot, t_mid, t_ref,
                                  rmax, vmax, t_sft, dterms)
    n_bins = k_last - k_first + 1
    n_sft = len(t_start)
    if noise == "device":
        sft = None              # shapes only: the noise is drawn on the GPU (synth.device)
    elif noise:
        z = rng.standard_normal((n_sft, n_bins, 2), dtype=np.float32) * np.float32(math.sqrt(0.5))
        sft = z.view(np.complex64).reshape(n_sft, n_bins).copy()
    else:
        sft = np.zeros((n_sft, n_bins), dtype=np.complex64)
    w = Workload(name=name, sft=sft, k_first=k_first, t_sft=t_sft, t_start=t_start, pos=pos, vel=vel,
                 det_offset=np.asarray(det_offset, dtype=np.int32), a=a, b=b, sky=sky, f0=f0, df=df,
                 n_f=n_f, fdot0=fdot_lo, dfdot=dfdot, n_fd=n_fd, t_ref=t_ref, dterms=dterms,
                 shape=(n_sft, n_bins))
    for inj in injections:
        if isinstance(inj, dict):
            inj = Injection(**inj)
        elif not isinstance(inj, Injection):
            s_i, fd_i, f_i, snr = inj
            inj = Injection(int(s_i), int(fd_i), int(f_i), float(snr), float(rng.uniform(-1, 1)),
                            float(rng.uniform(0, math.pi)), float(rng.uniform(0, 2 * math.pi)))
        _inject(w, inj, w.sft)
        w.injections.append(inj)
    return w


def make_config(idx: int, *, seed: Optional[int] = None, **over):
    """Workload recipes.  Index 0 is the small single-detector case, index 1
    the work-unit-shaped case; keyword overrides shrink a recipe for tests."""
    seed = 1000 + idx if seed is None else seed
    if idx == 0:
        p = dict(n_det=1, slots_per_det=32, keep_frac=1.0, jitter=60.0, t_sft=1800.0, f0=100.0,
                 n_f=256, n_sky=1, n_fd=1, fdot_lo=0.0, fdot_hi=0.0, dterms=16,
                 sky_override=[[math.cos(0.5) * math.cos(1.0), math.cos(0.5) * math.sin(1.0), math.sin(0.5)]],
                 injections=[(0, 0, 128, 10.0)])
    elif idx == 1:
        p = dict(n_det=2, slots_per_det=1667, keep_frac=0.6, jitter=0.0, t_sft=1800.0, f0=1000.0,
                 n_f=3600, n_sky=2000, n_fd=8, fdot_lo=-1.0e-9, fdot_hi=0.0, dterms=8,
                 injections=[(137, 3, 500, 10.0), (901, 7, 1800, 14.0), (1402, 0, 2700, 20.0),
                             (1999, 5, 3400, 12.0)])
    else:
        raise ValueError(f"no recipe {idx}")
    p.update(over)
    name = over.pop("name", None) or CONFIG_NAMES[idx] + ("" if not over else "-custom")
    p.pop("name", None)
    return make_workload(name, seed=seed, **p)


SEGMENT_NAMES = {
    20: "semicoherent-20seg-2det-2000sft-2000sky-8fd-3600f-D8",
}


def make_segments(n_seg: int, *, seed: int, seg_slots: int, gap_slots: int = 0, name: Optional[str] = None,
                  injections=(), **kw):
    """Consecutive time segments of one observation for the semi-coherent
    combination: segment k covers `seg_slots` T_sft slots per detector starting
    (seg_slots + gap_slots) * k slots after EPOCH, with its own noise and gaps
    (the remaining keywords as in make_workload).  All segments share the
    template grid and the reference time t_ref = EPOCH, so a template names
    the same signal in each of them.  Each injection (sky, fdot, f index, snr)
    gets one set of amplitude parameters and is added to every segment with
    that phase model, scaled to SNR `snr` in each segment."""
    rng = np.random.Generator(np.random.PCG64(seed))
    injs = []
    for inj in injections:
        s_i, fd_i, f_i, snr = inj
        injs.append(Injection(int(s_i), int(fd_i), int(f_i), float(snr), float(rng.uniform(-1, 1)),
                              float(rng.uniform(0, math.pi)), float(rng.uniform(0, 2 * math.pi))))
    t_sft = kw["t_sft"]
    segs = []
    for k in range(n_seg):
        segs.append(make_workload(f"{name or 'segments'}-{k}", seed=seed * 1000 + k, slots_per_det=seg_slots,
                                  epoch=EPOCH + k * (seg_slots + gap_slots) * t_sft, t_ref=EPOCH,
                                  injections=injs, **kw))
    return segs


def make_segment_config(n_seg: int = 20, *, seed: int = 2020, **over):
    """The work-unit-shaped case (2 detectors, 2000 sky points x 8
    spindowns x 3600 frequencies at 1000 Hz, Dterms 8, 60 % duty cycle) as
    `n_seg` consecutive segments whose SFT counts add up to that case's:
    1667 / n_seg slots per detector each (about 100 kept SFTs per segment for
    20 segments), four signals at SNR 4 to 7 per segment."""
    p = dict(n_det=2, seg_slots=1667 // n_seg, keep_frac=0.6, jitter=0.0, t_sft=1800.0, f0=1000.0, n_f=3600,
             n_sky=2000, n_fd=8, fdot_lo=-1.0e-9, fdot_hi=0.0, dterms=8,
             injections=[(137, 3, 500, 4.0), (901, 7, 1800, 5.0), (1402, 0, 2700, 7.0), (1999, 5, 3400, 6.0)])
    p.update(over)
    name = SEGMENT_NAMES.get(n_seg) if not over else None
    return make_segments(n_seg, seed=seed, name=name or f"semicoherent-{n_seg}seg-custom", **p)


BATCH_NAMES = {
    3: "batch-64wu-200to2000sft-900to7200bins",
    4: "large-256wu-2x1000to4000sft-14400bins-bf16",
}


def _make_workload_kw(kw):
    return make_workload(**kw)


def make_batch(idx: int = 3, *, seed: Optional[int] = None, n_wu: Optional[int] = None, scale: float = 1.0,
               noise: bool = True, workers: int = 1):
    """Many work units with uneven shapes.  Recipe 3: 64 work units, each with
    U{200..2000} SFTs split over 2 detectors (all slots kept, jitter 60 s),
    a band of U{900..7200} template bins starting at U[50, 1500] Hz,
    U{500..4000} sky points x U{4..16} spindowns in [-1e-9, 0], Dterms 8 or
    16, one injected signal.  `scale` < 1 shrinks SFT counts, bands and sky
    points proportionally (for tests); `n_wu` truncates the list."""
    if idx == 4:
        return _make_large_batch(seed=seed, n_wu=n_wu, scale=scale, workers=workers)
    if idx != 3:
        raise ValueError(f"no batch recipe {idx}")
    seed = 1000 + idx if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    total = 64 if n_wu is None else n_wu
    kws = []
    for u in range(total):
        n_sft = max(4, int(round(rng.integers(200, 2001) * scale)))
        band = max(64, int(round(rng.integers(900, 7201) * scale)))
        f0 = float(rng.uniform(50.0, 1500.0))
        f0 = round(f0 * 1800.0) / 1800.0
        n_sky = max(1, int(round(rng.integers(500, 4001) * scale)))
        n_fd = int(rng.integers(4, 17))
        dterms = int(rng.choice([8, 16]))
        inj = [(int(rng.integers(0, n_sky)), int(rng.integers(0, n_fd)), int(rng.integers(band // 4, 3 * band // 4)),
                float(rng.uniform(10.0, 20.0)))]
        kws.append(dict(name=f"{BATCH_NAMES[idx]}-{u}", seed=seed * 1000 + u, n_det=2,
                        slots_per_det=(n_sft + 1) // 2, keep_frac=1.0, jitter=60.0, t_sft=1800.0, f0=f0, n_f=band,
                        n_sky=n_sky, n_fd=n_fd, fdot_lo=-1.0e-9, fdot_hi=0.0, dterms=dterms, injections=inj,
                        noise=noise))
    if workers > 1 and total > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, total)) as ex:
            return list(ex.map(_make_workload_kw, kws))
    return [make_workload(**kw) for kw in kws]


def _make_large_batch(*, seed=None, n_wu=None, scale=1.0, workers=1):
    """Recipe 4 (shapes and geometry; the SFT noise is drawn on the device by
    synth.device.draw_noise_16bit): 256 work units, 2 detectors with
    U{1000..4000} SFTs each (all slots kept, jitter 60 s), 14400 template bins
    from U[50, 1500] Hz, 10000 sky points of one Fibonacci grid split evenly
    over the work units (39 or 40 each) x 32 spindowns in [-1e-9, 0],
    Dterms 16, no injection.  `scale` < 1 shrinks SFT counts and bands."""
    seed = 1004 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    total = 256 if n_wu is None else n_wu
    grid = sky_grid(10000)
    splits = np.array_split(np.arange(10000), 256)
    kws = []
    for u in range(total):
        per_det = max(2, int(round(rng.integers(1000, 4001) * scale)))
        band = max(64, int(round(14400 * scale)))
        f0 = round(float(rng.uniform(50.0, 1500.0)) * 1800.0) / 1800.0
        kws.append(dict(name=f"{BATCH_NAMES[4]}-{u}", seed=seed * 1000 + u, n_det=2, slots_per_det=per_det,
                        keep_frac=1.0, jitter=60.0, t_sft=1800.0, f0=f0, n_f=band, n_sky=len(splits[u]), n_fd=32,
                        fdot_lo=-1.0e-9, fdot_hi=0.0, dterms=16, injections=(), noise="device",
                        sky_override=grid[splits[u]]))
    if workers > 1 and total > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, total)) as ex:
            return list(ex.map(_make_workload_kw, kws))
    return [make_workload(**kw) for kw in kws]
