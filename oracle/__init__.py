"""FP64 CPU oracle for the F-statistic demodulation -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain C implementation in
`fstat_oracle.c` (built with gcc, -ffp-contract=off, OpenMP over templates)
and shares no code with the GPU library.  See `fstat_oracle.c` for the
formulas and the passages of the paper they follow (Listing 1, Section 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fstat_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

OK, E_ARG, E_BAND = 0, -1, -2


def build(force: bool = True) -> str:
    """Compile the oracle shared library in-tree."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _WU(ctypes.Structure):
    _fields_ = [
        ("n_sft", ctypes.c_int), ("n_bins", ctypes.c_int), ("k_first", ctypes.c_int64),
        ("t_sft", ctypes.c_double), ("sft", ctypes.c_void_p), ("t_start", ctypes.c_void_p),
        ("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("n_sky", ctypes.c_int),
        ("sky", ctypes.c_void_p), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
        ("f0", ctypes.c_double), ("df", ctypes.c_double), ("n_f", ctypes.c_int),
        ("fdot0", ctypes.c_double), ("dfdot", ctypes.c_double), ("n_fd", ctypes.c_int),
        ("t_ref", ctypes.c_double), ("dterms", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_fstat.argtypes = [ctypes.POINTER(_WU), ctypes.c_int, P, P, P, P, P, P, ctypes.c_int, P]
        lib.oracle_fstat.restype = ctypes.c_int
        lib.oracle_bins.argtypes = [ctypes.POINTER(_WU), ctypes.c_int, P, P, P, P, P, P, P]
        lib.oracle_bins.restype = ctypes.c_int
        lib.oracle_abc.argtypes = [ctypes.POINTER(_WU), ctypes.c_int, P, P, P, P]
        lib.oracle_abc.restype = None
        lib.oracle_sinc.argtypes = [ctypes.c_double]
        lib.oracle_sinc.restype = ctypes.c_double
        lib.oracle_window_weights.argtypes = [ctypes.c_double, ctypes.c_int, P]
        lib.oracle_window_weights.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Packed:
    """Keeps the FP64 copies alive while the C struct points at them."""

    def __init__(self, w, sft: Optional[np.ndarray]):
        x = w.sft if sft is None else sft
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
        self.sft = x.view(np.float64)
        self.t_start = np.ascontiguousarray(w.t_start, dtype=np.float64)
        self.pos = np.ascontiguousarray(w.pos, dtype=np.float64)
        self.vel = np.ascontiguousarray(w.vel, dtype=np.float64)
        self.sky = np.ascontiguousarray(w.sky, dtype=np.float64)
        self.a = np.ascontiguousarray(w.a, dtype=np.float64)
        self.b = np.ascontiguousarray(w.b, dtype=np.float64)
        self.s = _WU(int(x.shape[0]), int(x.shape[1]), int(w.k_first), float(w.t_sft), _p(self.sft).value,
                     _p(self.t_start).value, _p(self.pos).value, _p(self.vel).value, int(self.sky.shape[0]),
                     _p(self.sky).value, _p(self.a).value, _p(self.b).value, float(w.f0), float(w.df), int(w.n_f),
                     float(w.fdot0), float(w.dfdot), int(w.n_fd), float(w.t_ref), int(w.dterms))


def all_templates(w, sky_indices=None):
    """(sky, fdot, f) index arrays of every template of the listed sky points,
    in output order [sky][fdot][f]."""
    sk = np.arange(w.n_sky) if sky_indices is None else np.asarray(sky_indices)
    s, i, j = np.meshgrid(sk, np.arange(w.n_fd), np.arange(w.n_f), indexing="ij")
    return (s.ravel().astype(np.int32), i.ravel().astype(np.int32), j.ravel().astype(np.int32))


class Prepared:
    """A work unit converted once to the oracle's FP64 layout, for repeated calls."""

    def __init__(self, w, sft: Optional[np.ndarray] = None):
        self.w = w
        self.packed = _Packed(w, sft)

    def fstat(self, templates=None, nthreads: Optional[int] = None):
        return fstat(self.w, templates, nthreads=nthreads, _packed=self.packed)


def fstat(w, templates=None, *, sft: Optional[np.ndarray] = None, nthreads: Optional[int] = None, _packed=None):
    """2F (FP64), Fa, Fb (complex128) of the listed templates.  `sft` replaces
    the workload's SFT values (e.g. with exactly dequantised 16-bit storage).
    Raises ValueError naming the first template whose window leaves the band."""
    lib = _load()
    pk = _packed if _packed is not None else _Packed(w, sft)
    ts, ti, tj = all_templates(w) if templates is None else (np.ascontiguousarray(t, dtype=np.int32) for t in templates)
    n = len(ts)
    twoF = np.empty(n, dtype=np.float64)
    fa = np.empty((n, 2), dtype=np.float64)
    fb = np.empty((n, 2), dtype=np.float64)
    bad = ctypes.c_int(-1)
    nthreads = nthreads or min(16, os.cpu_count() or 1)
    rc = lib.oracle_fstat(ctypes.byref(pk.s), n, _p(ts), _p(ti), _p(tj), _p(twoF), _p(fa), _p(fb), nthreads,
                          ctypes.cast(ctypes.pointer(bad), ctypes.c_void_p))
    if rc == E_BAND:
        raise ValueError(f"band: window of template {bad.value} leaves the stored band")
    if rc != OK:
        raise ValueError(f"oracle error {rc}")
    return {"twoF": twoF, "Fa": fa[:, 0] + 1j * fa[:, 1], "Fb": fb[:, 0] + 1j * fb[:, 1],
            "templates": (ts, ti, tj)}


def bins(w, templates):
    """k* (int64), kappa, frac(phi), Dphi of every (template, SFT), [n_tmpl, n_sft]."""
    lib = _load()
    pk = _Packed(w, np.zeros((w.n_sft, 1), dtype=np.complex128))   # bins do not read SFT values
    ts, ti, tj = (np.ascontiguousarray(t, dtype=np.int32) for t in templates)
    n, m = len(ts), w.n_sft
    k = np.empty((n, m), dtype=np.int64)
    kap = np.empty((n, m), dtype=np.float64)
    ph = np.empty((n, m), dtype=np.float64)
    dp = np.empty((n, m), dtype=np.float64)
    lib.oracle_bins(ctypes.byref(pk.s), n, _p(ts), _p(ti), _p(tj), _p(k), _p(kap), _p(ph), _p(dp))
    return k, kap, ph, dp


def abc(w, s: int):
    lib = _load()
    pk = _Packed(w, None)
    out = [ctypes.c_double() for _ in range(4)]
    lib.oracle_abc(ctypes.byref(pk.s), int(s), *[ctypes.cast(ctypes.pointer(o), ctypes.c_void_p) for o in out])
    return tuple(o.value for o in out)


def sinc(x: float) -> float:
    return _load().oracle_sinc(float(x))


def window_weights(kappa: float, dterms: int) -> np.ndarray:
    out = np.empty(2 * dterms, dtype=np.float64)
    _load().oracle_window_weights(float(kappa), int(dterms), _p(out))
    return out


def toplist(twoF, threshold: float, k: int):
    """Toplist of a work unit from its 2F over all templates, given in linear
    template order ((sky * n_fd + fdot) * n_f + f): the indices of the k
    largest 2F among those >= threshold, largest first, equal 2F by smaller
    index first; and the number of templates >= threshold.  A plain
    selection by full sort."""
    v = np.asarray(twoF, dtype=np.float64).ravel()
    idx = np.nonzero(v >= threshold)[0]
    order = np.lexsort((idx, -v[idx]))          # primary key -2F, then index
    return idx[order[:k]], len(idx)


def semicoherent(segs, templates=None, *, sfts=None, nthreads: Optional[int] = None):
    """Semi-coherent statistic of the listed templates: the sum over the
    time segments `segs` (work units sharing one template grid and reference
    time) of each segment's coherent 2F, in FP64.  The paper's client
    combines per-segment F-statistics in a second, incoherent stage
    (Section 2) without describing it; the plain sum of 2F over segments is
    the reading taken here.  `sfts` optionally replaces each segment's SFT
    values."""
    total = None
    for k, w in enumerate(segs):
        r = fstat(w, templates, sft=None if sfts is None else sfts[k], nthreads=nthreads)
        total = r["twoF"].copy() if total is None else total + r["twoF"]
        templates = r["templates"]
    return {"twoF": total, "templates": templates}


class _Earth(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("t0", "orbit_radius", "orbit_rate", "orbit_phase", "obliquity",
                                               "earth_radius", "sidereal_rate", "sidereal_phase")]


class _Site(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("lat", "lon", "az_x", "az_y")]


def detector_inputs(earth: dict, sites, t_mid, site_of_sft, sky):
    """Detector positions r [n_sft, 3] (light-s), velocities v [n_sft, 3]
    (units of c) and antenna-pattern factors a, b [n_sky, n_sft], all FP64,
    from the orbit/rotation model `earth` (keys of _Earth), the sites
    (lat, lon, az_x, az_y in radians), SFT midpoints and sky directions.  See
    oracle_detector_inputs in fstat_oracle.c for the formulas."""
    lib = _load()
    if not hasattr(lib, "_det_ready"):
        P = ctypes.c_void_p
        lib.oracle_detector_inputs.argtypes = [ctypes.POINTER(_Earth), ctypes.c_int, P, ctypes.c_int, P, P,
                                               ctypes.c_int, P, P, P, P, P]
        lib.oracle_detector_inputs.restype = ctypes.c_int
        lib._det_ready = True
    e = _Earth(*[float(earth[k]) for k, _ in _Earth._fields_])
    st = (_Site * len(sites))(*[_Site(*map(float, x)) for x in sites])
    t = np.ascontiguousarray(t_mid, dtype=np.float64)
    idx = np.ascontiguousarray(site_of_sft, dtype=np.int32)
    n = np.ascontiguousarray(sky, dtype=np.float64).reshape(-1, 3)
    pos = np.empty((len(t), 3))
    vel = np.empty((len(t), 3))
    a = np.empty((len(n), len(t)))
    b = np.empty((len(n), len(t)))
    ptr = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    rc = lib.oracle_detector_inputs(ctypes.byref(e), len(sites), ctypes.cast(st, ctypes.c_void_p), len(t), ptr(t),
                                    ptr(idx), len(n), ptr(n), ptr(pos), ptr(vel), ptr(a), ptr(b))
    if rc != OK:
        raise ValueError(f"oracle_detector_inputs: code {rc}")
    return pos, vel, a, b
