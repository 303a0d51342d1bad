"""Python binding of libfstat (MI355X F-statistic demodulation).

Argument marshalling only: every step of the computation runs in the HIP
kernels of `csrc/`, behind the C-ABI declared in `include/fstat.h`.  torch
tensors provide device memory and streams.  The functions keep the C names.

A work unit is any object with the attributes of `fstat_wu` (see
`WorkUnit`): device tensors for the arrays and Python numbers for the
scalars.  Outputs are an object with `twoF` and optional `fa`, `fb` tensors.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libfstat.so")

FSTAT_OK = 0
FSTAT_E_ARG = -1
FSTAT_E_BAND = -2
FSTAT_E_SIZE = -3
FSTAT_E_NOMEM = -4
FSTAT_E_DEVICE = -5
FSTAT_E_UNSUPPORTED = -6

FSTAT_STORAGE_C64 = 0
FSTAT_STORAGE_BF16 = 1
FSTAT_STORAGE_FP16 = 2
FSTAT_PHASE_FP64 = 0
FSTAT_PHASE_SPLIT_FP32 = 1
FSTAT_KERNEL_AUTO = 0
FSTAT_KERNEL_DIRECT = 1
FSTAT_KERNEL_INTERP = 2
FSTAT_FLAG_NO_GRAPH = 1
FSTAT_FLAG_COEF16 = 2

STORAGE = {"c64": FSTAT_STORAGE_C64, "bf16": FSTAT_STORAGE_BF16, "fp16": FSTAT_STORAGE_FP16}
KERNELS = {"auto": FSTAT_KERNEL_AUTO, "direct": FSTAT_KERNEL_DIRECT, "interp": FSTAT_KERNEL_INTERP}
PHASES = {"fp64": FSTAT_PHASE_FP64, "split": FSTAT_PHASE_SPLIT_FP32}

# Every entry point include/fstat.h declares.
EXPORTS = ("fstat_plan_create", "fstat_compute", "fstat_batch_compute", "fstat_bins", "fstat_autotune",
           "fstat_last_kernel_ms", "fstat_plan_destroy", "fstat_strerror", "fstat_last_error",
           "fstat_detector_inputs", "fstat_semicoherent", "fstat_compute_noalloc", "fstat_interp_slice",
           "fstat_last_tile", "fstat_spindown_split", "fstat_sky_pairs")
LAST_TILE_LEN = 13                    # FSTAT_LAST_TILE_LEN
NOALLOC_SCRATCH_BYTES = 128 << 20     # FSTAT_NOALLOC_SCRATCH_BYTES


class FstatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class fstat_desc(ctypes.Structure):
    _fields_ = [("max_sft", ctypes.c_int64), ("max_bins", ctypes.c_int64), ("max_sky", ctypes.c_int64),
                ("max_fd", ctypes.c_int64), ("max_f", ctypes.c_int64), ("max_dterms", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("phase_mode", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("device", ctypes.c_int32), ("max_cands", ctypes.c_int64)]


class fstat_wu(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("det_offset", ctypes.c_void_p), ("n_sft", ctypes.c_int64),
                ("n_bins", ctypes.c_int64),
                ("k_first", ctypes.c_int64), ("t_sft", ctypes.c_double), ("sft", ctypes.c_void_p),
                ("sft_scale", ctypes.c_void_p), ("t_start", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("vel", ctypes.c_void_p), ("n_sky", ctypes.c_int64), ("sky", ctypes.c_void_p),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("f0", ctypes.c_double), ("df", ctypes.c_double),
                ("n_f", ctypes.c_int64), ("fdot0", ctypes.c_double), ("dfdot", ctypes.c_double),
                ("n_fd", ctypes.c_int64), ("t_ref", ctypes.c_double), ("dterms", ctypes.c_int32)]


class fstat_site(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("lat", "lon", "az_x", "az_y")]


class fstat_earth(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("t0", "orbit_radius", "orbit_rate", "orbit_phase", "obliquity",
                                               "earth_radius", "sidereal_rate", "sidereal_phase")]


class fstat_out(ctypes.Structure):
    _fields_ = [("twoF", ctypes.c_void_p), ("fa", ctypes.c_void_p), ("fb", ctypes.c_void_p),
                ("top_k", ctypes.c_int32), ("threshold", ctypes.c_float), ("top", ctypes.c_void_p),
                ("n_above", ctypes.c_void_p)]


_lib = None
_PLAN_STORAGE = {}        # plan handle value -> SFT storage of its descriptor


def _storage_of(plan) -> Optional[str]:
    v = getattr(plan, "value", plan)
    return _PLAN_STORAGE.get(v)


def load_library(path: str = LIB_PATH):
    """Load libfstat.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_0904_1826_amd.build`")
    lib = ctypes.CDLL(path)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.fstat_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(fstat_desc)]
    lib.fstat_plan_create.restype = ctypes.c_int
    lib.fstat_compute.argtypes = [P, ctypes.POINTER(fstat_wu), ctypes.POINTER(fstat_out), P]
    lib.fstat_compute.restype = ctypes.c_int
    lib.fstat_compute_noalloc.argtypes = [P, ctypes.POINTER(fstat_wu), ctypes.POINTER(fstat_out), P]
    lib.fstat_compute_noalloc.restype = ctypes.c_int
    lib.fstat_interp_slice.argtypes = [ctypes.c_double, ctypes.c_double, I32, I32, I32, ctypes.c_double,
                                       ctypes.c_double, ctypes.POINTER(I32)]
    lib.fstat_interp_slice.restype = I32
    lib.fstat_batch_compute.argtypes = [P, ctypes.POINTER(fstat_wu), I32, ctypes.POINTER(fstat_out), P]
    lib.fstat_batch_compute.restype = ctypes.c_int
    lib.fstat_semicoherent.argtypes = [P, ctypes.POINTER(fstat_wu), I32, ctypes.POINTER(fstat_out), P]
    lib.fstat_semicoherent.restype = ctypes.c_int
    lib.fstat_bins.argtypes = [P, ctypes.POINTER(fstat_wu), I64, P, P, P, P, P, P, P, P]
    lib.fstat_bins.restype = ctypes.c_int
    lib.fstat_autotune.argtypes = [P, ctypes.POINTER(fstat_wu), ctypes.POINTER(fstat_out), P, ctypes.c_char_p]
    lib.fstat_autotune.restype = ctypes.c_int
    lib.fstat_last_kernel_ms.argtypes = [P]
    lib.fstat_last_kernel_ms.restype = ctypes.c_double
    lib.fstat_last_tile.argtypes = [P, ctypes.POINTER(I32)]
    lib.fstat_last_tile.restype = ctypes.c_int
    lib.fstat_spindown_split.argtypes = [I64, I32, I32, I32, ctypes.POINTER(I64)]
    lib.fstat_spindown_split.restype = ctypes.c_int
    D = ctypes.c_double
    lib.fstat_sky_pairs.argtypes = [I64, ctypes.POINTER(D), D, D, I64, D, D, I64, D, D, D, D, D,
                                    ctypes.POINTER(I32), ctypes.POINTER(I64)]
    lib.fstat_sky_pairs.restype = I32
    lib.fstat_plan_destroy.argtypes = [P]
    lib.fstat_plan_destroy.restype = None
    lib.fstat_strerror.argtypes = [ctypes.c_int]
    lib.fstat_strerror.restype = ctypes.c_char_p
    lib.fstat_last_error.argtypes = [P]
    lib.fstat_last_error.restype = ctypes.c_char_p
    lib.fstat_detector_inputs.argtypes = [P, ctypes.POINTER(fstat_earth), I32, ctypes.POINTER(fstat_site), I64, P, P,
                                          I64, P, P, P, P, P, P]
    lib.fstat_detector_inputs.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    """Address of a tensor for the C-ABI, which takes contiguous device arrays
    only: a strided view or a host tensor is refused here, before a kernel
    could read it as device memory.  None passes through (the library reports
    a missing required array itself)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("the library takes contiguous tensors only")
    if not t.is_cuda:
        raise ValueError(f"the library takes device tensors only, got one on {t.device}")
    return t.data_ptr()


# ------------------------------------------------------------ array checks
# The kernels index every array by the sizes of the work unit, so each array's
# element type and element count are checked against those sizes before any
# call: a short or mistyped array would otherwise be read or written out of
# bounds on the device.  The checks look only at dtype and shape.
_ELEM = {"f32": ("float32",), "f64": ("float64",), "i32": ("int32",), "i64": ("int64",),
         "u16pair": ("int16", "uint16")}


def _dtype_name(t) -> str:
    return str(t.dtype).replace("torch.", "")


def _numel(t) -> int:
    n = 1
    for d in t.shape:
        n *= int(d)
    return n


def check_array(name: str, t, kind: str, numel: int, *, at_least: bool = False) -> None:
    """Raise ValueError unless `t` has element type `kind` ("f32", "f64", "i32",
    "i64", "u16pair") and exactly `numel` elements (at least, if at_least).
    None passes: the library reports a missing required array itself."""
    if t is None:
        return
    dt = _dtype_name(t)
    if dt not in _ELEM[kind]:
        raise ValueError(f"{name}: element type {dt}, expected {' or '.join(_ELEM[kind])}")
    n = _numel(t)
    if (n < numel) if at_least else (n != numel):
        raise ValueError(f"{name}: {n} elements, expected {'at least ' if at_least else ''}{numel}")


def check_work_unit(w, storage: str = "c64") -> None:
    """Element types and counts of a work unit's arrays against its sizes:
    n_sft and n_bins from sft.shape[:2], n_sky from sky.shape[0].  Scalars
    and missing arrays are left to the library's own checks."""
    if len(w.sft.shape) < 2:
        raise ValueError("sft: expected [n_sft, n_bins, 2] or [n_sft, n_bins]")
    n_sft, n_bins, n_sky = int(w.sft.shape[0]), int(w.sft.shape[1]), int(w.sky.shape[0])
    if storage == "c64":
        if _dtype_name(w.sft) == "complex64":            # [n_sft, n_bins] complex
            if _numel(w.sft) != n_sft * n_bins:
                raise ValueError(f"sft: {_numel(w.sft)} complex elements, expected {n_sft * n_bins}")
        else:                                            # [n_sft, n_bins, 2] float32
            check_array("sft", w.sft, "f32", 2 * n_sft * n_bins)
        if w.sft_scale is not None:
            check_array("sft_scale", w.sft_scale, "f32", n_sft)
    else:
        check_array("sft", w.sft, "u16pair", 2 * n_sft * n_bins)
        check_array("sft_scale", w.sft_scale, "f32", n_sft)
    check_array("t_start", w.t_start, "f64", n_sft)
    check_array("pos", w.pos, "f64", 3 * n_sft)
    check_array("vel", w.vel, "f64", 3 * n_sft)
    check_array("sky", w.sky, "f64", 3 * n_sky)
    check_array("a", w.a, "f32", n_sky * n_sft)
    check_array("b", w.b, "f32", n_sky * n_sft)


def check_output(w, o) -> None:
    """Element types and counts of the outputs against the template count
    n_sky * n_fd * n_f of work unit w."""
    n = int(w.sky.shape[0]) * int(w.n_fd) * int(w.n_f)
    top_k = int(getattr(o, "top_k", 0))
    check_array("twoF", o.twoF, "f32", n)
    check_array("fa", getattr(o, "fa", None), "f32", 2 * n)
    check_array("fb", getattr(o, "fb", None), "f32", 2 * n)
    if top_k > 0:
        check_array("top", getattr(o, "top", None), "i32", 4 * top_k, at_least=True)
        check_array("n_above", getattr(o, "n_above", None), "i64", 1, at_least=True)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


@dataclasses.dataclass
class WorkUnit:
    """Device-resident work unit (mirrors fstat_wu)."""
    n_det: int
    sft: object            # tensor [n_sft, n_bins, 2] float32, or [n_sft, n_bins, 2] int16/uint16 bits
    sft_scale: object      # tensor [n_sft] float32 or None
    k_first: int
    t_sft: float
    t_start: object        # float64 [n_sft]
    pos: object            # float64 [n_sft, 3]
    vel: object            # float64 [n_sft, 3]
    sky: object            # float64 [n_sky, 3]
    a: object              # float32 [n_sky, n_sft]
    b: object              # float32 [n_sky, n_sft]
    f0: float
    df: float
    n_f: int
    fdot0: float
    dfdot: float
    n_fd: int
    t_ref: float
    dterms: int
    det_offset: object = None  # host [n_det + 1] SFT offsets of the detectors, or None

    @property
    def n_sft(self):
        return int(self.sft.shape[0])

    @property
    def n_bins(self):
        return int(self.sft.shape[1])

    @property
    def n_sky(self):
        return int(self.sky.shape[0])


@dataclasses.dataclass
class Output:
    """Device outputs.  For a toplist set top_k > 0, threshold, top (int32
    tensor [top_k, 4]: 2F as float bits, sky, fdot, f) and n_above (int64
    tensor [1]); twoF may then be None."""
    twoF: object
    fa: object = None
    fb: object = None
    top_k: int = 0
    threshold: float = 0.0
    top: object = None
    n_above: object = None


def _wu_struct(w) -> fstat_wu:
    off = getattr(w, "det_offset", None)
    keep = None
    if off is not None:                                  # a host array the call reads synchronously
        vals = [int(x) for x in (off.tolist() if hasattr(off, "tolist") else off)]
        if len(vals) != int(w.n_det) + 1:
            raise ValueError(f"det_offset: {len(vals)} entries, expected n_det + 1 = {int(w.n_det) + 1}")
        keep = (ctypes.c_int64 * len(vals))(*vals)
    s = fstat_wu(int(w.n_det), ctypes.cast(keep, ctypes.c_void_p) if keep is not None else None, int(w.n_sft),
                 int(w.n_bins), int(w.k_first), float(w.t_sft), _ptr(w.sft), _ptr(w.sft_scale), _ptr(w.t_start),
                 _ptr(w.pos), _ptr(w.vel), int(w.n_sky), _ptr(w.sky), _ptr(w.a), _ptr(w.b), float(w.f0),
                 float(w.df), int(w.n_f), float(w.fdot0), float(w.dfdot), int(w.n_fd), float(w.t_ref),
                 int(w.dterms))
    s._keep = keep                                       # alive as long as the struct
    return s


def _out_struct(o) -> fstat_out:
    return fstat_out(_ptr(o.twoF), _ptr(getattr(o, "fa", None)), _ptr(getattr(o, "fb", None)),
                     int(getattr(o, "top_k", 0)), float(getattr(o, "threshold", 0.0)),
                     _ptr(getattr(o, "top", None)), _ptr(getattr(o, "n_above", None)))


def toplist(o):
    """Host copy of an Output's toplist: (twoF float32, sky, fdot, f) numpy
    arrays cut at min(n_above, top_k), and n_above."""
    import numpy as np
    t = o.top.cpu().numpy().reshape(-1, 4)
    n_above = int(o.n_above.cpu().numpy().reshape(-1)[0])
    n = min(n_above, t.shape[0])
    return (t[:n, 0].view(np.float32).copy(), t[:n, 1].copy(), t[:n, 2].copy(), t[:n, 3].copy(), n_above)


def fstat_detector_inputs(plan, earth: dict, sites, t_mid, site_of_sft, sky, pos, vel, a, b, stream=None) -> None:
    """Detector positions, velocities and antenna patterns on the device.
    earth: dict with the fstat_earth fields; sites: (lat, lon, az_x, az_y)
    tuples in radians; the arrays are device tensors (t_mid float64 [n_sft],
    site_of_sft int32 [n_sft], sky float64 [n_sky, 3], pos and vel float64
    [n_sft, 3], a and b float32 [n_sky, n_sft])."""
    e = fstat_earth(*[float(earth[k]) for k, _ in fstat_earth._fields_])
    st = (fstat_site * len(sites))(*[fstat_site(*map(float, x)) for x in sites])
    n_sft, n_sky = int(t_mid.shape[0]), int(sky.shape[0])
    for name, t, kind, n in (("t_mid", t_mid, "f64", n_sft), ("site_of_sft", site_of_sft, "i32", n_sft),
                             ("sky", sky, "f64", 3 * n_sky), ("pos", pos, "f64", 3 * n_sft),
                             ("vel", vel, "f64", 3 * n_sft), ("a", a, "f32", n_sky * n_sft),
                             ("b", b, "f32", n_sky * n_sft)):
        check_array(name, t, kind, n)
    _check(plan, load_library().fstat_detector_inputs(plan, ctypes.byref(e), len(sites), st, n_sft, _ptr(t_mid),
                                                      _ptr(site_of_sft), n_sky, _ptr(sky), _ptr(pos), _ptr(vel),
                                                      _ptr(a), _ptr(b), _stream_handle(stream)))


def fstat_strerror(code: int) -> str:
    return load_library().fstat_strerror(int(code)).decode()


def fstat_last_error(plan) -> str:
    return load_library().fstat_last_error(plan).decode()


def _check(plan, rc: int):
    if rc != FSTAT_OK:
        detail = fstat_last_error(plan) if plan else ""
        raise FstatError(rc, f"{fstat_strerror(rc)}: {detail}" if detail else fstat_strerror(rc))


def fstat_plan_create(*, max_sft, max_bins, max_sky, max_fd, max_f, max_dterms=16, storage="c64", phase="fp64",
                      kernel="auto", coef="f32", flags=0, device=-1, max_cands=0):
    """coef="f16" selects the mixed-precision form of the interp kernel
    (FP16 window-polynomial coefficients, FSTAT_FLAG_COEF16)."""
    lib = load_library()
    if coef not in ("f32", "f16"):
        raise ValueError(f"coef must be 'f32' or 'f16', not {coef!r}")
    if coef == "f16":
        flags |= FSTAT_FLAG_COEF16
    d = fstat_desc(int(max_sft), int(max_bins), int(max_sky), int(max_fd), int(max_f), int(max_dterms),
                   STORAGE.get(storage, storage), PHASES.get(phase, phase), KERNELS.get(kernel, kernel), int(flags),
                   int(device), int(max_cands))
    h = ctypes.c_void_p()
    rc = lib.fstat_plan_create(ctypes.byref(h), ctypes.byref(d))
    _check(None, rc)
    _PLAN_STORAGE[h.value] = {v: k for k, v in STORAGE.items()}.get(d.storage, "c64")
    return h


def fstat_plan_destroy(plan) -> None:
    if plan:
        _PLAN_STORAGE.pop(getattr(plan, "value", plan), None)
        load_library().fstat_plan_destroy(plan)


def _checked(plan, wu, out=None):
    """fstat_wu / fstat_out structs of a work unit and its output, after the
    array checks against the work unit's sizes and the plan's storage."""
    st = _storage_of(plan)
    if st is None:                                   # plan of unknown storage: either layout
        st = "c64" if _dtype_name(wu.sft) in ("float32", "complex64") else "bf16"
    check_work_unit(wu, st)
    if out is not None:
        check_output(wu, out)
    return _wu_struct(wu), (_out_struct(out) if out is not None else None)


def fstat_compute(plan, wu, out, stream=None) -> None:
    s, o = _checked(plan, wu, out)
    _check(plan, load_library().fstat_compute(plan, ctypes.byref(s), ctypes.byref(o), _stream_handle(stream)))


def fstat_compute_noalloc(plan, wu, out, stream=None) -> None:
    """fstat_compute with the library's static device scratch: allocates no
    device memory (see include/fstat.h)."""
    s, o = _checked(plan, wu, out)
    _check(plan, load_library().fstat_compute_noalloc(plan, ctypes.byref(s), ctypes.byref(o), _stream_handle(stream)))


def fstat_batch_compute(plan, wus: Sequence, outs: Sequence, stream=None) -> None:
    n = len(wus)
    if len(outs) != n:
        raise ValueError("one output per work unit")
    pairs = [_checked(plan, w, o) for w, o in zip(wus, outs)]
    ws = (fstat_wu * max(n, 1))(*[x[0] for x in pairs])
    os_ = (fstat_out * max(n, 1))(*[x[1] for x in pairs])
    _check(plan, load_library().fstat_batch_compute(plan, ws, n, os_, _stream_handle(stream)))


def fstat_semicoherent(plan, segs: Sequence, out, stream=None) -> None:
    n = len(segs)
    structs = [_checked(plan, w)[0] for w in segs]       # hold each struct's det_offset copy during the call
    ws = (fstat_wu * max(n, 1))(*structs)
    if n:
        check_output(segs[0], out)
    o = _out_struct(out)
    _check(plan, load_library().fstat_semicoherent(plan, ws, n, ctypes.byref(o), _stream_handle(stream)))


def fstat_bins(plan, wu, i_sky, i_fd, i_f, i_sft, kstar, kappa, phi_frac, stream=None) -> None:
    s, _ = _checked(plan, wu)
    n = _numel(i_sky)
    for name, t, kind in (("i_sky", i_sky, "i32"), ("i_fd", i_fd, "i32"), ("i_f", i_f, "i32"), ("i_sft", i_sft, "i32"),
                          ("kstar", kstar, "i64"), ("kappa", kappa, "f64"), ("phi_frac", phi_frac, "f64")):
        check_array(name, t, kind, n)
    _check(plan, load_library().fstat_bins(plan, ctypes.byref(s), n, _ptr(i_sky), _ptr(i_fd), _ptr(i_f), _ptr(i_sft),
                                           _ptr(kstar), _ptr(kappa), _ptr(phi_frac), _stream_handle(stream)))


def fstat_interp_slice(df: float, dfdot: float, nfd: int, threads: int, coef16: bool, max_abs_tau: float,
                       max_p: float):
    """(slice width in bins, fits) of the interp kernel's LDS slice for a tile
    (a host computation; see include/fstat.h)."""
    fits = ctypes.c_int32(0)
    w = load_library().fstat_interp_slice(float(df), float(dfdot), int(nfd), int(threads), int(bool(coef16)),
                                          float(max_abs_tau), float(max_p), ctypes.byref(fits))
    return int(w), bool(fits.value)


def fstat_autotune(plan, wu, out, stream=None, cache_path: Optional[str] = None) -> None:
    s, o = _checked(plan, wu, out)
    path = cache_path.encode() if cache_path else None
    _check(plan, load_library().fstat_autotune(plan, ctypes.byref(s), ctypes.byref(o), _stream_handle(stream), path))


def fstat_last_kernel_ms(plan) -> float:
    return float(load_library().fstat_last_kernel_ms(plan))


SPLIT_SIZES = (16, 8, 7, 6, 5, 4)


def fstat_spindown_split(n_fd: int, coef16: bool = False, allow16: bool = True, paired: bool = False) -> dict:
    """{spindowns per thread: spindowns run so} for n_fd spindowns (the
    library's split, see include/fstat.h)."""
    buf = (ctypes.c_int64 * len(SPLIT_SIZES))()
    rc = load_library().fstat_spindown_split(int(n_fd), int(bool(coef16)), int(bool(allow16)), int(bool(paired)),
                                             buf)
    if rc != 0:
        raise FstatError(rc, f"fstat_spindown_split({n_fd}): {fstat_strerror(rc)}")
    return {b: int(n) for b, n in zip(SPLIT_SIZES, buf) if n}


def fstat_sky_pairs(sky, f0, df, n_f, fdot0, dfdot, n_fd, t_sft, max_abs_tau, max_p, max_v, max_r):
    """(slice width, tiles as an [n, 2] int array) of the library's pairing
    of sky points (see include/fstat.h); width 0 and no tiles when it keeps
    one sky point per tile.  `sky` is a host array [n_sky][3]."""
    import numpy as np
    sky = np.ascontiguousarray(sky, dtype=np.float64)
    if sky.ndim != 2 or sky.shape[1] != 3:
        raise ValueError("sky must be [n_sky][3]")
    n = sky.shape[0]
    out = np.zeros(2 * max(n, 1), dtype=np.int32)
    n_pairs = ctypes.c_int64(0)
    w = load_library().fstat_sky_pairs(n, sky.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), f0, df, n_f, fdot0,
                                       dfdot, n_fd, t_sft, max_abs_tau, max_p, max_v, max_r,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(n_pairs))
    if w < 0:
        raise FstatError(w, f"fstat_sky_pairs: {fstat_strerror(w)}")
    return int(w), out[:2 * n_pairs.value].reshape(-1, 2).copy()


def fstat_last_tile(plan) -> dict:
    """Launch shape of the plan's last single-unit demodulation (see
    include/fstat.h): keys nf_reg, chunk, seg, sblock, threads, pair_seg,
    sky_tiles, and split = {spindowns per thread: spindowns run so}."""
    buf = (ctypes.c_int32 * LAST_TILE_LEN)()
    _check(plan, load_library().fstat_last_tile(plan, buf))
    v = list(buf)
    split = {b: n for b, n in zip((16, 8, 7, 6, 5, 4), v[7:]) if n}
    return dict(nf_reg=v[0], chunk=v[1], seg=v[2], sblock=v[3], threads=v[4], pair_seg=v[5], sky_tiles=v[6],
                split=split)


class Plan:
    """Owning wrapper around an fstat_plan handle."""

    def __init__(self, **desc):
        self.handle = fstat_plan_create(**desc)

    def compute(self, wu, out, stream=None):
        fstat_compute(self.handle, wu, out, stream)

    def compute_noalloc(self, wu, out, stream=None):
        fstat_compute_noalloc(self.handle, wu, out, stream)

    def batch_compute(self, wus, outs, stream=None):
        fstat_batch_compute(self.handle, wus, outs, stream)

    def semicoherent(self, segs, out, stream=None):
        fstat_semicoherent(self.handle, segs, out, stream)

    def bins(self, wu, i_sky, i_fd, i_f, i_sft, kstar, kappa, phi_frac, stream=None):
        fstat_bins(self.handle, wu, i_sky, i_fd, i_f, i_sft, kstar, kappa, phi_frac, stream)

    def detector_inputs(self, earth, sites, t_mid, site_of_sft, sky, pos, vel, a, b, stream=None):
        fstat_detector_inputs(self.handle, earth, sites, t_mid, site_of_sft, sky, pos, vel, a, b, stream)

    def autotune(self, wu, out, stream=None, cache_path=None):
        fstat_autotune(self.handle, wu, out, stream, cache_path)

    def last_kernel_ms(self) -> float:
        return fstat_last_kernel_ms(self.handle)

    def last_tile(self) -> dict:
        return fstat_last_tile(self.handle)

    def last_error(self) -> str:
        return fstat_last_error(self.handle)

    def close(self):
        if self.handle:
            fstat_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
