"""Move a synthetic work unit to device tensors in the layout of fstat_wu."""
from __future__ import annotations

import numpy as np

from .workloads import quantise_sfts


def to_device(w, storage: str = "c64", device: str = "cuda"):
    """Returns (paper_0904_1826_amd.WorkUnit, dequantised complex128 SFTs or
    None).  For 16-bit storage the second value holds the exact values the
    stored bits represent, for the oracle's arithmetic-parity comparison."""
    import torch
    from paper_0904_1826_amd import WorkUnit

    def t(x, dt):
        return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dt)

    deq = None
    if storage == "c64":
        sft = t(np.ascontiguousarray(w.sft).view(np.float32).reshape(w.n_sft, w.n_bins, 2), torch.float32)
        scale = None
    else:
        from .workloads import dequantise_16bit
        stored, sc = quantise_sfts(w.sft, storage)
        sft = torch.from_numpy(stored.view(np.int16)).to(device)
        scale = t(sc, torch.float32)
        deq = dequantise_16bit(stored, sc, storage)
    wu = WorkUnit(n_det=int(w.n_det), sft=sft, sft_scale=scale, k_first=int(w.k_first), t_sft=float(w.t_sft),
                  t_start=t(w.t_start, torch.float64), pos=t(w.pos, torch.float64), vel=t(w.vel, torch.float64),
                  sky=t(w.sky, torch.float64), a=t(w.a, torch.float32), b=t(w.b, torch.float32), f0=float(w.f0),
                  df=float(w.df), n_f=int(w.n_f), fdot0=float(w.fdot0), dfdot=float(w.dfdot), n_fd=int(w.n_fd),
                  t_ref=float(w.t_ref), dterms=int(w.dterms), det_offset=np.asarray(w.det_offset, dtype=np.int64))
    return wu, deq


def alloc_output(w, device: str = "cuda", fafb: bool = False, top_k: int = 0, threshold: float = 0.0,
                 full: bool = True):
    """Output buffers; with top_k > 0 also a toplist of that length (and,
    with full=False, no full 2F array)."""
    import torch
    from paper_0904_1826_amd import Output
    shape = (w.n_sky, w.n_fd, w.n_f)
    tw = torch.empty(shape, dtype=torch.float32, device=device) if full else None
    fa = torch.empty(shape + (2,), dtype=torch.float32, device=device) if fafb else None
    fb = torch.empty(shape + (2,), dtype=torch.float32, device=device) if fafb else None
    top = torch.empty((top_k, 4), dtype=torch.int32, device=device) if top_k > 0 else None
    n_above = torch.empty(1, dtype=torch.int64, device=device) if top_k > 0 else None
    return Output(twoF=tw, fa=fa, fb=fb, top_k=top_k, threshold=threshold, top=top, n_above=n_above)


def draw_noise_c64(w, seed: int = 0, device: str = "cuda"):
    """Device-side inputs for a work unit whose SFTs were not drawn on the host
    (noise="device"): CN(0,1) noise from torch's seeded generator on `device`,
    stored as complex64 ([n_sft, n_bins, 2] float32).  Returns a
    paper_0904_1826_amd.WorkUnit."""
    import torch
    from paper_0904_1826_amd import WorkUnit
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn((w.n_sft, w.n_bins, 2), generator=g, device=device, dtype=torch.float32) * (0.5 ** 0.5)

    def t(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)

    return WorkUnit(n_det=int(w.n_det), sft=x, sft_scale=None, k_first=int(w.k_first),
                    t_sft=float(w.t_sft), t_start=t(w.t_start, torch.float64), pos=t(w.pos, torch.float64),
                    vel=t(w.vel, torch.float64), sky=t(w.sky, torch.float64), a=t(w.a, torch.float32),
                    b=t(w.b, torch.float32), f0=float(w.f0), df=float(w.df), n_f=int(w.n_f), fdot0=float(w.fdot0),
                    dfdot=float(w.dfdot), n_fd=int(w.n_fd), t_ref=float(w.t_ref), dterms=int(w.dterms),
                    det_offset=np.asarray(w.det_offset, dtype=np.int64))


def quantise_device(wu, storage: str = "bf16"):
    """The 16-bit storage of a complex64 device work unit with a per-SFT scale
    max|re,im| / 256 (the rule of synth.quantise_sfts): a new WorkUnit sharing
    every other array with `wu`."""
    import dataclasses
    import torch
    x = wu.sft
    m = x.abs().amax(dim=(1, 2))
    scale = torch.where(m > 0, m / 256.0, torch.ones_like(m))
    y = x / scale[:, None, None]
    if storage == "bf16":
        stored = y.to(torch.bfloat16).view(torch.int16)
    elif storage == "fp16":
        stored = y.to(torch.float16).view(torch.int16)
    else:
        raise ValueError(storage)
    del y
    return dataclasses.replace(wu, sft=stored, sft_scale=scale.contiguous())


def draw_noise_16bit(w, storage: str = "bf16", seed: int = 0, device: str = "cuda"):
    """draw_noise_c64 stored as 16-bit pairs with a per-SFT scale
    (quantise_device).  Returns a paper_0904_1826_amd.WorkUnit."""
    wu = draw_noise_c64(w, seed, device)
    q = quantise_device(wu, storage)
    del wu
    return q


def host_values(wu, storage: str = "bf16"):
    """Exact complex128 values of a device work unit's 16-bit SFT storage."""
    from .workloads import dequantise_16bit
    stored = wu.sft.cpu().numpy().view(np.uint16)
    return dequantise_16bit(stored, wu.sft_scale.cpu().numpy(), storage)
