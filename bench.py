#!/usr/bin/env python3
"""Benchmark of the F-statistic demodulation on one MI355X.

A step is one full pass of the hot path over one work unit: per (sky, SFT)
geometry and band check, then the demodulation (bin index, phase, Dirichlet
window sums, a/b weighting, sum over SFTs and detectors, 2F).  The main
workload is the work-unit-shaped case: 2 detectors x 1000 SFTs of 1800 s,
a 3600-bin band at 1000 Hz, 2000 sky points x 8 spindowns x 3600
frequencies, Dterms = 8 (5.76e7 templates, 1.15e11 template-SFT pairs).
Inputs are synthetic (seeded noise and injected signals) and resident in HBM
before the timed region.  Prints one JSON line.

Besides the forms of the main case (complex64, the double-FP32 split phase,
BF16 and FP16 storage, and the FP16-coefficient form) it times the direct
kernel, the toplist-only output, the semi-coherent sum of the same case split
into 20 time segments, and the 256-unit batch (configuration "large") with
complex64 SFTs and with the BF16 storage of the same values, one warm-up call
and several timed replays each.

Every timed form's 2F is compared with the FP64 oracle on a sample of its
templates (the oracle leg, after the GPU timing: it is also the CPU baseline)
and its maximum and rms error e = |2F - 2F_ref| / max(2F_ref, 4) are reported
with whether the form is within the metric's 1e-4.  16-bit storage forms are
compared with the oracle run on their exactly dequantised values (arithmetic)
and with the oracle on the complex64 values (storage error).

With --workload large the 256-unit batch is the main case (a step is one
fstat_batch_compute call over all its units) and nothing else is timed.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms c64,c64+split,bf16,fp16,bf16+coef16]
                  [--workload workunit|semicoherent|large] [--batch 4|3|0] [--batch-replays R]
                  [--large-forms c64,bf16]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X (gfx950): 256 CUs at 2.4 GHz, 4 SIMDs of 16 lanes per CU: one wave64
# VALU instruction per SIMD every 4 clocks, i.e. 64 lane-ops per CU per clock
# = 3.93e13 lane-ops/s for every unpacked FP32 or FP64 operation (FP64 FMA
# is full rate: 78.6 TFLOP/s counting two flops; FP32 reaches 157.3 TFLOP/s
# only with packed dual-FP32 instructions, which this library does not use).
# Measured on the chip: FP32 and FP64 FMA issue at that rate, v_sin/v_cos
# take two issue slots.  One "slot" is one lane-op at full rate.
N_CU, CLK, LANES = 256, 2.4e9, 64
PEAK_SLOTS = N_CU * LANES * CLK               # 3.93e13 slot/s
HBM_PEAK = 8.0e12
METRIC = "templates·SFTs/s for 2F (plain vs mixed-precision) at 2F rel err ≤1e-4; % roofline"
METRIC_TOL = 1e-4


def slots_per_pair(kernel: str, dterms: int, nfd: int = 8, coef16: bool = False) -> float:
    """Algorithmic VALU slots per (template, SFT) pair of each kernel's
    formulation (instruction count of the arithmetic the method needs; no
    addressing, staging or loop control).  With FP16 coefficients the Horner
    steps are packed FP16 FMAs (real and imaginary part in one slot) and v is
    rounded to FP16 once."""
    if kernel == "direct":
        # FP64 Dphi (fma), k*, kappa, 1 - kappa and phase: 10; sign 3;
        # central weights 12 (sin and two reciprocals at 2 slots) and their
        # terms 6; far terms (2D-2) x 6; fraction folds 8; sin/cos of the
        # phase 4; rotation 4; Fa/Fb 4
        return 12 * dterms + 39
    if kernel == "interp":
        # FP64 Dphi (one fma), k*, kappa and its conversion 4, degree-7
        # complex Horner 14, phase factor product 4 + rotation 4, Fa/Fb 4;
        # frac(tau f) and its sin/cos (3 + 2 x 2) shared by the nfd spindowns
        # of a thread
        return (30 + 7.0 / nfd) if not coef16 else (30 - 7 + 1 + 7.0 / nfd)
    raise ValueError(kernel)


def method_slots(dterms: int) -> float:
    """Slots per pair of the literal Dterms loop with one reciprocal per
    window term (2D terms of 1 reciprocal at 4 and 1 complex-by-real MAC;
    3 sin/cos at 4; 8 FP64 and 8 FP32 others): 10 D + 28.  A kernel that
    folds the window into fewer operations does less than this per pair, so
    its rate against this count can exceed the peak."""
    return 10.0 * dterms + 28.0


def strip_comments(src: str) -> str:
    """C++ source without comments and blank lines (string literals in these
    sources hold no comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(l.rstrip() for l in src.splitlines() if l.strip())


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code (comments excluded), which ties a
    counter summary to the kernels it was taken on."""
    h = hashlib.sha256()
    for f in ("fstat_kernels.hip", "fstat_internal.h"):
        with open(os.path.join(ROOT, "paper_0904_1826_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name: str, workload: str):
    """HBM bytes of one demodulation pass (all its launches) of the dominant
    kernel from the committed rocprofv3 counter summary, and the number of
    launches in the pass, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None, None
    e = d.get(f"{kernel_name}:{workload}")
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None, None
    return e.get("bytes_per_pass"), e.get("launches_per_pass")


def host_threads() -> int:
    """Threads for the oracle: the process's CPU affinity, at most 16 (the
    host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def err_stats(gpu, ref, tol=METRIC_TOL):
    """max and rms of e = |2F_gpu - 2F_ref| / max(2F_ref, 4) over a sample."""
    import numpy as np
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    e = np.abs(g - r) / np.maximum(r, 4.0)
    if not np.all(np.isfinite(e)):
        return {"max_e": None, "rms_e": None, "n_templates": int(e.size), "finite": False,
                "at_metric_tolerance": False}
    return {"max_e": float(e.max()), "rms_e": float(math.sqrt(np.mean(e * e))), "n_templates": int(e.size),
            "at_metric_tolerance": bool(e.max() <= tol)}


def time_steps(torch, step, warmup, steps, kernel_ms):
    """Warm-up calls, then `steps` timed calls bracketed by synchronisations:
    (wall seconds per step, mean demodulation-kernel ms per step)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        kms.append(kernel_ms())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el / steps, sum(kms) / len(kms)


def take(t, idx):
    """Host copy of t[s, i, j] for index arrays (s, i, j) of a device tensor."""
    import torch
    ix = tuple(torch.from_numpy(x).to(device=t.device, dtype=torch.int64) for x in idx)
    return t[ix].cpu().numpy()


def parse_form(form):
    storage, *extra = form.split("+")
    return storage, "split" in extra, "coef16" in extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="c64,c64+split,bf16,fp16,bf16+coef16",
                    help="SFT storage (c64, bf16, fp16), optionally +split (double-FP32 phase) and +coef16 "
                         "(FP16 window-polynomial coefficients)")
    ap.add_argument("--kernel", default="auto", help="auto (= interp), interp or direct")
    ap.add_argument("--compare-direct", type=int, default=2,
                    help="also time this many steps of the direct kernel on complex64 storage")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work for the CPU baseline at the host's thread share")
    ap.add_argument("--toplist", type=int, default=1000,
                    help="also time the plain form writing only a top-K toplist above 2F = 20 (0: skip)")
    ap.add_argument("--semicoherent", type=int, default=20,
                    help="also time the semi-coherent sum over this many segments of the same case (0: skip)")
    ap.add_argument("--batch", type=int, default=4, choices=[0, 3, 4],
                    help="also time the batched form on the 256-unit case (4: complex64 and BF16 storage of the "
                         "same values) or the 64-unit case (3), 0: skip")
    ap.add_argument("--batch-replays", type=int, default=3, help="timed calls per batched form after one warm-up")
    ap.add_argument("--large-forms", default="c64,bf16",
                    help="forms of the 256-unit batch, in order: c64 and/or bf16 (the BF16 storage of the same "
                         "values), optionally +coef16")
    ap.add_argument("--workload", default="workunit", choices=["workunit", "semicoherent", "large"],
                    help="the case the forms are timed on: the work-unit-shaped case, the same case as "
                         "--semicoherent segments combined by fstat_semicoherent, or the 256-unit batch alone")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (no errors either)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the F-statistic shards by work unit or sky point with no exchange, "
              "and this benchmark runs and reports a single MI355X only (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from synth.device import to_device, alloc_output
    import paper_0904_1826_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    say = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        say(f"calibration copy: {n} bytes read, {n} bytes written")
        del src, dst
    if args.workload == "large":
        return main_large(args, torch, P, synth, say)
    t0 = time.time()
    semi_main = args.workload == "semicoherent"
    if semi_main:
        case = synth.make_segment_config(args.semicoherent or 20)
        case_name = case[0].name.rsplit("-", 1)[0]
    else:
        case = [synth.make_config(1)]
        case_name = case[0].name
    w = case[0]
    n_sft_total = sum(x.n_sft for x in case)
    say(f"workload {case_name}: {n_sft_total} SFTs in {len(case)} part(s) x {w.n_bins} bins, "
        f"{w.n_templates} templates (generated in {time.time() - t0:.1f} s)")
    pairs = w.n_templates * n_sft_total
    kernel = "direct" if args.kernel == "direct" else "interp"     # the library resolves auto to interp

    # templates whose GPU 2F is kept for the oracle leg: four whole sky points
    # (every spindown and frequency) and every injected template
    sample_sky = sorted({0, w.n_sky // 3, (2 * w.n_sky) // 3, w.n_sky - 1})
    ss, si, sj = (np.concatenate([a, np.array([getattr(x, k) for x in w.injections], dtype=np.int32)])
                  for a, k in zip(oracle_free_templates(w, sample_sky), ("sky_index", "fdot_index", "f_index")))

    forms = [f for f in args.forms.split(",") if f]
    results, samples, deq = {}, {}, {}
    for form in forms:
        storage, split, c16 = parse_form(form)
        devs = [to_device(x, storage) for x in case]
        wus = [d[0] for d in devs]
        if storage != "c64" and not semi_main:
            deq[storage] = devs[0][1]
        out = alloc_output(w)
        torch.cuda.synchronize()
        with P.Plan(max_sft=max(x.n_sft for x in case), max_bins=max(x.n_bins for x in case), max_sky=w.n_sky,
                    max_fd=w.n_fd, max_f=w.n_f, max_dterms=w.dterms, storage=storage, coef="f16" if c16 else "f32",
                    phase="split" if split else "fp64", kernel=args.kernel) as plan:
            step = (lambda: plan.semicoherent(wus, out)) if semi_main else (lambda: plan.compute(wus[0], out))
            steps = args.steps if form == forms[0] else max(2, args.steps // 2)
            s_step, kms = time_steps(torch, step, args.warmup, steps, plan.last_kernel_ms)
            launch = plan.last_tile()          # the shape the library ran (spindown split, sky pairs)
        samples[form] = take(out.twoF, (ss, si, sj))
        results[form] = {"steps": steps, "ms_per_step": 1e3 * s_step, "value": pairs / s_step, "kernel_ms": kms,
                         "launch": {k: v for k, v in launch.items() if k != "split"} | {"split": {str(b): n for b, n in launch["split"].items()}}}
        say(f"{form}: {results[form]}")
        del wus, devs, out
        torch.cuda.empty_cache()

    kernels = {}
    if args.compare_direct > 0 and kernel != "direct" and not semi_main:
        wu, _ = to_device(w, "c64")
        out = alloc_output(w)
        with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                    max_dterms=w.dterms, storage="c64", kernel="direct") as plan:
            s_step, kms = time_steps(torch, lambda: plan.compute(wu, out), 1, args.compare_direct, plan.last_kernel_ms)
        samples["direct"] = take(out.twoF, (ss, si, sj))
        kernels["direct"] = {"value": pairs / s_step, "kernel_ms": kms,
                             "roofline_frac": slots_per_pair("direct", w.dterms) * pairs / (kms * 1e-3) / PEAK_SLOTS}
        say(f"direct c64: {kernels['direct']}")
        del wu, out
        torch.cuda.empty_cache()
    toplist = None
    if args.toplist > 0 and not semi_main:
        wu, _ = to_device(w, "c64")
        out = alloc_output(w, top_k=args.toplist, threshold=20.0, full=False)
        with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                    max_dterms=w.dterms, kernel=args.kernel) as plan:
            s_step, _ = time_steps(torch, lambda: plan.compute(wu, out), 1, 2, plan.last_kernel_ms)
        n_above = int(out.n_above.cpu().item())
        toplist = {"top_k": args.toplist, "threshold": 20.0, "n_above": n_above, "ms_per_step": 1e3 * s_step,
                   "value": pairs / s_step, "full_2F_written": False}
        say(f"toplist: {toplist}")
        del wu, out
        torch.cuda.empty_cache()
    semi, semi_samples, segs = None, {}, None
    if args.semicoherent > 0 and not semi_main:
        t0 = time.time()
        segs = synth.make_segment_config(args.semicoherent)
        spairs = segs[0].n_templates * sum(x.n_sft for x in segs)
        devs = [to_device(x, "c64")[0] for x in segs]
        out = alloc_output(segs[0])
        gen_s = time.time() - t0
        semi = {"workload": segs[0].name.rsplit("-", 1)[0], "n_seg": len(segs),
                "n_sft": [int(x.n_sft) for x in segs][:3] + ["..."], "pairs_per_step": spairs}
        inj_sky = segs[0].injections[0].sky_index
        for coef in ("f32", "f16"):
            with P.Plan(max_sft=max(x.n_sft for x in segs), max_bins=max(x.n_bins for x in segs),
                        max_sky=segs[0].n_sky, max_fd=segs[0].n_fd, max_f=segs[0].n_f, max_dterms=segs[0].dterms,
                        coef=coef, kernel=args.kernel) as plan:
                s_step, kms = time_steps(torch, lambda: plan.semicoherent(devs, out), 1, 2, plan.last_kernel_ms)
            key = "coef16" if coef == "f16" else "plain"
            semi_samples[key] = out.twoF[inj_sky].cpu().numpy().ravel()
            semi[key] = {"value": spairs / s_step, "ms_per_step": 1e3 * s_step, "kernel_ms": kms,
                         "roofline_frac": slots_per_pair(kernel, segs[0].dterms, coef16=coef == "f16") * spairs
                         / (kms * 1e-3) / PEAK_SLOTS}
        say(f"semi-coherent ({gen_s:.1f} s to generate): {semi}")
        del devs, out
        torch.cuda.empty_cache()
    batch, batch_ref = None, None
    if args.batch and not semi_main and kernel != "direct":
        batch, batch_ref = run_batch(args, torch, P, synth, say)

    # ------------------------------------------------------------ oracle leg
    # The FP64 CPU oracle on the sampled templates: its timing is the CPU
    # baseline, and its values are the reference for the error of every GPU
    # form above.  Nothing here is timed on the GPU.
    cpu, refs = None, {}
    if not args.no_cpu_baseline and not semi_main:
        cpu, refs = oracle_leg(w, (ss, si, sj), deq, args.cpu_budget, say)
    for form, r in results.items():
        storage, split, c16 = parse_form(form)
        if refs:
            r["err"] = err_stats(samples[form], refs["c64" if storage == "c64" else storage])
            r["err"]["reference"] = ("oracle on the complex64 values" if storage == "c64"
                                     else f"oracle on the exactly dequantised {storage.upper()} values")
            if storage != "c64":
                r["storage_err_vs_c64"] = err_stats(samples[form], refs["c64"], tol=5e-3)
    if "direct" in kernels and refs:
        kernels["direct"]["err"] = err_stats(samples["direct"], refs["c64"])
    if semi is not None and not args.no_cpu_baseline:
        import oracle
        sw = segs[0]
        tm = oracle.all_templates(sw, [sw.injections[0].sky_index])
        ref = oracle.semicoherent(segs, tm, nthreads=host_threads())["twoF"]
        for key in ("plain", "coef16"):
            semi[key]["err"] = err_stats(semi_samples[key], ref)
            semi[key]["err"]["sample"] = f"sky point {sw.injections[0].sky_index}: {len(ref)} templates"
    if batch is not None and batch_ref is not None and not args.no_cpu_baseline:
        batch_errors(batch, batch_ref, say)

    main_form = forms[0]
    r = results[main_form]
    main_c16 = parse_form(main_form)[2]
    for form, v in results.items():
        c16 = parse_form(form)[2]
        v["roofline_frac"] = slots_per_pair(kernel, w.dterms, coef16=c16) * pairs / (v["kernel_ms"] * 1e-3) / PEAK_SLOTS
        v["traffic"] = measured_traffic("demod_interp_coef16" if c16 else f"demod_{kernel}",
                                        "semicoherent" if semi_main else "config1")[0]
        ok = v.get("err", {}).get("at_metric_tolerance")
        # a form outside the metric's 1e-4 gets no speed credit against the plain form
        v["vs_plain"] = v["value"] / r["value"] if ok or (ok is None and not c16) else None
        if v["vs_plain"] is None:
            v["speed_ratio_outside_metric"] = v["value"] / r["value"]
    traffic, launches = measured_traffic("demod_interp_coef16" if main_c16 else f"demod_{kernel}",
                                         "semicoherent" if semi_main else "config1")
    slots = slots_per_pair(kernel, w.dterms, coef16=main_c16) * pairs
    achieved = slots / (r["kernel_ms"] * 1e-3)
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "templates*SFTs/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case_name, "n_det": w.n_det, "n_sft": n_sft_total, "n_bins": w.n_bins,
                   "n_sky": w.n_sky, "n_fd": w.n_fd, "n_f": w.n_f, "dterms": w.dterms, "form": main_form,
                   "phase": "split" if parse_form(main_form)[1] else "fp64", "kernel": kernel,
                   "templates": w.n_templates, "pairs_per_step": pairs,
                   **({"n_seg": len(case)} if semi_main else {})},
        "err": r.get("err"),
        "forms": results,
        "kernels": kernels,
        "toplist": toplist,
        "semicoherent": semi,
        "large": batch,
        # per demodulation pass: all launches of the kernel in one step (the
        # library may split the SFT loop into several), timed together
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_SLOTS, "traffic": traffic, "launches_per_pass": launches,
                     "kernel": f"demod_{kernel}", "slots_per_pair": slots_per_pair(kernel, w.dterms, coef16=main_c16),
                     "kernel_ms": r["kernel_ms"],
                     # the same timing against the literal Dterms loop's work
                     # (10 D + 28 slots per pair): what folding the window buys
                     "method_slots_per_pair": method_slots(w.dterms),
                     "method_rate_vs_peak": method_slots(w.dterms) * pairs / (r["kernel_ms"] * 1e-3) / PEAK_SLOTS},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def main_large(args, torch, P, synth, say):
    """--workload large: the 256-unit batch is the main case; one JSON line
    whose value is the first form's rate (a step = one fstat_batch_compute
    call over the 256 units, after one warm-up call)."""
    args.batch = 4
    batch, ref = run_batch(args, torch, P, synth, say)
    if not args.no_cpu_baseline:
        batch_errors(batch, ref, say)
    first = [f for f in args.large_forms.split(",") if f][0]
    key = first
    r = batch[key]
    line = {
        "metric": METRIC, "value": r["value"], "unit": "templates*SFTs/s", "n_gpus": 1,
        "steps": args.batch_replays, "warmup": 1, "ms_per_step": 1e3 * r["s_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": batch["workload"], "n_wu": batch["n_wu"], "form": key, "kernel": "interp",
                   "pairs_per_step": batch["pairs_per_step"]},
        "err": r.get("err"), "large": batch,
        "roofline": {"bound": "alu", "achieved": r["slots_per_pair"] * batch["pairs_per_step"] / r["kernel_s"] / 1e12,
                     "peak": PEAK_SLOTS / 1e12, "unit": "TOP/s", "frac": r["roofline_frac"],
                     "traffic": r.get("traffic"), "kernel": "demod_interp_batch", "slots_per_pair": r["slots_per_pair"],
                     "kernel_ms": 1e3 * r["kernel_s"], "method_rate_vs_peak": r["method_rate_vs_peak"]},
    }
    print(json.dumps(line), flush=True)


def oracle_free_templates(w, sky_indices):
    """(sky, fdot, f) index arrays of every template of the listed sky points
    in output order (plain index arithmetic)."""
    import numpy as np
    s, i, j = np.meshgrid(np.asarray(sky_indices), np.arange(w.n_fd), np.arange(w.n_f), indexing="ij")
    return s.ravel().astype(np.int32), i.ravel().astype(np.int32), j.ravel().astype(np.int32)


def oracle_leg(w, templates, deq, budget_s, say):
    """The FP64 oracle on the sampled templates of the main case, for the
    complex64 values and for each 16-bit storage's dequantised values, at the
    host's thread share; then on one sky point's first spindowns with one
    thread.  Returns the CPU baseline and the reference 2F per input."""
    import oracle
    threads = host_threads()
    refs, done, el = {}, 0, 0.0
    for key, sft in [("c64", None)] + sorted(deq.items()):
        prep = oracle.Prepared(w, sft)
        t0 = time.perf_counter()
        refs[key] = prep.fstat(templates, nthreads=threads)["twoF"]
        el += time.perf_counter() - t0
        done += len(templates[0]) * w.n_sft
    # more of the same work unit, to reach the time budget at full threads
    prep = oracle.Prepared(w)
    extra_sky = 1
    while el < budget_s and extra_sky < w.n_sky:
        tm = oracle_free_templates(w, [extra_sky])
        t0 = time.perf_counter()
        prep.fstat(tm, nthreads=threads)
        el += time.perf_counter() - t0
        done += len(tm[0]) * w.n_sft
        extra_sky += 1
    # one thread: the first two spindowns of sky point 0
    tm = tuple(x[: 2 * w.n_f] for x in oracle_free_templates(w, [0]))
    t0 = time.perf_counter()
    prep.fstat(tm, nthreads=1)
    el1 = time.perf_counter() - t0
    one = len(tm[0]) * w.n_sft / el1
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count() or 1
    cpu = {"value": done / el, "unit": "templates*SFTs/s", "cores": threads, "kind": "oracle",
           "sample": f"the main work unit: {len(templates[0])} sampled templates x {w.n_sft} SFTs for each of "
                     f"{1 + len(deq)} inputs (complex64{''.join(', ' + k for k in sorted(deq))}) and sky points "
                     f"1..{extra_sky - 1} (all spindowns and frequencies), FP64, {el:.1f} s on {threads} threads",
           "one_thread": {"value": one, "sample": f"sky point 0, 2 spindowns x {w.n_f} frequencies x {w.n_sft} "
                                                  f"SFTs, {el1:.1f} s"},
           "cpu_model": cpu_model(), "cpus_available": nproc,
           "thread_share": "at most 16 threads: the host share of one GPU on the test box"}
    say(f"oracle leg: {cpu}")
    return cpu, refs


def run_batch(args, torch, P, synth, say):
    """The batched form on the 256-unit case: complex64 SFTs drawn on the
    device, then the BF16 storage of the same values (per-SFT scale), one
    warm-up call (which also captures the graphs) and args.batch_replays
    timed calls each.  On the 64-unit case (3): complex64 only.  Keeps the
    sampled outputs and host copies of the sampled units' inputs for the
    oracle leg."""
    import numpy as np
    from synth.device import to_device, alloc_output, draw_noise_c64, quantise_device, host_values
    t0 = time.time()
    bws = synth.make_batch(args.batch, workers=host_threads())
    bpairs = sum(x.n_templates * x.n_sft for x in bws)
    large = args.batch == 4
    if large:
        bdevs = [draw_noise_c64(x, seed=7000 + k) for k, x in enumerate(bws)]
    else:
        bdevs = [to_device(x, "c64")[0] for x in bws]
    bouts = [alloc_output(x) for x in bws]
    torch.cuda.synchronize()
    batch = {"workload": synth.BATCH_NAMES[args.batch].replace("-bf16", ""), "n_wu": len(bws),
             "pairs_per_step": bpairs, "inputs_s": time.time() - t0, "warmup": 1, "replays": args.batch_replays}
    def nfd_mix(c16):
        # (template, SFT) pairs per spindown block size, as the library splits
        # each unit's spindowns (16-blocks allowed; tiles of two sky points
        # taken for units of at least 4 sky points, which the library pairs
        # where their grid is dense enough; the pairing changes only the split)
        mix = {}
        for x in bws:
            for b, n in P.fstat_spindown_split(x.n_fd, coef16=c16, allow16=True, paired=x.n_sky >= 4).items():
                mix[b] = mix.get(b, 0) + x.n_sky * n * x.n_f * x.n_sft
        return mix
    dmax = max(x.dterms for x in bws)
    # sampled units: most, median and fewest SFTs; sky point 0, first and
    # last spindown, every frequency
    order = sorted(range(len(bws)), key=lambda k: -bws[k].n_sft)
    units = [order[0], order[len(order) // 2], order[-1]]
    ref = {"units": units, "ws": {k: bws[k] for k in units}, "sft": {}, "gpu": {}}
    tm = {}
    for k in units:
        x = bws[k]
        s, i, j = np.meshgrid([0], [0, x.n_fd - 1], np.arange(x.n_f), indexing="ij")
        tm[k] = (s.ravel().astype(np.int32), i.ravel().astype(np.int32), j.ravel().astype(np.int32))
    ref["templates"] = tm

    def timed(storage, c16=False):
        slots_b = sum(slots_per_pair("interp", dmax, b, c16) * n for b, n in nfd_mix(c16).items()) / bpairs
        with P.Plan(max_sft=max(x.n_sft for x in bws), max_bins=max(x.n_bins for x in bws),
                    max_sky=max(x.n_sky for x in bws), max_fd=max(x.n_fd for x in bws),
                    max_f=max(x.n_f for x in bws), max_dterms=16, storage=storage,
                    coef="f16" if c16 else "f32") as plan:
            if not large:
                # the 64-unit case runs with an autotuned launch shape: the batch
                # class is timed on the median unit (its single-unit class keeps
                # its default tile, written to the cache first)
                import tempfile
                k = order[len(order) // 2]
                fd, cache = tempfile.mkstemp(suffix=".tiles")
                os.close(fd)
                with open(cache, "w") as fh:
                    fh.write(f"s{P.STORAGE[storage]}_d{bws[k].dterms}_k0_c{int(c16)} 8 {5 if c16 else 4} 512 256\n")
                t1 = time.perf_counter()
                plan.autotune(bdevs[k], bouts[k], cache_path=cache)
                batch["autotune_s"] = time.perf_counter() - t1
                batch["tuned"] = open(cache).read().split("\n")[1]
                os.remove(cache)
            t1 = time.perf_counter()
            plan.batch_compute(bdevs, bouts)                   # warm-up: graph capture
            torch.cuda.synchronize()
            warm_s = time.perf_counter() - t1
            kms = []
            t1 = time.perf_counter()
            for _ in range(args.batch_replays):
                plan.batch_compute(bdevs, bouts)
                kms.append(plan.last_kernel_ms())
            torch.cuda.synchronize()
            el = (time.perf_counter() - t1) / args.batch_replays
        key = storage + ("+coef16" if c16 else "")
        ref["gpu"][key] = {k: take(bouts[k].twoF, tm[k]) for k in units}
        kmean = float(np.mean(kms))
        # HBM bytes per call from the committed counter summary (BF16 FP32-coefficient call of the 256-unit case)
        traffic = measured_traffic("demod_interp_batch", "large")[0] if (large and key == "bf16") else None
        return key, {"value": bpairs / el, "s_per_step": el, "warmup_s": warm_s, "kernel_s": kmean / 1e3,
                     "traffic": traffic, "slots_per_pair": slots_b,
                     "roofline_frac": slots_b * bpairs / (kmean * 1e-3) / PEAK_SLOTS,
                     "method_rate_vs_peak": method_slots(dmax) * bpairs / (kmean * 1e-3) / PEAK_SLOTS}

    forms = [f for f in getattr(args, "large_forms", "c64,bf16").split(",") if f] if large else ["c64"]
    say(f"batch {batch['workload']}: {len(bws)} units, {bpairs:.3e} pairs, inputs ready in {batch['inputs_s']:.1f} s")
    if large:
        for k in units:
            ref["sft"][k] = bdevs[k].sft.cpu().numpy().astype(np.float64).view(np.complex128)[..., 0]
    for form in [f for f in forms if f.startswith("c64")]:
        key, res = timed("c64", form.endswith("+coef16"))
        batch[key] = res
        say(f"batch {key}: {res}")
    if large and any(f.startswith("bf16") for f in forms):
        # the BF16 storage of the same values, unit by unit (the complex64
        # copy of each unit is released as its BF16 copy is made)
        for k in range(len(bdevs)):
            bdevs[k] = quantise_device(bdevs[k], "bf16")
        torch.cuda.empty_cache()
        for k in units:
            ref["sft"][("bf16", k)] = host_values(bdevs[k], "bf16")
        for form in [f for f in forms if f.startswith("bf16")]:
            key, res = timed("bf16", form.endswith("+coef16"))
            batch[key] = res
            say(f"batch {key}: {res}")
    if "bf16" in batch and "c64" in batch:
        batch["bf16_vs_c64"] = batch["bf16"]["value"] / batch["c64"]["value"]
    del bdevs, bouts
    torch.cuda.empty_cache()
    return batch, ref


def batch_errors(batch, ref, say):
    """Errors of the batched forms on the sampled units against the oracle:
    complex64 against the oracle on the complex64 values, BF16 against the
    oracle on its dequantised values (arithmetic) and on the complex64 values
    (storage)."""
    import numpy as np
    import oracle
    threads = host_threads()
    r64, r16 = [], []
    g = {key: [] for key in ref["gpu"]}
    for k in ref["units"]:
        w = ref["ws"][k]
        tm = ref["templates"][k]
        if w.sft is None and k not in ref["sft"]:
            return                          # no host copy of these inputs (complex64 form not run)
        r64.append(oracle.fstat(w, tm, sft=ref["sft"].get(k), nthreads=threads)["twoF"])
        if ("bf16", k) in ref["sft"]:
            r16.append(oracle.fstat(w, tm, sft=ref["sft"][("bf16", k)], nthreads=threads)["twoF"])
        for key in g:
            g[key].append(ref["gpu"][key][k])
    r64 = np.concatenate(r64)
    sample = (f"work units {ref['units']} (most, median and fewest SFTs): sky point 0, first and last spindown, "
              f"every frequency")
    for key in g:
        gk = np.concatenate(g[key])
        if key.startswith("c64"):
            batch[key]["err"] = err_stats(gk, r64)
            batch[key]["err"]["reference"] = "oracle on the complex64 values"
        else:
            batch[key]["err"] = err_stats(gk, np.concatenate(r16))
            batch[key]["err"]["reference"] = "oracle on the exactly dequantised BF16 values"
            batch[key]["storage_err_vs_c64"] = err_stats(gk, r64, tol=5e-3)
        batch[key]["err"]["sample"] = sample
    if "bf16" in batch and "c64" in batch and "err" in batch["bf16"] and "err" in batch["c64"]:
        ok = batch["bf16"]["err"]["at_metric_tolerance"] and batch["c64"]["err"]["at_metric_tolerance"]
        batch["mixed_exceeds_plain_at_tolerance"] = bool(ok and batch["bf16_vs_c64"] > 1.0)
    say(f"batch errors: { {k: batch[k].get('err') for k in g} }")


if __name__ == "__main__":
    main()
