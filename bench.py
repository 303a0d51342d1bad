#!/usr/bin/env python3
"""Benchmark of the F-statistic demodulation on one MI355X.

A step is one full pass of the hot path over one work unit: per (sky, SFT)
geometry and band check, then the demodulation kernel (bin index, phase,
Dirichlet window sums, a/b weighting, sum over SFTs and detectors, 2F).  The
workload is the work-unit-shaped case: 2 detectors x 1000 SFTs of 1800 s,
a 3600-bin band at 1000 Hz, 2000 sky points x 8 spindowns x 3600
frequencies, Dterms = 8 (5.76e7 templates, 1.15e11 template-SFT pairs).
Inputs are synthetic (seeded noise and injected signals) and resident in HBM
before the timed region.  Prints one JSON line.  Besides the forms of the
main case it times the direct kernel, the toplist-only output, the
semi-coherent sum of the same case split into 20 time segments and the
batched form on 256 work units with BF16 SFTs (one call each with FP32 and
FP16 coefficients, graph capture included); with
--workload semicoherent that split case is the main one (a step is then one
fstat_semicoherent call over all segments).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms c64,bf16,fp16]
                  [--workload workunit|semicoherent]
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
METRIC = "templates\u00b7SFTs/s for 2F (plain vs mixed-precision) at 2F rel err \u22641e-4; % roofline"


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


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle on the first sky points of the same work unit (every
    spindown, frequency and SFT), as many as fit in about `budget_s`."""
    import numpy as np
    import oracle
    nthreads = min(16, os.cpu_count() or 1)
    prep = oracle.Prepared(w)
    done_pairs, elapsed, n_sky = 0, 0.0, 0
    while elapsed < budget_s and n_sky < w.n_sky:
        tmpl = oracle.all_templates(w, [n_sky])
        t0 = time.perf_counter()
        prep.fstat(tmpl, nthreads=nthreads)
        elapsed += time.perf_counter() - t0
        done_pairs += len(tmpl[0]) * w.n_sft
        n_sky += 1
    return {"value": done_pairs / elapsed, "unit": "templates*SFTs/s", "cores": nthreads, "kind": "oracle",
            "sample": f"sky points 0..{n_sky - 1} of the same work unit: {n_sky * w.n_fd * w.n_f} templates "
                      f"x {w.n_sft} SFTs, FP64, {elapsed:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="c64,bf16,fp16,bf16+coef16",
                    help="SFT storage (c64, bf16, fp16), optionally +coef16 for the FP16-coefficient form")
    ap.add_argument("--kernel", default="auto", help="auto (= interp), interp or direct")
    ap.add_argument("--compare-direct", type=int, default=2,
                    help="also time this many steps of the direct kernel on complex64 storage")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--toplist", type=int, default=1000,
                    help="also time the plain form writing only a top-K toplist above 2F = 20 (0: skip)")
    ap.add_argument("--semicoherent", type=int, default=20,
                    help="also time the semi-coherent sum over this many segments of the same case (0: skip)")
    ap.add_argument("--batch", type=int, default=4, choices=[0, 3, 4],
                    help="also time the batched form on the 64-unit (3) or the 256-unit BF16 (4) case (0: skip)")
    ap.add_argument("--workload", default="workunit", choices=["workunit", "semicoherent"],
                    help="the case the forms are timed on: the work-unit-shaped case, or the same case as "
                         "--semicoherent segments combined by fstat_semicoherent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n} bytes read, {n} bytes written", file=sys.stderr, flush=True)
        del src, dst
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
    print(f"[bench] workload {case_name}: {n_sft_total} SFTs in {len(case)} part(s) x {w.n_bins} bins, "
          f"{w.n_templates} templates (generated in {time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    pairs = w.n_templates * n_sft_total
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    for form in forms:
        storage, _, extra = form.partition("+")
        coef = "f16" if extra == "coef16" else "f32"
        wus = [to_device(x, storage)[0] for x in case]
        out = alloc_output(w)
        torch.cuda.synchronize()
        with P.Plan(max_sft=max(x.n_sft for x in case), max_bins=max(x.n_bins for x in case), max_sky=w.n_sky,
                    max_fd=w.n_fd, max_f=w.n_f, max_dterms=w.dterms, storage=storage, coef=coef,
                    kernel=args.kernel) as plan:
            step = (lambda: plan.semicoherent(wus, out)) if semi_main else (lambda: plan.compute(wus[0], out))
            steps = args.steps if form == forms[0] else max(2, args.steps // 2)
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            kms = []
            t_start = time.perf_counter()
            for _ in range(steps):
                step()
                kms.append(plan.last_kernel_ms())
            torch.cuda.synchronize()
            el = time.perf_counter() - t_start
        results[form] = {"steps": steps, "ms_per_step": 1e3 * el / steps, "value": steps * pairs / el,
                         "kernel_ms": float(np.mean(kms)),
                         # the 2F error bound each form is tested to against the FP64 oracle
                         "err_bound": 5e-3 if (coef == "f16" or storage != "c64") else 1e-4}
        print(f"[bench] {form}: {results[form]}", file=sys.stderr, flush=True)
        del wus, out
        torch.cuda.empty_cache()

    kernel = "direct" if args.kernel == "direct" else "interp"     # the library resolves auto to interp
    kernels = {}
    if args.compare_direct > 0 and kernel != "direct" and not semi_main:
        wu, _ = to_device(w, "c64")
        out = alloc_output(w)
        with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                    max_dterms=w.dterms, storage="c64", kernel="direct") as plan:
            plan.compute(wu, out)
            torch.cuda.synchronize()
            kms = []
            t_start = time.perf_counter()
            for _ in range(args.compare_direct):
                plan.compute(wu, out)
                kms.append(plan.last_kernel_ms())
            torch.cuda.synchronize()
            el = time.perf_counter() - t_start
        kernels["direct"] = {"value": args.compare_direct * pairs / el, "kernel_ms": float(np.mean(kms)),
                             "roofline_frac": slots_per_pair("direct", w.dterms) * pairs / (np.mean(kms) * 1e-3) / PEAK_SLOTS}
        print(f"[bench] direct c64: {kernels['direct']}", file=sys.stderr, flush=True)
        del wu, out
        torch.cuda.empty_cache()
    toplist = None
    if args.toplist > 0 and not semi_main:
        wu, _ = to_device(w, "c64")
        out = alloc_output(w, top_k=args.toplist, threshold=20.0, full=False)
        with P.Plan(max_sft=w.n_sft, max_bins=w.n_bins, max_sky=w.n_sky, max_fd=w.n_fd, max_f=w.n_f,
                    max_dterms=w.dterms, kernel=args.kernel) as plan:
            plan.compute(wu, out)
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            for _ in range(2):
                plan.compute(wu, out)
            torch.cuda.synchronize()
            el = time.perf_counter() - t_start
        n_above = int(out.n_above.cpu().item())
        toplist = {"top_k": args.toplist, "threshold": 20.0, "n_above": n_above, "ms_per_step": 1e3 * el / 2,
                   "value": 2 * pairs / el, "full_2F_written": False}
        print(f"[bench] toplist: {toplist}", file=sys.stderr, flush=True)
        del wu, out
        torch.cuda.empty_cache()
    semi = None
    if args.semicoherent > 0 and not semi_main:
        t0 = time.time()
        segs = synth.make_segment_config(args.semicoherent)
        spairs = segs[0].n_templates * sum(x.n_sft for x in segs)
        devs = [to_device(x, "c64")[0] for x in segs]
        out = alloc_output(segs[0])
        gen_s = time.time() - t0
        semi = {"workload": segs[0].name.rsplit("-", 1)[0], "n_seg": len(segs),
                "n_sft": [int(x.n_sft) for x in segs][:3] + ["..."], "pairs_per_step": spairs}
        for coef in ("f32", "f16"):
            with P.Plan(max_sft=max(x.n_sft for x in segs), max_bins=max(x.n_bins for x in segs),
                        max_sky=segs[0].n_sky, max_fd=segs[0].n_fd, max_f=segs[0].n_f, max_dterms=segs[0].dterms,
                        coef=coef, kernel=args.kernel) as plan:
                plan.semicoherent(devs, out)
                torch.cuda.synchronize()
                kms = []
                t_start = time.perf_counter()
                for _ in range(2):
                    plan.semicoherent(devs, out)
                    kms.append(plan.last_kernel_ms())
                torch.cuda.synchronize()
                el = time.perf_counter() - t_start
            semi["coef16" if coef == "f16" else "plain"] = {
                "value": 2 * spairs / el, "ms_per_step": 1e3 * el / 2, "kernel_ms": float(np.mean(kms)),
                "roofline_frac": slots_per_pair(kernel, segs[0].dterms, coef16=coef == "f16") * spairs
                / (np.mean(kms) * 1e-3) / PEAK_SLOTS,
                "err_bound": 5e-3 if coef == "f16" else 1e-4}
        print(f"[bench] semi-coherent ({gen_s:.1f} s to generate): {semi}", file=sys.stderr, flush=True)
        del devs, out
        torch.cuda.empty_cache()
    batch = None
    if args.batch and not semi_main and kernel != "direct":
        from synth.device import draw_noise_16bit
        t0 = time.time()
        bws = synth.make_batch(args.batch, workers=min(16, os.cpu_count() or 1))
        bpairs = sum(x.n_templates * x.n_sft for x in bws)
        storage = "bf16" if args.batch == 4 else "c64"
        if args.batch == 4:
            bdevs = [draw_noise_16bit(x, "bf16", seed=7000 + k) for k, x in enumerate(bws)]
        else:
            bdevs = [to_device(x, "c64")[0] for x in bws]
        bouts = [alloc_output(x) for x in bws]
        torch.cuda.synchronize()
        batch = {"workload": synth.BATCH_NAMES[args.batch], "n_wu": len(bws), "pairs_per_step": bpairs,
                 "storage": storage, "inputs_s": time.time() - t0}
        nfd_mix = {8: 0, 4: 0}
        for x in bws:
            rem = x.n_fd % 8
            lanes8 = x.n_fd if rem > 4 else x.n_fd - rem
            nfd_mix[8] += x.n_sky * lanes8 * x.n_f * x.n_sft
            nfd_mix[4] += x.n_sky * (x.n_fd - lanes8) * x.n_f * x.n_sft
        for coef in ("f32", "f16"):
            c16 = coef == "f16"
            slots_b = (slots_per_pair(kernel, 8, 8, c16) * nfd_mix[8] + slots_per_pair(kernel, 8, 4, c16) * nfd_mix[4]) / bpairs
            with P.Plan(max_sft=max(x.n_sft for x in bws), max_bins=max(x.n_bins for x in bws),
                        max_sky=max(x.n_sky for x in bws), max_fd=max(x.n_fd for x in bws),
                        max_f=max(x.n_f for x in bws), max_dterms=16, storage=storage, coef=coef) as plan:
                reps = 1 if args.batch == 4 else 2            # the first call also captures the graph
                kms = []
                t_start = time.perf_counter()
                for _ in range(reps):
                    plan.batch_compute(bdevs, bouts)
                    kms.append(plan.last_kernel_ms())
                torch.cuda.synchronize()
                el = (time.perf_counter() - t_start) / reps
            key = "coef16" if coef == "f16" else "plain"
            batch[key] = {"value": bpairs / el, "s_per_step": el, "kernel_s": float(np.mean(kms)) / 1e3,
                          "slots_per_pair": slots_b,
                          "roofline_frac": slots_b * bpairs / (np.mean(kms) * 1e-3) / PEAK_SLOTS,
                          "err_bound": 5e-3 if (coef == "f16" or storage != "c64") else 1e-4}
            print(f"[bench] batch {key}: {batch[key]}", file=sys.stderr, flush=True)
        batch["coef16_vs_plain"] = batch["coef16"]["value"] / batch["plain"]["value"]
        del bdevs, bouts
        torch.cuda.empty_cache()
    traffic_key = "semicoherent" if semi_main else "config1"
    main_form = forms[0]
    r = results[main_form]
    main_c16 = main_form.endswith("+coef16")
    traffic, launches = measured_traffic("demod_interp_coef16" if main_c16 else f"demod_{kernel}", traffic_key)
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
                   "phase": "fp64", "kernel": kernel, "templates": w.n_templates, "pairs_per_step": pairs,
                   **({"n_seg": len(case)} if semi_main else {})},
        "forms": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"], "kernel_ms": v["kernel_ms"],
                      "err_bound": v["err_bound"],
                      "vs_plain": v["value"] / results[main_form]["value"],
                      "roofline_frac": slots_per_pair(kernel, w.dterms, coef16=k.endswith("+coef16")) * pairs
                      / (v["kernel_ms"] * 1e-3) / PEAK_SLOTS,
                      "traffic": measured_traffic("demod_interp_coef16" if k.endswith("+coef16") else f"demod_{kernel}",
                                                  traffic_key)[0]}
                  for k, v in results.items()},
        "kernels": kernels,
        "toplist": toplist,
        "semicoherent": semi,
        "batch": batch,
        # per demodulation pass: all launches of the kernel in one step (the
        # library may split the SFT loop into several), timed together
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_SLOTS, "traffic": traffic, "launches_per_pass": launches,
                     "kernel": f"demod_{kernel}", "slots_per_pair": slots_per_pair(kernel, w.dterms, coef16=main_c16),
                     "kernel_ms": r["kernel_ms"]},
    }
    if not args.no_cpu_baseline and not semi_main:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
