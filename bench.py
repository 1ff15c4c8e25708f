#!/usr/bin/env python3
"""Benchmark: greedy D-optimal sensor selection on one MI355X.

One timed step = one complete selection of `budget` sensors on the synthetic
600-sensor x 128-observation instance (K is 76,800 x 76,800 FP64, formed on the
GPU before timing): reload of the working copy from K (oed_reset) plus
oed_greedy(budget), all inside liboed's HIP kernels.  `value` is greedy steps
(picks) per second of the mixed-precision path (FP32 downdate on MFMA, FP64
factorisations); the plain FP64 path runs beside it on the same K.

Prints one JSON line (rank 0).  Only N=1 is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MFMA peaks of the downdate's arithmetic type (the split-product variant runs on BF16)
PEAK_TFLOPS = {"fp64": 78.6, "mixed_f32": 157.3, "mixed_bf16x3": 2500.0}
SYRK_KERNEL = {"fp64": "syrk_lds_kernel<double>", "mixed_f32": "syrk_lds_kernel<float>",
               "mixed_bf16x3": "syrk_bf16_kernel"}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="mixed_600x128")
    ap.add_argument("--budget", type=int, default=None, help="override the budget (not the headline)")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed_f32", "mixed_bf16x3"],
                    help="override the configuration's precision (not the headline)")
    ap.add_argument("--peaks", action="store_true",
                    help="measure the box's own ceilings (device copy, vendor GEMMs) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 4 times (HBM counter calibration)")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-bf16x3", action="store_true")
    ap.add_argument("--no-left", action="store_true", help="skip the left-looking legs")
    ap.add_argument("--left", action="store_true", help="batched workload: left-looking method")
    ap.add_argument("--branches", type=int, default=0,
                    help="batched workload: concurrent launch sequences (0: the library's choice)")
    ap.add_argument("--no-graph", action="store_true", help="batched workload: enqueue every run eagerly")
    ap.add_argument("--no-gaps", action="store_true", help="skip the per-step top-two gap scan (FP64)")
    ap.add_argument("--delay", type=int, default=0, help="downdate delay depth (0: the library's choice)")
    ap.add_argument("--tile-order", default="auto", choices=["auto", "row8", "col8", "col4", "col2"],
                    help="downdate tile order (auto: the autotuner's choice, else the library default)")
    ap.add_argument("--tile-size", type=int, default=0, choices=[0, 128, 256],
                    help="BF16 split-product downdate tile edge (0: the autotuner's choice)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="with --delay 0, take the library's fixed default instead of its autotuner")
    ap.add_argument("--no-eval", action="store_true", help="skip the design-evaluation leg")
    ap.add_argument("--eval-designs", type=int, default=64,
                    help="designs of the evaluation leg: the greedy one, the uniform one and random ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=int, default=16, help="picks of the oracle sample")
    ap.add_argument("--cpu-sensors", type=int, default=100)
    return ap.parse_args()


def timed_selections(sel, K, budget, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for s in range(steps):
        sel.reset(K)
        out = sel.greedy(budget)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, out


def syrk_kernel_name(prec, variant=1):
    """The downdate kernel a handle launches: variant 0 the direct kernel (delay 1), 1 the LDS kernel of
    128 x 128 tiles, 2 the BF16 split-product kernel of 256 x 256 tiles."""
    if variant == 0:
        return "syrk_direct_kernel<double>" if prec == "fp64" else "syrk_direct_kernel<float>"
    if variant == 2:
        return "syrk_bf16_big_kernel"
    return SYRK_KERNEL[prec]


def roofline_syrk(prof, prec, workload=None, delay=None, variant=1):
    """The downdate R -= W W^T: algorithmic flops (2 per multiply-add of the lower-triangle
    blocks) over its summed HIP-event time.  The BF16 split product executes three MFMA
    products per algorithmic one; its fraction is taken of the BF16 peak on the executed
    flops, and the HBM view (algorithmic bytes / time) is given beside it."""
    kname = syrk_kernel_name(prec, variant)
    ms = prof["ms"]["syrk"]
    n = max(1, prof["launches"]["syrk"])
    tflops = prof["syrk_flops"] / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    gbs = prof["syrk_bytes"] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    executed = tflops * (3 if prec == "mixed_bf16x3" else 1)
    out = {
        "kernel": kname,
        "bound": "mfma",
        "achieved": round(executed, 3),
        "peak": PEAK_TFLOPS[prec],
        "unit": "TFLOP/s",
        "frac": round(executed / PEAK_TFLOPS[prec], 4),
        "traffic": counted_traffic(workload, prec, kname, delay) if workload else None,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_bytes_per_launch": round(prof["syrk_bytes"] / n),
        "avg_launch_ms": round(ms / n, 4),
        "launches": n,
        "algorithmic_tflops": round(tflops, 3),
        "algorithmic_gbs": round(gbs, 1),
        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
    }
    if prec == "mixed_bf16x3":
        # three BF16 products per FP32 one: the kernel is bound by its HBM stream instead
        out.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "executed_bf16_tflops": round(executed, 3),
                    "bf16_mfma_frac": round(executed / PEAK_TFLOPS[prec], 4)})
    return out


def compare_picks(idx, gain, idx_ref, gain_ref):
    import numpy as np
    budget = len(idx_ref)
    agree = int(np.sum(idx == idx_ref))
    first_div = next((k for k in range(budget) if idx[k] != idx_ref[k]), None)
    upto = budget if first_div is None else first_div
    gerr = float(np.max(np.abs(gain[:upto] - gain_ref[:upto]) / np.maximum(1, np.abs(gain_ref[:upto])))) \
        if upto else 0.0
    return {"same_picks": agree == budget, "picks_equal_at_position": agree, "first_divergence_step": first_div,
            "max_rel_gain_diff_before_divergence": gerr, "per_step_rel_gain_diff": per_step_diff(gain, gain_ref, upto)}


def measured_peaks():
    """What this GPU reaches outside the selection kernels, as ceilings to read the roofline
    fractions against: a device-to-device copy of 4 GiB (HBM read + write) and the vendor GEMMs
    (torch.mm, square, contiguous operands) in FP32, FP64 and BF16, timed with HIP events on
    torch's stream after one untimed call."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    dev = "cuda:0"

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {}
    src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = timed(lambda: dst.copy_(src), 10)
    out["copy"] = {"bytes_moved": 2 * 4 << 30, "ms": round(ms, 3), "TB/s": round(2 * 4 * (1 << 30) / ms / 1e9, 3),
                   "frac_of_8TB/s": round(2 * 4 * (1 << 30) / ms / 1e9 / 8.0, 4)}
    del src, dst
    peak = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}
    out["gemm"] = []
    for name, dt, N in (("fp32", torch.float32, 8192), ("fp32", torch.float32, 16384), ("fp64", torch.float64, 8192),
                        ("bf16", torch.bfloat16, 8192), ("bf16", torch.bfloat16, 16384)):
        g = torch.Generator(device=dev)
        g.manual_seed(N)
        x = torch.randn(N, N, device=dev, dtype=torch.float32, generator=g).to(dt)
        y = torch.randn(N, N, device=dev, dtype=torch.float32, generator=g).to(dt)
        ms = timed(lambda: torch.mm(x, y), 5)
        tf = 2.0 * N ** 3 / ms / 1e9
        out["gemm"].append({"dtype": name, "N": N, "ms": round(ms, 3), "TFLOP/s": round(tf, 1),
                            "frac_of_peak": round(tf / peak[name], 4)})
        log(f"torch.mm {name} {N}: {tf:.1f} TFLOP/s")
        del x, y
    print(json.dumps({"measured_peaks": out, "device": torch.cuda.get_device_name(0)}), flush=True)


def copy_calibration():
    """A plain device-to-device copy of 2^28 floats (1 GiB read + 1 GiB written), four times:
    what FETCH_SIZE / WRITE_SIZE read for it scales the counters of the selection kernels."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 1 << 30, "bytes_written": 1 << 30, "launches": 4}}),
          flush=True)


def source_digest():
    """SHA-256 of the downdate kernels' source: HBM traffic counted for other source is stale."""
    import hashlib
    h = hashlib.sha256()
    for f in ("oed_update.hip", "oed_device.h", "oed_internal.h"):
        with open(os.path.join(ROOT, "paper_2604_08812_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(workload, prec, kernel_name, delay):
    """HBM bytes per launch of the downdate at this delay depth (W slots per launch) from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the copy calibration), or None
    when absent, taken at another depth or on other source."""
    path = os.path.join(ROOT, "profiles", f"syrk_hbm_traffic_{workload}.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(prec)
    if not ent or ent.get("source_sha256") != source_digest() or ent.get("kernel") != kernel_name:
        return None
    at = ent.get("by_delay", {}).get(str(delay))
    return at.get("hbm_bytes_per_launch") if at else None


def naive_flops(n, N_t, budget):
    """Flops of the oracle's from-scratch greedy: at step k (1-based) every one of the n - k + 1
    remaining candidates factors a (k N_t)^2 matrix, (k N_t)^3 / 3 flops."""
    return sum((n - k + 1) * (k * N_t) ** 3 / 3.0 for k in range(1, budget + 1))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(K, N_t, s2, n_sensors, budget, full_shape=None, single_budget=6):
    """The oracle (from-scratch FP64 Cholesky of every test matrix, OpenMP over candidates)
    on the first n_sensors sensors of the same K; a shorter single-thread run beside it, and
    the full-size time extrapolated from the measured flop rate."""
    import numpy as np

    import oracle
    from oed_inputs import k_sub_lower
    sub = k_sub_lower(K, N_t, list(range(n_sensors)))
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    res = oracle.greedy(sub, n_sensors, N_t, s2, budget, threads=threads)
    dt = time.perf_counter() - t0
    rate = naive_flops(n_sensors, N_t, budget) / dt
    t1 = time.perf_counter()
    oracle.greedy(sub, n_sensors, N_t, s2, single_budget, threads=1)
    dt1 = time.perf_counter() - t1
    out = {"value": round(budget / dt, 4), "unit": "greedy steps/s", "cores": threads, "kind": "oracle",
           "sample": f"sensors 0..{n_sensors - 1} of the same K ({n_sensors * N_t}^2 principal block), "
                     f"budget {budget}, {dt:.1f} s", "seconds": round(dt, 2),
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "oracle_gflops": round(rate / 1e9, 2),
           "single_thread": {"budget": single_budget, "seconds": round(dt1, 2),
                             "greedy_steps_per_s": round(single_budget / dt1, 4),
                             "gflops": round(naive_flops(n_sensors, N_t, single_budget) / dt1 / 1e9, 2)},
           "idx": [int(x) for x in res["idx"]], "gain": [float(x) for x in np.asarray(res["gain"])]}
    if full_shape:
        N_s, B = full_shape
        out["full_size_extrapolated_s"] = {
            "value": round(naive_flops(N_s, N_t, B) / rate, 1),
            "note": f"extrapolated, not measured: {naive_flops(N_s, N_t, B):.3g} oracle flops for "
                    f"{N_s} sensors, budget {B}, at the sample's measured rate"}
    return out


def top_two_gaps(sel, K, budget):
    """Relative gap between the best and second-best FP64 score at every step (the near-tie
    margin that the pick comparisons depend on)."""
    import numpy as np
    sel.reset(K)
    gaps = []
    for k in range(budget):
        g = sel.scores()
        fin = np.sort(g[np.isfinite(g)])
        if fin.size >= 2:
            gaps.append((fin[-1] - fin[-2]) / max(abs(fin[-1]), 1.0))
        sel.greedy(1)
    gaps = np.array(gaps)
    return {"per_step": [float(x) for x in gaps], "steps": int(gaps.size), "min": float(gaps.min()), "median": float(np.median(gaps)),
            "below_2e-4": int(np.sum(gaps <= 2e-4)), "below_2e-10": int(np.sum(gaps <= 2e-10)),
            "quantiles_10_50_90": [float(x) for x in np.quantile(gaps, [0.1, 0.5, 0.9])]}


def per_step_diff(gain, gain_ref, upto):
    import numpy as np
    if not upto:
        return None
    d = np.abs(gain[:upto] - gain_ref[:upto]) / np.maximum(1, np.abs(gain_ref[:upto]))
    return {"max": float(d.max()), "median": float(np.median(d)), "p90": float(np.quantile(d, 0.9))}


# The paper's own figures for its greedy (Sec. IV), quoted as context: other hardware, its real
# data-space matrix, Algorithm 1 with pipelined file I/O; it reports no steps/s or TFLOP/s.
PAPER_CONTEXT = {
    "note": "context only, not a target: other hardware, the paper's real K, its own loop order and I/O",
    "greedy_wall_time": "about 1.5 h for the full selection",
    "hardware": "16 x NVIDIA A100 (Perlmutter)",
    "workload": "600 candidate sensors x 420 observations (K 252,000^2, 508 GB FP64 on disk), budget 175",
    "derived_greedy_steps_per_s": round(175 / 5400.0, 4),
    "scaling": "near-ideal strong and weak scaling up to 1,024 A100 (Perlmutter) and 2,048 MI250X GCDs "
               "(Frontier)",
    "single_gpu_capacity": "at most 300 / 340 / 530 picks at N_t = 420 on one MI250X GCD / A100 80 GB / MI300X",
}


def design_evaluation(K, spec, s2, prec, budget, idx, gain, n):
    """Objective of the greedy design (pick order), the uniformly spaced one and n - 2 random
    ones of the same size, in batched launch sequences of n/2 designs; a warm-up run captures
    the graph, the second run is timed."""
    import numpy as np
    import torch
    from paper_2604_08812_amd import Evaluator
    rng = np.random.default_rng(5)
    unif = np.round(np.linspace(0, spec.N_s - 1, budget)).astype(np.int32)
    rand = [rng.permutation(spec.N_s)[:budget] for _ in range(n - 2)]
    designs = np.stack([np.asarray(idx, dtype=np.int32), unif] + rand).astype(np.int32)
    nb = (n + 1) // 2
    with Evaluator(K, spec.N_s, spec.N_t, s2, budget, max_batch=nb, precision=prec, profile=True) as ev:
        ev.run(designs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obj, terms = ev.run(designs)
        wall = time.perf_counter() - t0
        st = ev.stats()
    r = obj[2:]
    mu, sd = float(r.mean()), float(r.std(ddof=1))
    log(f"design evaluation: {n} designs of {budget} in {wall:.2f} s; greedy {obj[0]:.6f}, uniform {obj[1]:.6f}, "
        f"random mean {mu:.6f} sd {sd:.3e} max {r.max():.6f}")
    return {"value": round(n / wall, 3), "unit": "designs/s", "designs": n, "B": budget, "precision": prec,
            "batch": st["batch"], "ms_per_design": round(wall * 1e3 / n, 3),
            "graph_ms": round(st["run_ms"], 3),
            "downdate_tflops_over_run": round(st["syrk_flops"] / (st["run_ms"] * 1e-3) / 1e12, 3)
            if st["run_ms"] > 0 else None,
            "greedy_objective": float(obj[0]), "uniform_objective": float(obj[1]),
            "random_mean": mu, "random_sd": sd, "random_max": float(r.max()),
            "greedy_z_score": round((float(obj[0]) - mu) / sd, 3) if sd > 0 else None,
            "greedy_above_best_random_in_sd": round((float(obj[0]) - float(r.max())) / sd, 3) if sd > 0 else None,
            "greedy_terms_vs_gains_max_rel": float(np.max(np.abs(terms[0] - gain) / np.maximum(1, np.abs(gain))))}


def run_paper_shape(args):
    """The paper's shape, 600 sensors x 420 observations, mixed FP32 (or --precision mixed_bf16x3,
    the BF16 split product; FP64 would need 254 GB for the working copy alone).  K (252,000^2) is never whole:
    F stays resident and K's row panels are formed by GEMM and packed one at a time (untimed, like
    the formation of K elsewhere).  A step is one oed_greedy(175) on the packed working copy; the
    selection conditions the working copy, so each step after the first resets and packs again,
    outside the timed region."""
    import torch

    from oed_inputs import CONFIGS, f_matrix, k_row_panels
    from paper_2604_08812_amd import Selector, library
    library()
    spec = CONFIGS["paper_600x420"]
    budget = args.budget or spec.budget
    prec = args.precision or "mixed_f32"
    if prec == "fp64":
        sys.exit("the paper's shape runs the mixed precisions: an FP64 working copy would take 254 GB")
    t0 = time.perf_counter()
    F, scale = f_matrix(spec.N_d, spec.n_m, spec.seed, device="cuda:0", dtype=torch.float32,
                        progress=lambda i, n: log(f"  F column chunk {i}/{n}") if i % 4 == 0 or i == n else None)
    s2 = spec.c * scale
    torch.cuda.synchronize()
    log(f"F {spec.N_d} x {spec.n_m} formed in {time.perf_counter() - t0:.1f} s, sigma2={s2:.6e}")
    sel = Selector(None, spec.N_s, spec.N_t, s2, precision=prec, profile=True, delay=args.delay)
    delay, variant, _, tiles = sel.config()

    def pack(target, panel=56):
        t = time.perf_counter()
        for s0, n, P in k_row_panels(F, spec.N_s, spec.N_t, s2, panel):
            target.pack_rows(P, s0, n)
            del P
        torch.cuda.synchronize()
        return time.perf_counter() - t

    pack_s = []
    for w in range(args.warmup):
        pack_s.append(pack(sel))
        sel.greedy(budget)
        sel.reset(None)
        log(f"warmup {w + 1}/{args.warmup} done")
    ms_list = []
    sel.profile(reset=True)
    for st in range(args.steps):
        pack_s.append(pack(sel))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx, gain = sel.greedy(budget)
        torch.cuda.synchronize()
        ms_list.append((time.perf_counter() - t0) * 1e3)
        log(f"step {st + 1}/{args.steps}: {ms_list[-1]:.1f} ms")
        if st + 1 < args.steps:
            sel.reset(None)
    prof = sel.profile(reset=True)
    dev_bytes = sel.device_bytes()
    sel.close()
    ms = sum(ms_list) / len(ms_list)
    left = None
    if not args.no_left:
        # left-looking (Algorithm 1's order) on the same K: pack, free F (the W history needs
        # the room), one timed selection
        sell = Selector(None, spec.N_s, spec.N_t, s2, precision=prec, profile=True, method="left",
                        max_budget=budget)
        # the BF16 blocks are padded to 448 rows and its W history holds hi and lo parts: narrower
        # row panels keep F, the panel, R and the history within the GPU's memory
        pack_l = pack(sell, 56 if prec == "mixed_f32" else 14)
        del F
        torch.cuda.empty_cache()
        F = None
        torch.cuda.synchronize()
        sell.profile(reset=True)
        t0 = time.perf_counter()
        il, gl = sell.greedy(budget)
        torch.cuda.synchronize()
        msl = (time.perf_counter() - t0) * 1e3
        pl = sell.profile(reset=True)
        devl = sell.device_bytes()
        sell.close()
        log(f"left-looking: {msl:.1f} ms per selection")
        tfl = pl["syrk_flops"] / (pl["ms"]["syrk"] * 1e-3) / 1e12 if pl["ms"]["syrk"] > 0 else 0.0
        ex = 3 if prec == "mixed_bf16x3" else 1  # BF16 split product: three MFMA products per one
        left = {"value": round(budget / (msl * 1e-3), 3), "unit": "greedy steps/s", "ms_per_step": round(msl, 3),
                "column_kernel": {"kernel": "column_bf16_rt_kernel" if ex == 3 else "column_rt_kernel<float>",
                                  "algorithmic_tflops": round(tfl, 3), "executed_tflops": round(ex * tfl, 3),
                                  "peak": PEAK_TFLOPS[prec], "frac": round(ex * tfl / PEAK_TFLOPS[prec], 4),
                                  "algorithmic_flops_per_selection": pl["syrk_flops"]},
                "kernel_ms_per_step": {k: round(v, 3) for k, v in pl["ms"].items()},
                "pack_s": round(pack_l, 3), "device_bytes_of_handle": devl,
                "vs_right_looking": compare_picks(il, gl, idx, gain)}
    result = {
        "metric": "greedy steps/s + SYRK TFLOP/s (% MFMA peak), mixed vs FP64, same picks",
        "value": round(budget / (ms * 1e-3), 3), "unit": "greedy steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == "mixed_f32" else "bf16x3", "data": "synthetic",
        "config": {"workload": spec.name, "N_s": spec.N_s, "N_t": spec.N_t, "n_m": spec.n_m, "seed": spec.seed,
                   "budget": budget, "precision": prec, "K_dtype": "f32 (row panels, never whole)",
                   "delay": delay, "downdate_variant": ["direct", "lds", "lds256"][variant],
                   "step": "oed_greedy(budget) on the packed working copy"},
        "roofline": {**roofline_syrk(prof, prec, spec.name, delay),
                     "kernel": "syrk_bf16_rt_kernel" if prec == "mixed_bf16x3" else
                     "syrk_direct_kernel<float>" if variant == 0 else "syrk_lds_rt_kernel<float>"},
        "kernel_ms_per_step": {k: round(v / args.steps, 3) for k, v in prof["ms"].items()},
        "pack_s_per_fill": round(sum(pack_s) / len(pack_s), 3),
        "device_bytes_of_handle": dev_bytes,
        "picks_head": [int(x) for x in idx[:10]], "gain_first_last": [float(gain[0]), float(gain[-1])],
        "paper_context": PAPER_CONTEXT,
    }
    if left is not None:
        result["left_looking_" + prec] = left
    del F
    print(json.dumps(result), flush=True)


def batched_checks(specs, items, res, prec, delay, method, args):
    """The timed batch's picks and gains against a single handle per instance (same kernels and
    delay: equal bit for bit), and the oracle on a bounded sample: the instances with N_t <= 32,
    each restricted to its first min(N_s, 100) sensors with budget min(N_s, 100) // 4, selected
    by the GPU as one batch and by the oracle instance by instance (timed: the cpu_baseline)."""
    import numpy as np

    import oracle
    from oed_inputs import k_sub_lower
    from paper_2604_08812_amd import BatchSelector, Selector
    same, worst = 0, 0.0
    for (K, N_s, N_t, s2, B), (idx, gain, stt) in zip(items, res):
        kw = {"method": "left", "max_budget": B} if method == "left" else {"delay": delay}
        with Selector(K, N_s, N_t, s2, precision=prec, **kw) as sel:
            i1, g1 = sel.greedy(B)
        if stt == 0 and list(idx) == list(i1):
            same += 1
            worst = max(worst, float(np.max(np.abs(gain - g1) / np.maximum(1.0, np.abs(g1)))))
    out = {"batch_vs_single_handles": {"instances_with_equal_picks": same, "instances": len(items),
                                       "max_rel_gain_diff": worst}}
    if args.no_cpu_baseline:
        return out
    sample = [(q, min(sp.N_s, 100)) for q, sp in enumerate(specs) if sp.N_t <= 32]
    sub_items = [(items[q][0], n, specs[q].N_t, items[q][3], n // 4) for q, n in sample]
    kw = {"method": "left"} if method == "left" else {"delay": delay}
    with BatchSelector(sub_items, precision=prec, **kw) as sb:
        gres = sb.run()
    threads = oracle.default_threads()
    agree, gerr, secs, flops = 0, 0.0, 0.0, 0.0
    for (q, n), (idx, gain, _) in zip(sample, gres):
        sp = specs[q]
        sub = k_sub_lower(items[q][0], sp.N_t, range(n))
        t0 = time.perf_counter()
        ref = oracle.greedy(sub, n, sp.N_t, items[q][3], n // 4, threads=threads)
        secs += time.perf_counter() - t0
        flops += naive_flops(n, sp.N_t, n // 4)
        if list(ref["idx"]) == list(idx):
            agree += 1
            gerr = max(gerr, float(np.max(np.abs(gain - ref["gain"]) / np.maximum(1.0, np.abs(ref["gain"])))))
    steps = sum(n // 4 for _, n in sample)
    out["cpu_baseline"] = {
        "value": round(steps / secs, 4), "unit": "greedy steps/s", "cores": threads, "kind": "oracle",
        "sample": f"the {len(sample)} instances with N_t <= 32, each on its first min(N_s, 100) sensors with "
                  f"budget min(N_s, 100) // 4 ({steps} picks), {secs:.1f} s",
        "seconds": round(secs, 2), "oracle_gflops": round(flops / secs / 1e9, 2), "cpu_model": cpu_model(),
        "gpu_same_sample_instances_with_equal_picks": agree, "gpu_same_sample_instances": len(sample),
        "gpu_same_sample_max_rel_gain_err": gerr}
    return out


def run_batched(args):
    """The 48 uneven designs (seeds 100+i), FP32 K, mixed precision, one graph launch per run."""
    import torch

    from oed_inputs import batched_instance_specs, make_K_lower_panels
    from paper_2604_08812_amd import BatchSelector, library
    library()
    specs = batched_instance_specs()
    dev = torch.device("cuda:0")
    items = []
    t0 = time.perf_counter()
    for q, sp in enumerate(specs):
        K, s2 = make_K_lower_panels(sp.N_s, sp.N_t, sp.n_m, sp.seed, sp.c, device=dev, dtype=torch.float32)
        items.append((K, sp.N_s, sp.N_t, s2, sp.budget))
        if (q + 1) % 8 == 0:
            log(f"  formed {q + 1}/{len(specs)} instances")
    torch.cuda.synchronize()
    log(f"48 instances formed in {time.perf_counter() - t0:.1f} s")
    total_steps = sum(sp.budget for sp in specs)
    tune = args.delay == 0 and not args.no_autotune and not args.left
    bs = BatchSelector(items, precision=args.precision or "mixed_f32", profile=True, delay=args.delay, autotune=tune,
                       method="left" if args.left else "right", branches=args.branches, graph=not args.no_graph,
                       tile_order=args.tile_order)
    delay, tuned, tiles, branches = bs.config()
    for w in range(args.warmup):
        bs.reset(items)
        bs.run()
    ms_list = []
    res = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        bs.reset(items)
        res = bs.run()
        ms_list.append(bs.stats()["run_ms"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    st = bs.stats()
    run_ms = sum(ms_list) / len(ms_list)
    bs.close()
    prec = args.precision or "mixed_f32"
    checks = batched_checks(specs, items, res, prec, delay, "left" if args.left else "right", args)
    gbs = st["syrk_bytes"] / (run_ms * 1e-3) / 1e9
    result = {
        "metric": "greedy steps/s + SYRK TFLOP/s (% MFMA peak), mixed vs FP64, same picks",
        "value": round(total_steps / (ms * 1e-3), 3), "unit": "greedy steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_48_uneven", "instances": len(specs), "total_picks": total_steps,
                   "precision": args.precision or "mixed_f32", "K_dtype": "f32", "delay": delay, "tile_order": tiles,
                   "branches": branches, "graph": not args.no_graph, "autotuned": tune,
                   "method": "left-looking" if args.left else "right-looking",
                   "autotuner_run_ms_by_delay": [round(float(x), 3) for x in tuned] if tune else None,
                   "step": "oed_batch_reset + oed_batch_run"},
        "roofline": {"kernel": "whole batched run (graph)", "bound": "hbm", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "note": "algorithmic downdate bytes / whole-run time (gains, picks and W included in the time)",
                     "syrk_tflops_over_run": round(st["syrk_flops"] / (run_ms * 1e-3) / 1e12, 3)},
        "graph_run_ms": round(run_ms, 3),
        **checks,
    }
    if not args.left and not args.no_left:
        # the same designs left-looking (only each pick's block column formed), beside it
        bl = BatchSelector(items, precision=args.precision or "mixed_f32", profile=True, method="left")
        bl.reset(items)
        bl.run()
        tl = []
        torch.cuda.synchronize()
        for s_ in range(args.steps):
            t1 = time.perf_counter()
            bl.reset(items)
            bl.run()
            torch.cuda.synchronize()
            tl.append(time.perf_counter() - t1)
        bl.close()
        msl = 1e3 * sum(tl) / len(tl)
        result["left_looking"] = {"value": round(total_steps / (msl * 1e-3), 3), "unit": "greedy steps/s",
                                  "ms_per_step": round(msl, 3), "step": "oed_batch_reset + oed_batch_run"}
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the selection is a single-GPU kernel pipeline; "
              "see the sharding paragraph of the design notes", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from oed_inputs import CONFIGS, make_K_lower_panels
    from paper_2604_08812_amd import Selector, library

    if args.copy_calibration:
        return copy_calibration()
    if args.peaks:
        return measured_peaks()
    library()
    if args.config == "batched_48":
        return run_batched(args)
    if args.config == "paper_600x420":
        return run_paper_shape(args)
    spec = CONFIGS[args.config]
    budget = args.budget or spec.budget
    prec = args.precision or spec.precision
    dev = torch.device("cuda:0")
    log(f"forming K for {spec.name}: N_s={spec.N_s} N_t={spec.N_t} n_m={spec.n_m} seed={spec.seed}")
    t0 = time.perf_counter()
    kdt = torch.float64 if spec.k_dtype == "f64" else torch.float32
    K, s2 = make_K_lower_panels(spec.N_s, spec.N_t, spec.n_m, spec.seed, spec.c, device=dev, dtype=kdt,
                                progress=lambda i, n: log(f"  K column chunk {i}/{n}") if i % 4 == 0 or i == n
                                else None)
    torch.cuda.synchronize()
    log(f"K formed in {time.perf_counter() - t0:.1f} s, sigma2={s2:.6e}")

    # ---- headline path
    tune = args.delay == 0 and not args.no_autotune
    tiles_kw = {"tile_order": args.tile_order}
    bf16_kw = {**tiles_kw, "tile_size": args.tile_size}
    sel = Selector(K, spec.N_s, spec.N_t, s2, precision=prec, profile=True, delay=args.delay, autotune=tune,
                   **(bf16_kw if prec == "mixed_bf16x3" else tiles_kw))
    delay, variant, tuned, tiles = sel.config()
    for w in range(args.warmup):
        timed_selections(sel, K, budget, 1)
        log(f"warmup {w + 1}/{args.warmup} done")
    sel.profile(reset=True)
    ms, (idx, gain) = timed_selections(sel, K, budget, args.steps)
    prof = sel.profile(reset=True)
    log(f"{prec}: {ms:.1f} ms per selection of {budget}")
    result = {
        "metric": "greedy steps/s + SYRK TFLOP/s (% MFMA peak), mixed vs FP64, same picks",
        "value": round(budget / (ms * 1e-3), 3),
        "unit": "greedy steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": spec.name, "N_s": spec.N_s, "N_t": spec.N_t, "n_m": spec.n_m, "seed": spec.seed,
                   "budget": budget, "precision": prec, "K_dtype": spec.k_dtype, "delay": delay,
                   "downdate_variant": ["direct", "lds", "lds256"][variant], "tile_order": tiles, "autotuned": tune,
                   "autotuner_ms_per_pick_by_delay": [round(float(x), 4) for x in tuned] if tune else None,
                   "step": "oed_reset + oed_greedy(budget)"},
        "roofline": roofline_syrk(prof, prec, spec.name, delay, variant),
        "kernel_ms_per_step": {k: round(v / args.steps, 3) for k, v in prof["ms"].items()},
        "paper_context": PAPER_CONTEXT,
    }
    sel.close()

    # ---- FP64 beside it, same K
    if not args.no_fp64 and prec != "fp64":
        sel64 = Selector(K, spec.N_s, spec.N_t, s2, precision="fp64", profile=True, delay=args.delay, autotune=tune,
                         **tiles_kw)
        sel64.profile(reset=True)
        ms64, (idx64, gain64) = timed_selections(sel64, K, budget, args.fp64_steps)
        p64 = sel64.profile(reset=True)
        d64, v64, _, o64 = sel64.config()
        if not args.no_gaps:
            gaps = top_two_gaps(sel64, K, budget)
        sel64.close()
        log(f"fp64: {ms64:.1f} ms per selection")
        result["fp64"] = {"value": round(budget / (ms64 * 1e-3), 3), "unit": "greedy steps/s",
                          "delay": d64, "tile_order": o64,
                          "ms_per_step": round(ms64, 3), "roofline": roofline_syrk(p64, "fp64", spec.name, d64, v64),
                          "kernel_ms_per_step": {k: round(v / args.fp64_steps, 3) for k, v in p64["ms"].items()}}
        result["mixed_vs_fp64"] = {"speedup": round(ms64 / ms, 3), **compare_picks(idx, gain, idx64, gain64)}
        if not args.no_gaps:
            per = gaps.pop("per_step")
            result["fp64"]["top_two_gap"] = gaps
            fd = result["mixed_vs_fp64"]["first_divergence_step"]
            if fd is not None and fd < len(per):
                result["mixed_vs_fp64"]["fp64_top_two_gap_at_divergence"] = per[fd]

    # ---- the BF16 split-product downdate beside it, same K
    if not args.no_bf16x3 and prec == "mixed_f32" and spec.N_t <= 128 and not args.precision:
        selb = Selector(K, spec.N_s, spec.N_t, s2, precision="mixed_bf16x3", profile=True, delay=args.delay,
                        autotune=tune, **bf16_kw)
        timed_selections(selb, K, budget, 1)
        selb.profile(reset=True)
        msb, (idxb, gainb) = timed_selections(selb, K, budget, args.steps)
        pb = selb.profile(reset=True)
        db, vb, _, ob = selb.config()
        selb.close()
        log(f"mixed_bf16x3: {msb:.1f} ms per selection")
        result["mixed_bf16x3"] = {"value": round(budget / (msb * 1e-3), 3), "unit": "greedy steps/s", "delay": db,
                                  "downdate_variant": ["direct", "lds", "lds256"][vb], "tile_order": ob,
                                  "ms_per_step": round(msb, 3),
                                  "roofline": roofline_syrk(pb, "mixed_bf16x3", spec.name, db, vb),
                                  "kernel_ms_per_step": {k: round(v / args.steps, 3) for k, v in pb["ms"].items()},
                                  "speedup_vs_mixed_f32": round(ms / msb, 3),
                                  "vs_mixed_f32": compare_picks(idxb, gainb, idx, gain)}
        if "fp64" in result:
            result["mixed_bf16x3"]["vs_fp64"] = compare_picks(idxb, gainb, idx64, gain64)
            fd = result["mixed_bf16x3"]["vs_fp64"]["first_divergence_step"]
            if fd is not None and not args.no_gaps and fd < len(per):
                result["mixed_bf16x3"]["vs_fp64"]["fp64_top_two_gap_at_divergence"] = per[fd]

    # ---- left-looking (the order of Algorithm 1) beside it, same K
    if not args.no_left and spec.N_t <= 128:
        for lp in ("mixed_f32", "mixed_bf16x3", "fp64"):
            if lp != prec and lp != "fp64" and not (lp == "mixed_bf16x3" and prec == "mixed_f32"):
                continue
            sell = Selector(K, spec.N_s, spec.N_t, s2, precision=lp, profile=True, method="left", max_budget=budget)
            timed_selections(sell, K, budget, 1)
            sell.profile(reset=True)
            nst = args.steps if lp == prec else args.fp64_steps
            msl, (idxl, gainl) = timed_selections(sell, K, budget, nst)
            pl = sell.profile(reset=True)
            sell.close()
            log(f"left-looking {lp}: {msl:.1f} ms per selection")
            tfl = pl["syrk_flops"] / (pl["ms"]["syrk"] * 1e-3) / 1e12 if pl["ms"]["syrk"] > 0 else 0.0
            leg = {"value": round(budget / (msl * 1e-3), 3), "unit": "greedy steps/s", "ms_per_step": round(msl, 3),
                   "column_kernel": {"kernel": {"mixed_f32": "column_kernel<float>", "fp64": "column_kernel<double>",
                                                "mixed_bf16x3": "column_bf16_kernel"}[lp],
                                     "algorithmic_tflops": round(tfl, 3), "peak": PEAK_TFLOPS[lp],
                                     # the BF16 split product executes three MFMA products per one
                                     "frac": round(tfl * (3 if lp == "mixed_bf16x3" else 1) / PEAK_TFLOPS[lp], 4),
                                     "algorithmic_flops_per_selection": pl["syrk_flops"] / nst},
                   "kernel_ms_per_step": {k: round(v / nst, 3) for k, v in pl["ms"].items()}}
            ref = (idx64, gain64) if "fp64" in result else (idx, gain)
            leg["vs_fp64_right_looking" if "fp64" in result else "vs_headline"] = compare_picks(idxl, gainl, *ref)
            result["left_looking_" + lp] = leg

    # ---- design evaluation: the greedy design against random and uniformly spaced ones
    if not args.no_eval and spec.N_t <= 128 and args.eval_designs >= 3:
        result["design_evaluation"] = design_evaluation(K, spec, s2, prec, budget, idx, gain, args.eval_designs)

    # ---- CPU oracle baseline on a bounded sample of the same K
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(K, spec.N_t, s2, args.cpu_sensors, args.cpu_budget, full_shape=(spec.N_s, budget))
        sel_s = Selector(K, spec.N_s, spec.N_t, s2, precision=prec, candidates=range(args.cpu_sensors))
        i_s, g_s = sel_s.greedy(args.cpu_budget)
        sel_s.close()
        cb["gpu_same_sample_picks_equal"] = [int(x) for x in i_s] == cb["idx"]
        cb["gpu_same_sample_max_rel_gain_err"] = float(np.max(np.abs(g_s - np.array(cb["gain"])) /
                                                             np.maximum(1, np.abs(np.array(cb["gain"])))))
        del cb["idx"], cb["gain"]
        result["cpu_baseline"] = cb
        log(f"cpu baseline {cb['value']} steps/s on {cb['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
