#!/usr/bin/env python3
"""Benchmark of the dedispersion + single-pulse-search hot path on one MI355X.

One step = the whole path over one synthetic beam already resident in HBM:
staging/downsampling, brute-force dedispersion of every plan row, per-trial
statistics, boxcar search with run extraction, fragment joining and
friends-of-friends grouping of the candidates.

Default workload (realistic band): 4096 channels over 1000-1500 MHz, tsamp
49.152 us, 2^20 uint8 samples (51.5 s), DDplan ladder 0-3000 pc cm^-3 with
steps 0.1/0.3/1/3 and downsampling 1/2/4/8 (3850 trials), boxcar widths
1..512, 6 sigma, 20 injected pulses.

Prints ONE JSON line on stdout.  Metric: DM-trial x samples per second
(sum over rows of n_dm * n_out at each row's own resolution, per second);
the real-time factor (data seconds per wall second) rides along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DM-trial×samples/s & real-time factor (4096 ch); batched+CNN vs plain"
PEAK_INT32_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: int32 VALU ops/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2110_12749_amd import synth
    return {"realistic": synth.realistic, "wideband": synth.wideband, "tiny": synth.tiny}[name]()


def describe(w, desc):
    return {
        "workload": f"{w.name}: 1 beam, {w.nchan} ch over {w.f_lo:g}-{w.f_hi:g} MHz, tsamp {w.tsamp * 1e6:g} us, "
                    f"{w.nsamp} uint8 samples, {w.n_trials} DM trials in {len(w.segments)} DDplan rows "
                    f"(D {'/'.join(str(s[3]) for s in w.segments)}), widths {w.widths[0]}..{w.widths[-1]}, "
                    f"{w.threshold:g} sigma, {len(w.pulses)} injected pulses",
        "nchan": w.nchan, "nsamp": w.nsamp, "n_trials": w.n_trials,
        "rows": [list(s) for s in w.segments],
        "dm_trial_samples": int(sum(desc.seg[s].n_dm * desc.n_out[s] for s in range(desc.n_seg))),
    }


def cpu_baseline(w, X, desc, every: int):
    """The oracle as it stands, on a deterministic sample of the trials
    (every `every`-th trial of each row, full time range, dedispersion and
    search), extrapolated row by row to the whole plan."""
    import oracle
    t_full = 0.0
    sampled = 0
    t_all = 0.0
    for s, seg in enumerate(w.segments):
        idx = list(range(0, seg[2], every))
        t0 = time.perf_counter()
        for i in idx:
            row = oracle.dedisperse_segment(X, w.freqs, w.tsamp, seg, trials=(i, i + 1))
            oracle.search_series(row[0], w.widths, w.threshold, trial=i)
        dt = time.perf_counter() - t0
        t_all += dt
        sampled += len(idx)
        t_full += dt * seg[2] / len(idx)
        log(f"  cpu row {s}: {len(idx)} trials in {dt:.2f} s")
    total = sum(desc.seg[s].n_dm * desc.n_out[s] for s in range(desc.n_seg))
    return {"value": total / t_full, "unit": "DM-trial×samples/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"every {every}th trial of each DDplan row ({sampled} of {w.n_trials} trials, full length), "
                      f"dedispersion + boxcar search, {t_all:.1f} s measured, extrapolated per row to the full plan",
            "rtf": (w.nsamp * w.tsamp) / t_full}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="realistic", choices=["realistic", "wideband", "tiny"])
    ap.add_argument("--cpu-every", type=int, default=96, help="oracle sample: every n-th trial per row")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path (beams or DM ranges would shard "
            "across GPUs with no exchange step; see DESIGN.md).  Run with --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_12749_amd import gsp

    w = workload(args.workload)
    log(f"generating {w.name}: {w.nsamp} x {w.nchan}")
    t0 = time.perf_counter()
    X = w.generate()
    log(f"  {time.perf_counter() - t0:.1f} s")
    fb = torch.from_numpy(X).to("cuda:0")
    ctx = gsp.Context(0)
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    dmt = torch.empty(desc.total, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step():
        ctx.dedisperse(fb, w.freqs, desc, out=dmt, stream=stream)
        c = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold, stream=stream)
        rep, ng = gsp.group_candidates(c)
        return c, ng

    for k in range(args.warmup):
        t = time.perf_counter()
        c, ng = step()
        torch.cuda.synchronize()
        log(f"warmup {k}: {time.perf_counter() - t:.3f} s, {len(c)} candidates, {ng} events")
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        c, ng = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    ms = wall / args.steps * 1e3
    cfg = describe(w, desc)
    value = cfg["dm_trial_samples"] / (ms / 1e3)
    rtf = (w.nsamp * w.tsamp) / (ms / 1e3)
    n, tot_ms, adds = prof["dedisperse"]
    achieved = adds / (tot_ms / 1e3)
    kernels = {k: {"launches_per_step": v[0] / args.steps, "ms_per_step": v[1] / args.steps,
                   "avg_launch_ms": v[1] / v[0],
                   ("adds_per_s" if k == "dedisperse" else "bytes_per_s"): v[2] / (v[1] / 1e3)}
               for k, v in prof.items()}
    out = {
        "metric": METRIC, "value": value, "unit": "DM-trial×samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8->int32", "data": "synthetic", "config": cfg,
        "rtf": rtf,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32_OPS / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_INT32_OPS, "traffic": None,
                     "kernel": "k_dedisp", "work": "integer adds (n_dm * n_out * nchan per launch)"},
        "kernels": kernels,
        "candidates": int(len(c)), "events": int(ng),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, X, desc, args.cpu_every)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
