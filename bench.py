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
# Sample additions per 32-bit VALU lane operation: the 16-bit tile adds two
# 16-bit sample sums per packed add; the byte-quad tile adds four bytes per
# v_sad_u8.  Their ALU ceilings in sample additions:
PEAK_SAMPLE_ADDS = {"dedisperse": 2 * PEAK_INT32_OPS, "dedisperse_quad": 4 * PEAK_INT32_OPS}
# LDS bytes the kernels read per sample addition (a dword holds two 16-bit
# samples, or four channels' bytes)
LDS_BYTES_PER_ADD = {"dedisperse": 2.0, "dedisperse_quad": 1.0}
KERNEL_NAME = {"dedisperse": "k_dedisp", "dedisperse_quad": "k_dedisp_quad"}
QUAD_KERNEL_BY_KIND = {1: "k_dedisp_quad", 2: "k_dedisp_quad_pc", 3: "k_dedisp_quad_pc"}  # byte-quad kernels by shape kind
# LDS read rates measured on the MI355X for the kernels' access pattern, B/clk/CU
LDS_READ2ST64 = 110.2  # ds_read2st64_b32, offsets from registers (the kernels' form)
LDS_B128 = 176.7       # ds_read_b128 at 16-byte aligned addresses


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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dedisp_realistic_traffic.md")
# the device code of each dedispersion tile, by its profile key
KERNEL_SOURCES = {"k_dedisp_quad": [os.path.join(ROOT, "paper_2110_12749_amd", "csrc", "dedisp_quad.hip")],
                  "k_dedisp": [os.path.join(ROOT, "paper_2110_12749_amd", "csrc", "dedisp_tile.h")]}


def kernel_source_hash(key: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[key]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name: str, key: str):
    """HBM bytes per launch of a dedispersion tile (key "k_dedisp_quad" or
    "k_dedisp") from the committed rocprofv3 counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy kernel), or None when there is none for
    this workload or the kernel's source changed since."""
    if workload_name != "realistic" or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", "|", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get(key + ".source_sha256") != kernel_source_hash(key):
        return None
    try:
        return float(kv[key + ".fetch_bytes_per_launch"]) + float(kv[key + ".write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    cores = oracle.num_threads()
    # one core: the first trial of each row, extrapolated the same way
    oracle.set_threads(1)
    t1_full, t1_all = 0.0, 0.0
    for s, seg in enumerate(w.segments):
        t0 = time.perf_counter()
        row = oracle.dedisperse_segment(X, w.freqs, w.tsamp, seg, trials=(0, 1))
        oracle.search_series(row[0], w.widths, w.threshold, trial=0)
        dt = time.perf_counter() - t0
        t1_all += dt
        t1_full += dt * seg[2]
        log(f"  cpu row {s} on one core: 1 trial in {dt:.2f} s")
    oracle.set_threads(cores)
    return {"value": total / t_full, "unit": "DM-trial×samples/s", "cores": cores,
            "kind": "oracle",
            "sample": f"every {every}th trial of each DDplan row ({sampled} of {w.n_trials} trials, full length), "
                      f"dedispersion + boxcar search, {t_all:.1f} s measured, extrapolated per row to the full plan",
            "rtf": (w.nsamp * w.tsamp) / t_full,
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "one_core": {"value": total / t1_full, "rtf": (w.nsamp * w.tsamp) / t1_full,
                         "sample": f"the first trial of each row on one thread ({t1_all:.1f} s measured), "
                                   f"extrapolated per row"}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_stream(paced: bool, pool_blocks: int = 24, max_blocks: int | None = None, triage: str | None = None,
                 triage_thr: float = 0.0):
    """19 beams (4096 ch, tsamp 49.152 us, lengths 2^18..2^20, per-beam ladders
    of 1000-4000 trials) streaming in blocks of 20480 samples (1.00663 s).
    Block contents come from a pool of pre-generated realistic blocks (noise
    and pulses) reused across beams; only the performance is measured here,
    the streaming results are checked against the oracle by the tests.
    paced: block k of every beam is pushed at k x 1.00663 s (+ up to 5 ms
    seeded jitter) and the worker thread processes whatever has arrived;
    otherwise every block is pushed at once (capacity)."""
    import numpy as np
    import torch
    from paper_2110_12749_amd import gsp, synth
    B = 20480
    beams = synth.stream_beams()
    src = synth.realistic()
    log(f"stream: generating {pool_blocks} pool blocks")
    pool = [src.generate(t_begin=k * B, nrows=B) for k in range(pool_blocks)]
    ctx = gsp.Context(0)
    s = gsp.Stream(ctx, 200 << 30, B, synth.WIDTHS_512, 6.0)
    net = None
    if triage:  # network weights (a gsp_cnn_save file, or "random": timing only) scoring each step's candidates
        net = gsp.Cnn(ctx, seed=1)
        if triage != "random":
            net.load(triage)
        s.set_triage(net, triage_thr)
    ids = []
    for w in beams:
        bid, ok = s.open_beam(w.nchan, w.freqs, w.tsamp, w.segments)
        ids.append(bid)
    nblk = [(w.nsamp + B - 1) // B for w in beams]
    if max_blocks:
        nblk = [min(n, max_blocks) for n in nblk]
    rng = np.random.default_rng(2110127494)
    work = 0  # DM-trial x samples produced
    for w, n in zip(beams, nblk):
        desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
        for r in range(desc.n_seg):
            D = w.segments[r][3]
            outs = max(0, min(n * B, w.nsamp) // D - desc.max_delay[r])
            work += w.segments[r][2] * outs
    # warm-up: the graph capture and first launches on a throw-away beam
    wb, _ = s.open_beam(beams[0].nchan, beams[0].freqs, beams[0].tsamp, beams[0].segments)
    s.push(wb, pool[0])
    s.step()
    s.close_beam(wb)
    s.poll()
    s.start()
    period = B * 49.152e-6
    t0 = time.perf_counter()
    for k in range(max(nblk)):
        if paced:
            target = t0 + k * period
            while time.perf_counter() < target:
                time.sleep(0.0005)
        for j, (w, bid) in enumerate(zip(beams, ids)):
            if k < nblk[j]:
                if paced:
                    time.sleep(float(rng.uniform(0, 0.005)) / len(beams))
                blk = pool[(7 * j + k) % pool_blocks]
                n = min(B, w.nsamp - k * B)
                s.push(bid, blk[:n] if n < B else blk)
    s.flush()
    wall = time.perf_counter() - t0
    s.stop()
    rep = s.report()
    c = s.poll()
    s.close()
    if net is not None:
        net.close()
    ctx.close()
    data_s = sum(min(n * B, w.nsamp) for w, n in zip(beams, nblk)) * 49.152e-6
    return {"mode": "paced (real-time arrivals)" if paced else "unpaced (all blocks at once)",
            "beams": len(beams), "blocks": int(rep["blocks"]), "steps": int(rep["steps"]),
            "wall_s": wall, "busy_s": rep["busy_s"], "dm_trial_samples": int(work),
            "dm_trial_samples_per_s": work / wall, "rtf_aggregate": data_s / wall,
            "lat_p50_s": rep["lat_p50_s"], "lat_p99_s": rep["lat_p99_s"], "lat_max_s": rep["lat_max_s"],
            "block_s": period, "candidates": int(len(c)),
            "triage": None if net is None else {
                "threshold": triage_thr, "scored": int(rep["triage_scored"]), "rejected": int(rep["triage_rejected"]),
                "ms_per_block": rep["triage_s"] / max(1, rep["blocks"]) * 1e3}}


# bands per row by downsampling (16-bit sub-band series: 255 * D * channels per
# band <= 65535) and trials per group; chosen by a sweep on the realistic
# workload (step time against the injected pulses' SNR relative to brute force)
SUBBAND_NSUB = {1: 32, 2: 32, 4: 64, 8: 128}
SUBBAND_GROUP = 32  # at most this many trials per group


def subband_groups(segments, gmax=SUBBAND_GROUP, tile=32):
    """Per row, the smallest group size that needs no more stage-1 tiles of
    `tile` groups than groups of gmax would (so no tile is padded more than
    needed): e.g. 1500 trials -> 24 (63 groups in 2 tiles), 600 -> 19."""
    out = []
    for s in segments:
        n_dm = s[2]
        tiles = -(-n_dm // (tile * gmax))
        out.append(-(-n_dm // (tile * tiles)))
    return out


def bench_subband(ctx, w, fb, stream, steps):
    """The step with sub-band (two-stage) dedispersion instead of brute
    force: staging, both stages, statistics, search, grouping."""
    import torch
    from paper_2110_12749_amd import gsp
    n_sub = [SUBBAND_NSUB.get(s[3], 128) for s in w.segments]
    group = subband_groups(w.segments)
    desc = gsp.subband_plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments, n_sub, group)
    dmt = torch.empty(desc.total, dtype=torch.int32, device="cuda:0")

    def step():
        ctx.dedisperse_subband(fb, w.freqs, desc, n_sub, group, out=dmt, stream=stream)
        c = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold, stream=stream)
        return c, gsp.group_candidates(c)[1]

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    t = time.perf_counter()
    for _ in range(steps):
        c, ng = step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    work = sum(desc.seg[s].n_dm * desc.n_out[s] for s in range(desc.n_seg))
    brute_adds = sum(desc.seg[s].n_dm * desc.n_out[s] * desc.nchan for s in range(desc.n_seg))
    kernels = {k: {"ms_per_step": v[1] / steps, "avg_launch_ms": v[1] / v[0],
                   "adds_per_s" if k.startswith("subband") else "bytes_per_s": v[2] / (v[1] / 1e3)}
               for k, v in prof.items()}
    ded_s = sum(prof[k][1] for k in ("subband1", "subband2", "stage") if k in prof) / steps / 1e3
    del dmt
    return {"n_sub": n_sub, "group": group, "ms_per_step": wall * 1e3, "value": work / wall,
            "rtf": (w.nsamp * w.tsamp) / wall, "candidates": int(len(c)), "events": int(ng),
            "dedispersion_ms": ded_s * 1e3,
            "brute_force_equivalent_adds_per_s": brute_adds / ded_s,
            "kernels": kernels,
            "what": "sub-band dedispersion (stage 1: nchan/group adds per output, stage 2: n_sub) + statistics + "
                    "search + grouping; an approximation of brute force judged by the injected pulses' SNR in "
                    "the tests"}


SWEEP_SHAPES = [(4, 4, 8, 32), (4, 4, 8, 16), (4, 4, 8, 8), (4, 4, 4, 32), (4, 8, 4, 32), (2, 8, 8, 32),
                (8, 4, 8, 32),
                # byte-quad tile (D = 1 rows with whole channel quads)
                (8, 4, 8, 64, 1), (8, 4, 16, 64, 1), (8, 2, 16, 64, 1), (4, 8, 8, 64, 1), (16, 2, 16, 64, 1),
                (4, 4, 16, 64, 1), (4, 8, 16, 64, 1), (4, 8, 4, 64, 1),
                # byte-quad tile with 4 staging waves besides the summing ones
                (4, 8, 12, 64, 2), (4, 8, 8, 64, 2), (4, 8, 10, 64, 2), (8, 4, 8, 64, 2), (8, 4, 12, 64, 2),
                (4, 8, 4, 64, 2),
                # split rows: kind 2 over the channels whose copies fit, the 16-bit tile over the rest
                (4, 8, 8, 64, 3), (4, 8, 12, 64, 3), (8, 4, 8, 64, 3),
                (8, 4, 4, 64, 2)]


def shape_sweep(w):
    """Each row of the plan alone, dedispersed with each shape (groups, trials
    per wave, waves, channels per chunk; the library clamps the chunk to what
    its staging registers and LDS hold): kernel time from the library's
    event timing, mean of 2 launches after one untimed launch."""
    import torch
    from paper_2110_12749_amd import gsp
    X = w.generate()
    fb = torch.from_numpy(X).to("cuda:0")
    del X
    ctx = gsp.Context(0)
    print(f"| row | D | n_dm | requested (groups, tpw, waves, chunk[, kind]) | used | ms | T adds/s |")
    print("|---|---|---|---|---|---|---|")
    for s, seg in enumerate(w.segments):
        d1 = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, [seg])
        out = torch.empty(d1.total, dtype=torch.int32, device="cuda:0")
        adds = seg[2] * d1.n_out[0] * w.nchan
        for c in SWEEP_SHAPES:
            try:
                ctx.set_row_shape(w.freqs, d1, 0, *c)
            except gsp.GspError as e:
                print(f"| {s} | {seg[3]} | {seg[2]} | {c} | rejected: {e} | | |", flush=True)
                continue
            ctx.dedisperse(fb, w.freqs, d1, out=out)
            ctx.profile_enable(True)
            ctx.profile_read()
            for _ in range(2):
                ctx.dedisperse(fb, w.freqs, d1, out=out)
            p = ctx.profile_read()
            ctx.profile_enable(False)
            ms = sum(p[k][1] for k in ("dedisperse", "dedisperse_quad") if k in p) / 2
            used = tuple(ctx.row_shape(w.freqs, d1, 0))
            print(f"| {s} | {seg[3]} | {seg[2]} | {c} | {used} | {ms:.2f} | {adds / ms / 1e9:.2f} |", flush=True)
        del out
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="realistic", choices=["realistic", "wideband", "tiny"])
    ap.add_argument("--cpu-every", type=int, default=96, help="oracle sample: every n-th trial per row")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cnn", action="store_true", help="plain search only (no cutouts + network triage)")
    ap.add_argument("--stream", choices=["paced", "unpaced"], default=None,
                    help="run the 19-beam streaming workload instead (prints its own JSON line)")
    ap.add_argument("--stream-max-blocks", type=int, default=None)
    ap.add_argument("--triage-weights", default=None, help="stream: attach a trained network (gsp_cnn_save file)")
    ap.add_argument("--triage-threshold", type=float, default=0.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shapes (otherwise the autotuner picks one per row before the warm-up)")
    ap.add_argument("--shapes", action="store_true",
                    help="time a fixed set of dedispersion tile shapes on every row of the workload (markdown table)")
    ap.add_argument("--rows", default=None,
                    help="comma-separated plan rows to keep (e.g. 0 for the D = 1 row alone; profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy kernel (reference for hardware byte counters)")
    ap.add_argument("--e2e-steps", type=int, default=2, help="steps timed with the host-to-device copy included")
    ap.add_argument("--rfi", action="store_true",
                    help="clip outlying zero-DM spectra (blocks of 2048) and apply the zero-DM filter inside the step")
    ap.add_argument("--clip-sigma", type=float, default=6.0)
    ap.add_argument("--no-subband", dest="subband", action="store_false",
                    help="skip the sub-band dedispersion measurement")
    ap.add_argument("--no-stream", dest="stream_in_line", action="store_false",
                    help="skip the paced 19-beam streaming run reported under 'stream'")
    ap.add_argument("--stream-line-blocks", type=int, default=12,
                    help="blocks per beam of the streaming run in the default line (19 beams)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU only: the library has no multi-GPU path (beams or DM ranges would shard "
            "across GPUs with no exchange step).  Run with --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_12749_amd import gsp

    if args.stream:
        r = bench_stream(args.stream == "paced", max_blocks=args.stream_max_blocks, triage=args.triage_weights,
                         triage_thr=args.triage_threshold)
        print(json.dumps({"metric": METRIC, "value": r["dm_trial_samples_per_s"], "unit": "DM-trial×samples/s",
                          "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "u8->int32", "data": "synthetic", "config": {"workload": "stream: 19 beams, "
                          "4096 ch over 1000-1500 MHz, tsamp 49.152 us, 20480-sample blocks, lengths 2^18..2^20, "
                          "1000-4000 trials per beam"}, "stream": r}), flush=True)
        return

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.mul(src, 1, out=dst)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    w = workload(args.workload)
    if args.rows is not None:
        keep = [int(r) for r in args.rows.split(",")]
        w.segments = [w.segments[r] for r in keep]
    if args.shapes:
        shape_sweep(w)
        return
    log(f"generating {w.name}: {w.nsamp} x {w.nchan}")
    t0 = time.perf_counter()
    X = w.generate()
    log(f"  {time.perf_counter() - t0:.1f} s")
    fb = torch.from_numpy(X).to("cuda:0")
    ctx = gsp.Context(0)
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    dmt = torch.empty(desc.total, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    shapes = None
    if not args.no_autotune:  # once per plan, untimed: each row gets its fastest bit-exact shape
        t = time.perf_counter()
        shapes = ctx.autotune(fb, w.freqs, desc, out=dmt, stream=stream)
        torch.cuda.synchronize()
        log(f"autotune: {shapes} in {time.perf_counter() - t:.1f} s")

    net = None if args.no_cnn else gsp.Cnn(ctx, seed=1)
    # room for 16384 events per network call (an event-richer step is cut out
    # and scored in chunks of that many)
    cut = torch.empty((16384, 2, 64, 64), dtype=torch.int16, device="cuda:0")
    logits = torch.empty(16384, dtype=torch.float32, device="cuda:0")
    t_triage = [0.0]

    raw = None
    if args.rfi:  # RFI mitigation inside the step: the raw input stays untouched, the cleaned copy is searched
        raw = fb
        fb = torch.empty_like(raw)

    def step(src=None):
        # src: the device copy of the input this step reads (default: fb, or
        # raw with RFI mitigation, which cleans it into fb)
        fin = fb
        if raw is not None:
            ctx.rfi_clean(raw if src is None else src, args.clip_sigma, 2048, zero_dm=True, out=fb, count=False,
                          stream=stream)
        elif src is not None:
            fin = src
        ctx.dedisperse(fin, w.freqs, desc, out=dmt, stream=stream)
        c = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold, stream=stream)
        rep, ng = gsp.group_candidates(c)
        if net is not None and ng:
            # triage: cutouts of each event's representative, network scores
            t = time.perf_counter()
            ev = c[np.unique(rep)]  # one candidate per event: its max-SNR member
            keep = 0
            for e0 in range(0, len(ev), cut.shape[0]):
                part = ev[e0:e0 + cut.shape[0]]
                x = gsp.cutouts(ctx, fin, w.freqs, dmt, desc, part, out=cut[:len(part)], stream=stream)
                net.forward(x, out=logits[:len(part)], stream=stream)
                keep += int((logits[:len(part)] > 0).sum().item())
            assert len(ev) == ng
            t_triage[0] += time.perf_counter() - t
        return c, ng

    for k in range(args.warmup):
        t = time.perf_counter()
        c, ng = step()
        torch.cuda.synchronize()
        log(f"warmup {k}: {time.perf_counter() - t:.3f} s, {len(c)} candidates, {ng} events")
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t_triage[0] = 0.0
    t = time.perf_counter()
    for _ in range(args.steps):
        c, ng = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    ms = wall / args.steps * 1e3
    cfg = describe(w, desc)
    cfg["tile_shapes"] = [list(ctx.row_shape(w.freqs, desc, r)) for r in range(desc.n_seg)]
    cfg["rfi_mitigation"] = (f"clip {args.clip_sigma:g} sigma in blocks of 2048 spectra + zero-DM filter" if args.rfi
                             else None)
    cfg["autotuned"] = shapes is not None
    value = cfg["dm_trial_samples"] / (ms / 1e3)
    rtf = (w.nsamp * w.tsamp) / (ms / 1e3)
    # the dominant kernel: the dedispersion tile with the most time per step
    dom = max((k for k in PEAK_SAMPLE_ADDS if k in prof), key=lambda k: prof[k][1])
    n, tot_ms, adds = prof[dom]
    achieved = adds / (tot_ms / 1e3)
    peak = PEAK_SAMPLE_ADDS[dom]
    lds_b = LDS_BYTES_PER_ADD[dom]
    kernels = {k: {"launches_per_step": v[0] / args.steps, "ms_per_step": v[1] / args.steps,
                   "avg_launch_ms": v[1] / v[0],
                   ("adds_per_s" if k.startswith("dedisperse") else "bytes_per_s"): v[2] / (v[1] / 1e3)}
               for k, v in prof.items()}
    kname = KERNEL_NAME[dom]
    if dom == "dedisperse_quad":  # the byte-quad kernel of the rows' shapes (the D = 1 rows share one)
        kinds = {sh[4] for sh in cfg["tile_shapes"] if sh[4] != 0}
        kname = "/".join(QUAD_KERNEL_BY_KIND[k] for k in sorted(kinds))
    all_adds = sum(prof[k][2] for k in PEAK_SAMPLE_ADDS if k in prof)
    all_ms = sum(prof[k][1] for k in PEAK_SAMPLE_ADDS if k in prof)
    out = {
        "metric": METRIC, "value": value, "unit": "DM-trial×samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8->int32", "data": "synthetic", "config": cfg,
        "rtf": rtf,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(w.name, "k_dedisp_quad" if dom == "dedisperse_quad" else "k_dedisp"),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": kname, "launches_per_step": n / args.steps,
                     "work": "integer sample additions (n_dm * n_out * nchan per launch)",
                     "peak_note": ("four 8-bit sample additions per v_sad_u8 lane operation: 4 x 256 CUs x 64 "
                                   "lanes x 2.4 GHz" if dom == "dedisperse_quad" else
                                   "two 16-bit sample additions per packed 32-bit VALU add: 2 x 256 CUs x 64 "
                                   "lanes x 2.4 GHz") +
                                  "; the kernel is bound by its LDS reads (see 'lds') and the VALU work of "
                                  "staging them",
                     "all_dedispersion": {"adds_per_s": all_adds / (all_ms / 1e3), "ms_per_step": all_ms / args.steps,
                                          "what": "every dedispersion launch of the step (both tiles)"},
                     "int32_reference": {"peak": PEAK_INT32_OPS / 1e12, "frac": achieved / PEAK_INT32_OPS,
                                         "all_dedispersion_frac": all_adds / (all_ms / 1e3) / PEAK_INT32_OPS,
                                         "what": "against one 32-bit add per VALU lane and clock (256 CUs x 64 "
                                                 "lanes x 2.4 GHz), the rate of a tile that adds one sample per "
                                                 "lane operation; above 1 where samples are packed"}},
        "lds": {"what": f"LDS read bandwidth of {kname}: {lds_b:g} byte(s) of staged samples per "
                        "sample addition, read as ds_read2st64_b32",
                "achieved_TBps": lds_b * achieved / 1e12,
                "peak_form_TBps": LDS_READ2ST64 * 256 * 2.4e9 / 1e12,
                "frac_form": lds_b * achieved / (LDS_READ2ST64 * 256 * 2.4e9),
                "peak_b128_TBps": LDS_B128 * 256 * 2.4e9 / 1e12,
                "frac_b128": lds_b * achieved / (LDS_B128 * 256 * 2.4e9),
                "note": "measured on MI355X: ds_read2st64_b32 with register offsets 110.2 B/clk/CU, "
                        "ds_read_b128 (16-byte aligned) 176.7 B/clk/CU"},
        "kernels": kernels,
        "candidates": int(len(c)), "events": int(ng),
        "triage": None if net is None else {
            "ms_per_step": t_triage[0] / args.steps * 1e3,
            "what": "cutouts of each event's max-SNR candidate + CNN forward (490,897 parameters, random "
                    "initialisation: timing only) + logits to host",
            "plain_ms_per_step": ms - t_triage[0] / args.steps * 1e3},
    }
    out["native_dm_trial_samples_per_s"] = sum(desc.seg[r].n_dm * desc.n_out[r] * desc.seg[r].downsamp
                                               for r in range(desc.n_seg)) / (ms / 1e3)
    # end to end: the same step with the input copied from pinned host memory
    # first (PCIe) and the candidates brought back (as every step does)
    if args.e2e_steps > 0:
        Xp = torch.from_numpy(X).pin_memory()
        dst = raw if raw is not None else fb  # where the input lands
        dst.copy_(Xp, non_blocking=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.e2e_steps):
            dst.copy_(Xp, non_blocking=True)
        torch.cuda.synchronize()
        h2d = (time.perf_counter() - t) / args.e2e_steps
        t = time.perf_counter()
        for _ in range(args.e2e_steps):
            dst.copy_(Xp, non_blocking=True)
            step()
        torch.cuda.synchronize()
        e2e = (time.perf_counter() - t) / args.e2e_steps
        # pipelined: the next input is copied on a second stream (default
        # priority) into the other of two device buffers while the current
        # step runs; a step waits for its copy, a copy for the step that last
        # read its buffer
        bufs = [dst, torch.empty_like(dst)]
        cs = torch.cuda.Stream()
        ready = [torch.cuda.Event(), torch.cuda.Event()]
        free = [torch.cuda.Event(), torch.cuda.Event()]
        for e in free:
            e.record(stream)

        def enqueue_copy(k):
            b = k % 2
            cs.wait_event(free[b])
            with torch.cuda.stream(cs):
                bufs[b].copy_(Xp, non_blocking=True)
            ready[b].record(cs)

        n_pipe = max(args.e2e_steps, 6)
        torch.cuda.synchronize()
        t = time.perf_counter()
        enqueue_copy(0)
        for k in range(n_pipe):
            if k + 1 < n_pipe:
                enqueue_copy(k + 1)
            stream.wait_event(ready[k % 2])
            step(bufs[k % 2])
            free[k % 2].record(stream)
        torch.cuda.synchronize()
        pipe = (time.perf_counter() - t) / n_pipe
        del Xp, bufs
        out["end_to_end"] = {"ms_per_step": e2e * 1e3, "value": cfg["dm_trial_samples"] / e2e,
                             "rtf": (w.nsamp * w.tsamp) / e2e, "h2d_ms": h2d * 1e3,
                             "h2d_GBps": w.nsamp * w.nchan / h2d / 1e9, "steps": args.e2e_steps,
                             "what": "host-to-device copy of the uint8 input from pinned memory + the step "
                                     "(candidates to the host included)",
                             "pipelined": {"ms_per_step": pipe * 1e3, "value": cfg["dm_trial_samples"] / pipe,
                                           "rtf": (w.nsamp * w.tsamp) / pipe, "steps": n_pipe,
                                           "what": "the same, with each step's input copied on a second stream "
                                                   "while the previous step runs (two device input buffers)"}}
    if args.subband:
        out["subband"] = bench_subband(ctx, w, fb, stream, args.steps)
    del dmt
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, X, desc, args.cpu_every)
    ctx.close()
    del fb
    raw = None
    torch.cuda.empty_cache()
    if args.stream_in_line:
        log("stream: 19 beams, paced, network attached (random weights: timing only) ...")
        out["stream"] = bench_stream(True, max_blocks=args.stream_line_blocks, triage="random")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
