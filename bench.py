"""Benchmark of the reliability-guided DIC hot path on one MI355X.

Workload: the 2048 x 2048 12-bit speckle pair with a sinusoidal displacement
u = 0.5 sin(2 pi x / lambda(y)), lambda from 10 to 300 px along y, v = 0,
noise sigma 4; subset 31, step 2 (1009^2 grid), affine shape, tol 1e-4,
50 iterations, one seed at the centre.  Synthetic inputs, rendered on the host
and resident in HBM before timing starts.

A step is one batched pass of the whole path (deformed-image prefilter, seed
search, every frontier wave of IC-GN, output) over a batch of B deformed
frames of that pair against the resident reference; `value` is converged
subsets per second over the K timed steps.  The plain (one frame per call)
engine is timed beside it, with its p50/p99 pair latency.  The two forms use
their own launch shapes, each picked by the autotuner on the workload itself.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOP_PER_PX_IT = {6: 91.0, 12: 115.0}   # algorithmic flops per subset pixel per IC-GN iteration
PEAK_FP32_TFLOPS = 157.3                  # MI355X published FP32 vector peak
PEAK_HBM_GBPS = 8000.0                   # MI355X published HBM3E bandwidth


def render_frames(w, nframes):
    """Reference plus `nframes` deformed frames that differ only in their noise."""
    from paper_2601_12941_amd import synth
    return synth.noise_frames(w, nframes)


def host_info():
    """The host CPUs the oracle baseline runs on (nproc, lscpu's model and topology)."""
    import subprocess
    info = {"os_cpu_count": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except Exception:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keep = ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)", "CPU max MHz")
        info["lscpu"] = {k.strip(): v.strip() for k, v in (ln.split(":", 1) for ln in out.splitlines() if ":" in ln)
                         if k.strip() in keep}
    except Exception:
        pass
    return info


def _oracle_crop(ref, deformed, roi, w, crop, threads):
    import oracle
    H, W = ref.shape
    y0, x0 = (H - crop) // 2, (W - crop) // 2
    sl = (slice(y0, y0 + crop), slice(x0, x0 + crop))
    t0 = time.perf_counter()
    r = oracle.correlate(ref[sl], deformed[sl], roi[sl], seeds=[(crop / 2, crop / 2, 0, 0)], threads=threads,
                         **w.params())
    return r, time.perf_counter() - t0


def cpu_baseline(ref, deformed, roi, w, crop, single_crop):
    """The FP64 oracle (WAVE order, OpenMP over the nodes of each wave) on the
    central crop x crop window of the same pair with the host's CPU share, and on
    the central single_crop window on one core.  Returns the record and the
    multi-core oracle result (the whole pair when crop is the image side)."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    r, dt = _oracle_crop(ref, deformed, roi, w, crop, threads)
    conv = int((r["status"] == 0).sum())
    rec = {"value": conv / dt, "unit": "converged subsets/s", "cores": threads, "kind": "oracle",
           "sample": "central %dx%d window of the same pair (%d converged subsets in %.1f s, WAVE order, "
                     "OpenMP over the nodes of each wave, %d threads)" % (crop, crop, conv, dt, threads),
           "host": host_info()}
    if single_crop > 0:
        r1, dt1 = _oracle_crop(ref, deformed, roi, w, single_crop, 1)
        c1 = int((r1["status"] == 0).sum())
        rec["single_core"] = {"value": c1 / dt1, "unit": "converged subsets/s", "cores": 1,
                              "sample": "central %dx%d window (%d converged subsets in %.1f s)" % (
                                  single_crop, single_crop, c1, dt1)}
    return rec, r


def accuracy(g, o, w, truth=None):
    """Error of a GPU result against the FP64 oracle on the same pair (nodes both
    call CONVERGED), status and wave-index agreement, and error against the
    ground-truth field at the node centres."""
    gs, os_ = g["status"].astype(np.int32), o["status"]
    active = os_ != 2
    both = (gs == 0) & (os_ == 0)
    du = np.abs(g["p"][0].astype(np.float64) - o["p"][0])[both]
    dv = np.abs(g["p"][1].astype(np.float64) - o["p"][1])[both]
    dz = np.abs(g["zncc"].astype(np.float64) - o["zncc"])[both]
    h = (w.N - 1) / 2.0
    dgrad = np.abs(g["p"][2:6].astype(np.float64) - o["p"][2:6])[:, both] * h
    rep = {"nodes_compared": int(both.sum()), "max_du_px": float(du.max()), "max_dv_px": float(dv.max()),
           "rms_du_px": float(np.sqrt(np.mean(du ** 2))), "rms_dv_px": float(np.sqrt(np.mean(dv ** 2))),
           "p999_duv_px": float(np.percentile(np.maximum(du, dv), 99.9)),
           "max_dgrad_times_h_px": float(dgrad.max()), "max_dzncc": float(dz.max()),
           "status_mismatch": float((gs != os_)[active].mean()),
           "wave_mismatch": float((g["wave"] != o["wave"])[both].mean())}
    if truth is not None:
        u, v = truth
        conv = gs == 0
        eu = np.abs(g["p"][0].astype(np.float64) - u)[conv]
        ev = np.abs(g["p"][1].astype(np.float64) - v)[conv]
        rep["vs_truth"] = {"rms_du_px": float(np.sqrt(np.mean(eu ** 2))), "rms_dv_px": float(np.sqrt(np.mean(ev ** 2))),
                           "max_du_px": float(eu.max()), "max_dv_px": float(ev.max())}
    return rep


def profiled_traffic():
    """HBM bytes per batched k_wave wave step (the launches of both launch chains)
    from the committed FETCH_SIZE / WRITE_SIZE counter runs, if they were taken on
    the kernel source and compile flags built now."""
    from paper_2601_12941_amd import build
    rec_path = os.path.join(ROOT, "profiles", "k_wave_2048_batched_traffic.json")
    try:
        rec = json.load(open(rec_path))
    except OSError:
        return None
    if rec.get("kernel_build_sha256") != build.kernel_build_id():
        return None
    return rec.get("traffic_bytes_per_wave_step", rec["traffic_bytes_per_launch"])


# the launch shapes the autotuner picks on the 2048^2 workload, fixed for the profiled runs
PROFILE_SHAPES = dict(tps=64, tile=36, plain_tps=128, plain_tile=36)
_SHAPE_ARGS = "--tps %(tps)d --tile %(tile)d --plain-tps %(plain_tps)d --plain-tile %(plain_tile)d" % PROFILE_SHAPES
PROFILE_BENCH = "bench.py --steps 2 --warmup 1 --latency-runs 3 --cpu-crop 0 " + _SHAPE_ARGS
PMC_BENCH = "bench.py --steps 1 --warmup 0 --latency-runs 1 --cpu-crop 0 " + _SHAPE_ARGS


def _short(name):
    name = name.replace("(anonymous namespace)::", "").replace("dicmi::", "").replace("void ", "")
    return name.split("(")[0]


BATCHED_KERNEL = "k_wave<6, 64, 16, true>"


def batched_steps(trace_dir, kb=BATCHED_KERNEL):
    """The batched k_wave launches of a rocprofv3 kernel trace: launch chains (the
    streams they ran on), launches, their average duration, and the duration of a
    wave step (the union of the time the chains' launches of one wave index run,
    which overlap), averaged over the steps."""
    import csv
    f = next(os.path.join(r, x) for r, _, fs in os.walk(trace_dir) for x in fs if x.endswith("kernel_trace.csv"))
    iv = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Stream_Id"])
          for r in csv.DictReader(open(f)) if _short(r["Kernel_Name"]) == kb]
    chains = len({q for _, _, q in iv})
    iv.sort()
    union, cs, ce = 0, iv[0][0], iv[0][1]
    for a, b, _ in iv[1:]:
        if a > ce:
            union += ce - cs
            cs, ce = a, b
        else:
            ce = max(ce, b)
    union += ce - cs
    steps = len(iv) / chains
    return dict(chains=chains, launches=len(iv), avg_launch_us=sum(b - a for a, b, _ in iv) / len(iv) / 1e3,
                step_us=union / steps / 1e3, steps=steps)


def _live_step_us(log):
    """roofline.avg_launch_us of the bench JSON line in a run's output, if any."""
    if not log or not os.path.exists(log):
        return None
    for ln in reversed(open(log, errors="replace").read().splitlines()):
        if ln.startswith("{") and '"roofline"' in ln:
            return json.loads(ln)["roofline"]["avg_launch_us"]
    return None


def summarize_trace(d, out, log=None):
    """profiles/*.md from a rocprofv3 --kernel-trace --stats directory (and the
    profiled run's output, for the live wave-step figure it printed)."""
    import csv
    stats = next(os.path.join(r, f) for r, _, fs in os.walk(d) for f in fs if f.endswith("kernel_stats.csv"))
    rows = list(csv.DictReader(open(stats)))
    from paper_2601_12941_amd import build
    kid = build.kernel_build_id()
    lines = ["# k_wave on the 2048^2 workload: rocprofv3 kernel trace", "",
             "Command (from the repository root on the MI355X box; rocprofv3 run from /tmp with TMPDIR=/tmp):", "",
             "```", "rocprofv3 --kernel-trace --stats -f csv -d <out> -o run -- python3 " + PROFILE_BENCH, "```", "",
             "Summary written by `python bench.py --summarize-trace <out> --summary-out <this file>`.", "",
             "Workload: 2048x2048 u16 speckle, sinusoidal u, subset 31, step 2, affine (1 010 025 active subsets per "
             "frame, 1005 waves). Batched form: 32 frames per call in two launch chains of 16 frames on two "
             "streams, %d threads per subset, %d-sample window "
             "(the autotuner's pick on this workload); plain form: one frame per call, %d threads per subset, "
             "%d-sample window (64 and 128 threads tie within 1%% for the plain form)." % (
                 PROFILE_SHAPES["tps"], PROFILE_SHAPES["tile"], PROFILE_SHAPES["plain_tps"],
                 PROFILE_SHAPES["plain_tile"]), "",
             "| Kernel | Calls | Total ms | Average us | % | Min us | Max us |", "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
        lines.append("| `%s` | %s | %.1f | %.1f | %.2f | %.1f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["Percentage"]), float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    b = batched_steps(d)
    live = _live_step_us(log)
    lines += ["", "Batched form (`%s`): %d launches on %d streams, %.1f us each on average; the two chains' launches "
              "of one wave index run side by side, so a wave step (the union of the time they run) takes %.1f us "
              "over %d wave steps. `bench.py` measures the wave step live with HIP events (`roofline.avg_launch_us`, "
              "chunks of back-to-back steps including the few-microsecond gaps between them)%s." % (
                  BATCHED_KERNEL, b["launches"], b["chains"], b["avg_launch_us"], b["step_us"], b["steps"],
                  ": %.1f us in this profiled run" % live if live else ""),
              "Kernel build at the time of this profile: sha256 `%s` of `paper_2601_12941_amd/csrc/dic_kernels.hip` "
              "and its compile flags (`build.kernel_build_id()`)."
              % kid]
    open(out, "w").write("\n".join(lines) + "\n")
    print("wrote", out)


def summarize_ext_trace(d, out):
    """profiles/*.md for the entry points around the path (--workload extensions)
    from a rocprofv3 --kernel-trace --stats directory: every kernel, calls, time."""
    import csv
    stats = next(os.path.join(r, f) for r, _, fs in os.walk(d) for f in fs if f.endswith("kernel_stats.csv"))
    rows = sorted(csv.DictReader(open(stats)), key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Entry points around the path: rocprofv3 kernel trace of `bench.py --workload extensions`", "",
             "Command (from the repository root on the MI355X box; rocprofv3 run from /tmp with TMPDIR=/tmp):", "",
             "```", "rocprofv3 --kernel-trace --stats -f csv -d <out> -o run -- python3 bench.py --workload extensions",
             "```", "",
             "Summary written by `python bench.py --summarize-ext-trace <out> --summary-out <this file>`. The run "
             "correlates: the 2048^2 large-displacement pair (multi-window guess 5 times with the sub-pixel fit, "
             "then `dic_correlate_mw` 3 times and one plain correlation); the 2048^2 u8 affine pair (ZNSSD "
             "affine 3 times, strain 10 times for each of two settings, the rigid shape, NSSD, SSD, LM and the "
             "quadratic shape 3 times each plus one warm-up each, out-of-core twice); the 1024^2 8-frame "
             "sequence twice. Calls count every launch of the run.", "",
             "| Kernel | Calls | Total ms | Average us | Min us | Max us |", "|---|---|---|---|---|---|"]
    for r in rows:
        if float(r["TotalDurationNs"]) < 1e5:
            continue
        lines.append("| `%s` | %s | %.2f | %.1f | %.1f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    lines += ["", "Kernels under 0.1 ms in total are left out."]
    open(out, "w").write("\n".join(lines) + "\n")
    print("wrote", out)


def summarize_pmc(fetch_dir, write_dir, cfetch_dir, cwrite_dir, out_md, out_json):
    """HBM byte counters per dispatch, scaled by what the same counters read for a
    256 MiB device copy; writes the summary table and the per-launch traffic of
    the batched k_wave that bench.py reports."""
    import csv

    def per_kernel(d, counter):
        f = next(os.path.join(r, x) for r, _, fs in os.walk(d) for x in fs if x.endswith("counter_collection.csv"))
        acc, disp = {}, {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            k = _short(r["Kernel_Name"])
            acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
            disp.setdefault(k, set()).add(r["Dispatch_Id"])
        return {k: (acc[k] / len(disp[k]), len(disp[k])) for k in acc}
    copy_bytes = 256 * (1 << 20)
    cf = max(per_kernel(cfetch_dir, "FETCH_SIZE").values(), key=lambda v: v[0])[0]
    cw = max(per_kernel(cwrite_dir, "WRITE_SIZE").values(), key=lambda v: v[0])[0]
    ff, wf = copy_bytes / 1024.0 / cf, copy_bytes / 1024.0 / cw
    fe, wr = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    from paper_2601_12941_amd import build
    kid = build.kernel_build_id()
    lines = ["# k_wave on the 2048^2 workload: HBM-side byte counters", "",
             "Commands (each a separate pass; rocprofv3 run from /tmp with TMPDIR=/tmp):", "", "```",
             "rocprofv3 --pmc FETCH_SIZE -f csv -d <fetch> -o run -- python3 " + PMC_BENCH,
             "rocprofv3 --pmc WRITE_SIZE -f csv -d <write> -o run -- python3 " + PMC_BENCH,
             "rocprofv3 --pmc FETCH_SIZE -f csv -d <copy_fetch> -o run -- python3 bench.py --copy-probe",
             "rocprofv3 --pmc WRITE_SIZE -f csv -d <copy_write> -o run -- python3 bench.py --copy-probe", "```", "",
             "Summary written by `python bench.py --summarize-pmc <fetch> <write> <copy_fetch> <copy_write>`.", "",
             "Calibration: a 256 MiB device copy reads FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB per dispatch "
             "(exact: 262144 KiB), so FETCH_SIZE is scaled by %.4f and WRITE_SIZE by %.4f." % (cf, cw, ff, wf), "",
             "| Kernel | Dispatches | FETCH_SIZE KiB/dispatch | scaled fetch MB/dispatch | WRITE_SIZE KiB/dispatch | "
             "scaled write MB/dispatch |", "|---|---|---|---|---|---|"]
    for k in sorted(fe, key=lambda k: -fe[k][0] * fe[k][1])[:10]:
        w = wr.get(k, (0.0, 0))[0]
        lines.append("| `%s` | %d | %.1f | %.2f | %.1f | %.2f |" % (k, fe[k][1], fe[k][0], fe[k][0] * 1024 * ff / 1e6,
                                                                    w, w * 1024 * wf / 1e6))
    kb = BATCHED_KERNEL
    fetch_b = fe[kb][0] * 1024 * ff
    write_b = wr[kb][0] * 1024 * wf
    # one batched step = 1020 wave steps of 2 launch chains on this workload
    chains = max(1, round(fe[kb][1] / 1020.0))
    lines += ["", "The batched form runs two launch chains of 16 frames: %d dispatches of `%s` per step, so a wave "
              "step (one launch of each chain) moves %.1f MB fetched + %.1f MB written." % (
                  fe[kb][1], kb, chains * fetch_b / 1e6, chains * write_b / 1e6),
              "Kernel build at the time of these counters: sha256 `%s` of the source and its compile flags." % kid]
    open(out_md, "w").write("\n".join(lines) + "\n")
    json.dump({"kernel": kb + " (batched form, 32 frames per call in %d launch chains)" % chains,
               "kernel_build_sha256": kid, "launch_chains": chains,
               "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
               "traffic_bytes_per_launch": fetch_b + write_b,
               "traffic_bytes_per_wave_step": chains * (fetch_b + write_b), "dispatches": fe[kb][1],
               "copy_calibration": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw, "fetch_factor": ff,
                                    "write_factor": wf}}, open(out_json, "w"), indent=1)
    print("wrote", out_md, out_json)


def summarize_l2(bench_dir, copy_dir, trace_dir, out_md):
    """profiles/k_wave_2048_l2_counters.md: L2 (TCC) read requests, hits and misses per
    dispatch of the batched k_wave, the request size calibrated on the 256 MiB copy, and
    the rate over the launch time of a kernel trace of the same build."""
    import csv

    def per_kernel(d):
        f = next(os.path.join(r, x) for r, _, fs in os.walk(d) for x in fs if x.endswith("counter_collection.csv"))
        acc, disp = {}, {}
        for r in csv.DictReader(open(f)):
            k = (_short(r["Kernel_Name"]), r["Counter_Name"])
            acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
            disp.setdefault(k, set()).add(r["Dispatch_Id"])
        return {k: (acc[k] / len(disp[k]), len(disp[k])) for k in acc}
    b, c = per_kernel(bench_dir), per_kernel(copy_dir)
    copy_reads = max(v[0] for k, v in c.items() if k[1] == "TCC_READ_sum")
    req_b = 256 * (1 << 20) / copy_reads
    kb = BATCHED_KERNEL
    rd, n = b[(kb, "TCC_READ_sum")]
    hit, miss = b[(kb, "TCC_HIT_sum")][0], b[(kb, "TCC_MISS_sum")][0]
    bt = batched_steps(trace_dir)
    avg_us, chains = bt["step_us"], bt["chains"]
    from paper_2601_12941_amd import build
    lines = ["# k_wave on the 2048^2 workload: L2 (TCC) counters", "",
             "Commands (each a separate pass; rocprofv3 run from /tmp with TMPDIR=/tmp, from the repository root "
             "on the MI355X box):", "", "```",
             "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum TCC_READ_sum -f csv -d <bench> -o run -- python3 " + PMC_BENCH,
             "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum TCC_READ_sum -f csv -d <copy> -o run -- python3 bench.py "
             "--copy-probe", "```", "",
             "Summary written by `python bench.py --summarize-l2 <bench> <copy> <trace>` (<trace>: the kernel trace "
             "of `k_wave_2048_kernel_trace.md`, for the launch time).", "",
             "Calibration: the 256 MiB device copy issues %.0f TCC read requests per dispatch, i.e. %.1f B per "
             "request (one 128 B line)." % (copy_reads, req_b), "",
             "| Kernel | Dispatches | TCC_READ_sum / dispatch | L2 read bytes / dispatch | TCC_HIT_sum | TCC_MISS_sum "
             "| hit rate |", "|---|---|---|---|---|---|---|",
             "| `%s` (batched, one launch chain of 16 frames) | %d | %.0f | %.0f MB | %.0f | %.0f | %.1f %% |" % (
                 kb, n, rd, rd * 128 / 1e6, hit, miss, 100.0 * hit / max(1.0, hit + miss)), "",
             "A wave step (one launch of each of the %d chains) reads %.0f MB from L2; over the %.1f us of a wave "
             "step (kernel trace of the same build) that is %.1f TB/s of L2 reads; the "
             "achievable L2 re-read rate measured by `dic_roof_cache_read` is 32.6 TB/s "
             "(`achievable_rates_mi355x.md`)." % (chains, chains * rd * 128 / 1e6, avg_us,
                                                   chains * rd * 128 / (avg_us * 1e-6) / 1e12), "",
             "Kernel build at the time of these counters: sha256 `%s`." % build.kernel_build_id()]
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("wrote", out_md)


SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_BUSY_CYCLES"]


def summarize_sq(sq_dir, trace_dir, out_md):
    """profiles/k_wave_2048_sq_counters.md: instructions per subset of the batched
    k_wave (one wavefront per subset at 64 threads) from one rocprofv3 --pmc pass, and
    the VALU issue rate over the launch time of a kernel trace of the same build."""
    import csv
    f = next(os.path.join(r, x) for r, _, fs in os.walk(sq_dir) for x in fs if x.endswith("counter_collection.csv"))
    acc, disp = {}, {}
    for r in csv.DictReader(open(f)):
        k = (_short(r["Kernel_Name"]), r["Counter_Name"])
        acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r["Dispatch_Id"])
    kb = BATCHED_KERNEL
    v = {c: acc[(kb, c)] / len(disp[(kb, c)]) for c in SQ_COUNTERS if (kb, c) in acc}
    n = len(disp[(kb, "SQ_WAVES")])
    bt = batched_steps(trace_dir)
    avg_us, chains = bt["step_us"], bt["chains"]
    # workgroups that find no subset exit at once: the subsets of the profiled step are
    # the converged subsets the benchmark counts (1 010 025 per frame, 32 frames), over
    # all `n` dispatches (the look-ahead launches that find no subset included)
    subsets = 1010025 * 32 / float(n)
    issue = chains * v["SQ_INSTS_VALU"] / (avg_us * 1e-6)
    simd_rate = 256 * 4 * 2.4e9 / 4          # one wave64 VALU instruction per SIMD every 4 clocks
    from paper_2601_12941_amd import build
    lines = ["# k_wave on the 2048^2 workload: SQ instruction counters", "",
             "Command (rocprofv3 run from /tmp with TMPDIR=/tmp, from the repository root on the MI355X box):", "",
             "```", "rocprofv3 --pmc " + " ".join(SQ_COUNTERS) + " -f csv -d <sq> -o run -- python3 " + PMC_BENCH,
             "```", "",
             "Summary written by `python bench.py --summarize-sq <sq> <trace>` (<trace>: the kernel trace of "
             "`k_wave_2048_kernel_trace.md`, for the launch time).", "",
             "| Counter | per dispatch of `%s` (%d dispatches) | per subset |" % (kb, n), "|---|---|---|"]
    for c in SQ_COUNTERS:
        if c in v:   # wavefronts and busy cycles are per launch, not per subset
            per = "" if c in ("SQ_WAVES", "SQ_BUSY_CYCLES") else "%.1f" % (v[c] / subsets)
            lines.append("| `%s` | %.0f | %s |" % (c, v[c], per))
    lines += ["", "Subsets per launch: %.1f on average (1 010 025 per frame, 32 frames in %d launch chains, %d "
              "launches)." % (subsets, chains, n),
              "VALU issue over the %.1f us wave step (the union of the %d chains' concurrent launches, kernel trace of "
              "the same build): %.2e instructions/s, %.0f %% of the %.2e that 1024 SIMDs issue at one wave64 "
              "instruction every 4 clocks (2.4 GHz)." % (avg_us, chains, issue, 100.0 * issue / simd_rate, simd_rate),
              "",
              "Kernel build at the time of these counters: sha256 `%s`." % build.kernel_build_id()]
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("wrote", out_md)


SQ_STALL_COUNTERS = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                     "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU"]


def summarize_sq_stalls(sq_dir, out_md):
    """profiles/k_wave_2048_sq_stalls.md: where the batched k_wave's wavefronts spend
    their cycles (issuing, waiting on memory or LDS, waiting for an issue slot), from
    one rocprofv3 --pmc pass over SQ_STALL_COUNTERS."""
    import csv
    f = next(os.path.join(r, x) for r, _, fs in os.walk(sq_dir) for x in fs if x.endswith("counter_collection.csv"))
    acc, disp = {}, {}
    for r in csv.DictReader(open(f)):
        k = (_short(r["Kernel_Name"]), r["Counter_Name"])
        acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r["Dispatch_Id"])
    kb = BATCHED_KERNEL
    tot = {c: acc[(kb, c)] for c in SQ_STALL_COUNTERS if (kb, c) in acc}
    n = len(disp[(kb, "SQ_WAVES")])
    subsets = 1010025 * 32.0
    wc = tot["SQ_WAVE_CYCLES"]
    from paper_2601_12941_amd import build
    lines = ["# k_wave on the 2048^2 workload: where the wavefronts' cycles go", "",
             "Command (rocprofv3 run from /tmp with TMPDIR=/tmp, from the repository root on the MI355X box):", "",
             "```", "rocprofv3 --pmc " + " ".join(SQ_STALL_COUNTERS) + " -f csv -d <sq> -o run -- python3 " + PMC_BENCH,
             "```", "",
             "Summary written by `python bench.py --summarize-sq-stalls <sq>`. Batched form: one step of 32 frames "
             "in two launch chains, %d dispatches of `%s` (the look-ahead launches included)." % (n, kb), "",
             "| Counter | total over the step | per subset | share of SQ_WAVE_CYCLES |", "|---|---|---|---|"]
    for c in SQ_STALL_COUNTERS:
        if c not in tot:
            continue
        share = "%.3f" % (tot[c] / wc) if c.startswith(("SQ_WAIT", "SQ_ACTIVE")) else ""
        lines.append("| `%s` | %.4g | %.1f | %s |" % (c, tot[c], tot[c] / subsets, share))
    lines += ["", "SQ_WAVE_CYCLES counts every resident wavefront's cycles; SQ_WAIT_ANY the cycles a wavefront "
              "waits on an `s_waitcnt` (memory, LDS, scalar loads), SQ_WAIT_INST_ANY those it waits for an "
              "instruction to issue, SQ_ACTIVE_INST_VALU those it issues VALU work (the SQ's own cycle units: the "
              "shares, not the absolute counts, are what this table is for). Two wavefronts share each SIMD.", "",
              "Kernel build at the time of these counters: sha256 `%s`." % build.kernel_build_id()]
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("wrote", out_md)


def copy_probe(mib=256, reps=3):
    """A device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE counters
    read `mib` MiB each per dispatch on an exact counter."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": mib * (1 << 20), "reps": reps}))


def gigapixel(args, repeats=6, samples=24):
    """The 32768^2 u8 pair (rigid shift + Gaussian bump, subset 41, step 20, 16
    seeds): repeated correlations for the pair latency, and sampled parity
    against the oracle on 256^2 crops centred on the sampled nodes."""
    import torch
    import oracle
    from paper_2601_12941_amd import dic, synth

    w = synth.workload("c4")
    t0 = time.perf_counter()

    def note(msg):
        print("# %6.1f s  %s" % (time.perf_counter() - t0, msg), file=sys.stderr, flush=True)
    X, Y, S, A = synth.draw_blobs(w.W, w.H, w.nblobs, w.sigma, w.amp, w.seed_blobs)
    note("%d blobs drawn" % X.size)
    field = w.field()
    ref = synth._finish(synth._render_blobs_large(w.W, w.H, X, Y, S, A), w.noise, w.seed_noise_ref, w.bits)
    note("reference rendered")
    u0, v0 = field(X, Y)
    de = synth._finish(synth._render_blobs_large(w.W, w.H, X + u0, Y + v0, S, A), w.noise, w.seed_noise_def, w.bits)
    note("deformed rendered")
    del X, Y, S, A, u0, v0
    pair = synth.Pair(ref, de, synth.roi_from_field(w.W, w.H, field), field, w.bits)
    note("roi done")
    t_render = time.perf_counter() - t0
    d_ref = dic.to_device_image(pair.ref)
    d_def = dic.to_device_image(pair.deformed)
    d_roi = torch.from_numpy(pair.roi).cuda()
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    eng = dic.Engine(0)
    # launch shape: time each candidate on the pair itself (two correlations each)
    shapes = [(args.giga_tps, args.giga_tile)] if args.giga_tps else \
        [(tps, w.N + dt) for tps in (128, 256) for dt in (5, 9)]
    sweep = []
    if len(shapes) > 1:
        for tps, ts in shapes:
            eng.set_reference(d_ref, d_roi, **w.params(), threads_per_subset=tps, tile_side=ts)
            tt = []
            for _ in range(2):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                eng.correlate(d_def, w.seeds)
                torch.cuda.synchronize()
                tt.append(time.perf_counter() - t1)
            sweep.append({"threads_per_subset": tps, "tile_side": ts, "ms": min(tt) * 1e3})
            note("shape %d threads, window %d: %.1f ms" % (tps, ts, min(tt) * 1e3))
    best = min(sweep, key=lambda r: r["ms"]) if sweep else {"threads_per_subset": shapes[0][0],
                                                            "tile_side": shapes[0][1]}
    t0 = time.perf_counter()
    eng.set_reference(d_ref, d_roi, **w.params(), threads_per_subset=best["threads_per_subset"],
                      tile_side=best["tile_side"])
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    lat = []
    out = None
    for i in range(repeats + 1):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = eng.correlate(d_def, w.seeds)
        torch.cuda.synchronize()
        if i > 0:
            lat.append(time.perf_counter() - t1)
    st = eng.stats()
    free1, _ = torch.cuda.mem_get_info()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    # sampled parity: oracle from the ground-truth shape on a crop around the node
    rng = np.random.default_rng(11)
    h = (w.N - 1) // 2
    u, v, (ux, uy, vx, vy) = synth.truth_at_nodes(pair.field, w.W, w.H, w.N, w.step)
    cand = np.argwhere(g["status"] == 0)
    pick = cand[rng.choice(len(cand), min(samples, len(cand)), replace=False)]
    C = 128
    errs, dz, used = [], [], 0
    for j, i in pick:
        xc, yc = h + i * w.step, h + j * w.step
        y0, x0 = max(0, yc - C), max(0, xc - C)
        sl = (slice(y0, min(w.H, yc + C)), slice(x0, min(w.W, xc + C)))
        t = np.array([u[j, i], v[j, i], ux[j, i], uy[j, i], vx[j, i], vy[j, i]])
        a = oracle.icgn(pair.ref[sl], pair.deformed[sl], xc - x0, yc - y0, t, w.N, 6, tol=w.tol, max_iter=w.max_iter)
        b = oracle.icgn(pair.ref[sl], pair.deformed[sl], xc - x0, yc - y0, t + np.array([0.3, -0.3, 0, 0, 0, 0]),
                        w.N, 6, tol=w.tol, max_iter=w.max_iter)
        if a[3] != 0 or b[3] != 0 or np.abs(a[0][:2] - b[0][:2]).max() > 2e-4:
            continue
        used += 1
        errs.append(max(abs(g["p"][0, j, i] - a[0][0]), abs(g["p"][1, j, i] - a[0][1])))
        dz.append(abs(g["zncc"][j, i] - a[1]))
    conv = (g["status"] == 0)
    err_truth = np.hypot(g["p"][0] - u, g["p"][1] - v)[conv]
    lat_ms = np.array(lat) * 1e3
    rec = {"workload": "32768x32768 u8 speckle, shift (3.41, -7.92) + Gaussian bump, subset 41, step 20, 16 seeds",
           "nodes": st["nodes"], "active": st["active"], "converged": int(conv.sum()), "waves": st["waves"],
           "threads_per_subset": st["threads_per_subset"], "tile_side": best["tile_side"],
           "launch_shape_sweep": sweep, "repeats": repeats,
           "latency_ms_p50": float(np.percentile(lat_ms, 50)), "latency_ms_p99": float(np.percentile(lat_ms, 99)),
           "converged_subsets_per_s": float(conv.sum() / np.median(lat)), "set_reference_ms": t_ref * 1e3,
           "render_s": t_render, "sampled_parity": {"nodes": used, "max_duv_px": float(max(errs)) if errs else None,
                                                     "max_dzncc": float(max(dz)) if dz else None},
           "error_vs_truth_px": {"rms": float(np.sqrt((err_truth ** 2).mean())), "max": float(err_truth.max())},
           "library_device_memory_gb": (free0 - free1) / 1e9,
           "input_device_memory_gb": (pair.ref.nbytes + pair.deformed.nbytes + pair.roi.nbytes) / 1e9}
    print(json.dumps(rec))
    eng.close()


def precision(args):
    """Precision sweep on the 4096^2-recipe u8 pair with the quadratic field and
    2 % strain, drawn at --precision-size: subsets 21 and 41 (step 4), affine and
    quadratic shape functions, FP32- and FP16-stored deformed coefficients (FP32
    interpolation, FP64 reductions and solve), each compared node by node with
    the FP64 oracle run in the same wave order, and with the ground truth."""
    import torch
    import oracle
    from paper_2601_12941_amd import dic, synth

    size = args.precision_size
    w0 = synth.workload("c3", size=size)
    pair = w0.pair()
    d_ref = dic.to_device_image(pair.ref)
    d_def = dic.to_device_image(pair.deformed)
    d_roi = torch.from_numpy(pair.roi).cuda()
    rows = []
    for N in (21, 41):
        for shape in (6, 12):
            w = synth.workload("c3", size=size, N=N, shape=shape)
            t0 = time.perf_counter()
            o = oracle.correlate(pair.ref, pair.deformed, pair.roi, seeds=w.seeds, threads=16,
                                 **{k: v for k, v in w.params().items()})
            t_or = time.perf_counter() - t0
            print("# oracle N%d shape %d: %.1f s" % (N, shape, t_or), file=sys.stderr, flush=True)
            u, v, _ = synth.truth_at_nodes(pair.field, size, size, N, w.step)
            for fp16 in (False, True):
                eng = dic.Engine(0)
                eng.set_reference(d_ref, d_roi, **w.params(), coef_fp16=fp16)
                out = eng.correlate(d_def, w.seeds)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                out = eng.correlate(d_def, w.seeds)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t1) * 1e3
                g = {k: t.cpu().numpy() for k, t in out.items()}
                eng.close()
                act = o["status"] != oracle.ST["NOT_IN_ROI"]
                both = (g["status"] == 0) & (o["status"] == 0)
                duv = np.maximum(np.abs(g["p"][0] - o["p"][0]), np.abs(g["p"][1] - o["p"][1]))[both]
                dz = np.abs(g["zncc"] - o["zncc"])[both]
                et = np.hypot(g["p"][0] - u, g["p"][1] - v)[g["status"] == 0]
                rows.append({"subset": N, "shape": "quadratic" if shape == 12 else "affine",
                             "coefficients": "fp16" if fp16 else "fp32", "nodes_compared": int(both.sum()),
                             "max_duv_px": float(duv.max()), "rms_duv_px": float(np.sqrt((duv ** 2).mean())),
                             "nodes_over_1e-3_px": int((duv > 1e-3).sum()),
                             "p999_duv_px": float(np.percentile(duv, 99.9)), "max_dzncc": float(dz.max()),
                             "status_mismatch": float((g["status"] != o["status"])[act].mean()),
                             "vs_truth_rms_px": float(np.sqrt((et ** 2).mean())), "vs_truth_max_px": float(et.max()),
                             "gpu_ms": ms, "oracle_s": t_or})
                print("# " + json.dumps(rows[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"workload": "precision sweep: %d^2 u8 speckle, u = 1e-5 x^2 + 0.3 + 0.02 x, "
                                  "v = -2e-5 xy + 0.2 + 0.02 y about the centre, step 4" % size,
                      "reductions": "fp64", "rows": rows}))


def serve(args):
    """The serving mix: 8 resident 4096^2 u8 references; requests arrive as a
    Poisson process (rate per second, fixed duration) and each correlates a
    deformed centred S x S window (S from 256 to 4096) with its own subset
    size (15..51), step (1, 2, 5) and random affine field.  Frames are rendered
    and resident on the device before the clock starts.  Reference precomputes
    are made resident on demand and the least recently used idle ones are
    released when the HBM budget needs room; that registration time is inside
    the measured latency.  Latency runs from the arrival on the virtual clock to
    u, v, ZNCC and status on the host."""
    import collections
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from paper_2601_12941_amd import dic, synth

    t00 = time.perf_counter()

    def note(msg):
        print("# %6.1f s  %s" % (time.perf_counter() - t00, msg), file=sys.stderr, flush=True)
    trace = synth.serve_trace(args.duration, args.rate)
    nref = 8
    blobs = [synth.serve_reference_blobs(r) for r in range(nref)]
    with ThreadPoolExecutor(4) as ex:
        refs = list(ex.map(lambda r: synth.serve_reference(r, blobs[r]), range(nref)))
    d_refs = [torch.from_numpy(r).cuda() for r in refs]
    note("%d references rendered" % nref)
    # a sample checked against the oracle afterwards: small windows only
    rng = np.random.default_rng(7)
    small = [q.index for q in trace if q.S <= 512 and q.N <= 31]
    sample = set(rng.choice(small, min(args.parity_samples, len(small)), replace=False).tolist()) if small else set()
    frames, host_frames = [None] * len(trace), {}
    with ThreadPoolExecutor(4) as ex:
        for q, f in zip(trace, ex.map(lambda q: synth.serve_frame(q, blobs[q.ref]), trace)):
            frames[q.index] = torch.from_numpy(f).cuda()
            if q.index in sample:
                host_frames[q.index] = f
            if q.index % 200 == 0:
                note("frame %d of %d rendered" % (q.index, len(trace)))
    rois = {S: torch.from_numpy(synth.serve_roi(S)).cuda() for S in synth.SERVE_SIZES}
    torch.cuda.synchronize()
    note("%d frames resident" % len(trace))

    def window(r, S):
        o = synth.serve_window(S)
        return d_refs[r][o:o + S, o:o + S]

    # launch shapes per subset size, tuned for many requests in flight (batch 16)
    from paper_2601_12941_amd import autotune
    shapes = {}
    for N in synth.SERVE_SUBSETS:
        ch = autotune.choose(N, 2, batch=16, size=1024, seed_radius=8, use_cache=False,
                             log=lambda m: print("# " + m, file=sys.stderr, flush=True))
        shapes[N] = (ch["threads_per_subset"], ch["tile_side"])
    note("launch shapes tuned: %s" % shapes)

    def params(N, st):
        return dict(subset_size=N, step=st, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7, seed_radius=8,
                    threads_per_subset=shapes[N][0], tile_side=shapes[N][1])

    srv = dic.Server(0, max_active=args.max_active, hbm_budget_bytes=args.budget_gb * 1e9)
    # warm-up: every kernel shape once on a 256^2 request, outside the clock
    wq = min((q for q in trace if q.S == 256), key=lambda q: q.index, default=None)
    for N in synth.SERVE_SUBSETS if wq is not None else ():
        rid = srv.add_reference(window(wq.ref, 256), rois[256], **params(N, 5))
        t, _ = srv.submit(rid, frames[wq.index], [(128.0, 128.0, 0.0, 0.0)])
        while not srv.poll(t)[0]:
            srv.step(8)
        srv.remove_reference(rid)
    torch.cuda.synchronize()
    note("warm-up done")

    resident = collections.OrderedDict()      # (ref, S, N, step) -> reference id, least recently used first
    inuse = collections.Counter()
    reg = dict(count=0, ms=0.0, evictions=0)

    def ensure(q):
        key = (q.ref, q.S, q.N, q.step)
        if key in resident:
            resident.move_to_end(key)
            return resident[key]
        while True:
            t1 = time.perf_counter()
            try:
                rid = srv.add_reference(window(q.ref, q.S), rois[q.S], **params(q.N, q.step))
            except dic.DicError as e:
                if e.code != dic.DIC_E_NOMEM:
                    raise
                idle = [k for k, v in resident.items() if inuse[v] == 0]
                if not idle:
                    return None
                srv.remove_reference(resident.pop(idle[0]))
                reg["evictions"] += 1
                continue
            reg["count"] += 1
            reg["ms"] += (time.perf_counter() - t1) * 1e3
            resident[key] = rid
            return rid

    cs = torch.cuda.Stream()
    pending = collections.deque()
    inflight, copies = {}, []
    done_at, conv = {}, {}
    kept = {}
    qlog = []
    nxt = 0
    next_log = 0.0
    t0 = time.perf_counter()
    while len(done_at) < len(trace):
        now = time.perf_counter() - t0
        while nxt < len(trace) and trace[nxt].arrival <= now:
            pending.append(nxt)
            nxt += 1
        # hand requests to the server while its own queue is short, so that queued
        # requests do not pin references that idle ones could make room for
        while pending and srv.stats()["waiting"] < 2:
            q = trace[pending[0]]
            rid = ensure(q)
            if rid is None:
                break
            c = q.S / 2.0
            t, out = srv.submit(rid, frames[q.index], [(c, c, 0.0, 0.0)])
            inflight[t] = (q.index, out, rid)
            inuse[rid] += 1
            pending.popleft()
        if inflight:
            srv.step(args.chunk)
            ss = srv.stats()
            # requests that finished in this step leave free slots that the next step's
            # admission fills, so a waiting request beside a free slot is held by the
            # budget only once the used bytes are within one request's scratch of it
            # (below 1 GB on this mix: a 4096^2 window at step 1 needs 0.4 GB)
            if (ss["waiting"] > 0 and ss["active"] < args.max_active
                    and ss["used_bytes"] > args.budget_gb * 1e9 - 1e9):
                # admission is held by the budget: release the least recently used idle reference
                idle = [k for k, v in resident.items() if inuse[v] == 0]
                if idle:
                    srv.remove_reference(resident.pop(idle[0]))
                    reg["evictions"] += 1
            for t in list(inflight):
                done, status, st = srv.poll(t)
                if not done:
                    continue
                i, out, rid = inflight.pop(t)
                srv.forget(t)
                inuse[rid] -= 1
                if status != dic.DIC_OK:
                    raise RuntimeError("request %d failed with status %d" % (i, status))
                conv[i] = st["converged"]
                cs.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(cs):
                    host = {k: torch.empty(out[k][:2].shape if k == "p" else out[k].shape, dtype=out[k].dtype,
                                           pin_memory=True) for k in ("p", "zncc", "status")}
                    host["p"].copy_(out["p"][:2], non_blocking=True)
                    host["zncc"].copy_(out["zncc"], non_blocking=True)
                    host["status"].copy_(out["status"], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(cs)
                copies.append((i, ev, host, out))
        elif not pending and nxt < len(trace):
            time.sleep(max(0.0, min(0.002, trace[nxt].arrival - (time.perf_counter() - t0))))
        still = []
        for i, ev, host, out in copies:
            if ev.query():
                done_at[i] = time.perf_counter() - t0
                if i in sample:
                    kept[i] = {k: v.numpy().copy() for k, v in host.items()}
            else:
                still.append((i, ev, host, out))
        copies = still
        now = time.perf_counter() - t0
        if now >= next_log:
            s = srv.stats()
            qlog.append([round(now, 2), len(pending) + s["waiting"], s["active"], len(resident),
                         round(s["used_bytes"] / 1e9, 1)])
            next_log += 1.0
    t_end = time.perf_counter() - t0
    note("serving done")
    lat = np.array([done_at[q.index] - q.arrival for q in trace]) * 1e3
    sizes = {}
    for q in trace:
        sizes.setdefault(q.S, []).append(done_at[q.index] - q.arrival)
    subsets = sum(conv.values())
    offered = sum(np.prod(synth.grid_shape(q.S, q.S, q.N, q.step)) for q in trace) / args.duration
    last_arrival = trace[-1].arrival
    # sampled parity against the oracle, and error against the ground truth
    errs, dz, agree, terr = [], [], [], []
    for i in sorted(kept):
        q = trace[i]
        o = synth.serve_window(q.S)
        refw = refs[q.ref][o:o + q.S, o:o + q.S]
        r = oracle.correlate(np.ascontiguousarray(refw), host_frames[i], synth.serve_roi(q.S),
                             seeds=[(q.S / 2.0, q.S / 2.0, 0.0, 0.0)], threads=16,
                             **{k: v for k, v in params(q.N, q.step).items()
                                if k not in ("threads_per_subset", "tile_side")})
        g = kept[i]
        both = (g["status"] == 0) & (r["status"] == 0)
        act = r["status"] != oracle.ST["NOT_IN_ROI"]
        agree.append(float((g["status"] == r["status"])[act].mean()))
        if both.any():
            errs.append(float(max(np.abs(g["p"][0] - r["p"][0])[both].max(), np.abs(g["p"][1] - r["p"][1])[both].max())))
            dz.append(float(np.abs(g["zncc"] - r["zncc"])[both].max()))
        u, v, _ = synth.truth_at_nodes(q.field(), q.S, q.S, q.N, q.step)
        cg = g["status"] == 0
        if cg.any():
            terr.append(float(np.sqrt(((g["p"][0] - u) ** 2 + (g["p"][1] - v) ** 2)[cg].mean())))
    note("sampled parity done")
    rec = {"workload": "serving mix: 8 resident 4096^2 u8 references, Poisson %.0f req/s for %.0f s, windows "
                       "256..4096, subsets 15..51, steps 1/2/5, affine" % (args.rate, args.duration),
           "requests": len(trace), "max_active": args.max_active, "budget_gb": args.budget_gb,
           "steps_per_call": args.chunk,
           "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
           "latency_ms_p50_by_window": {str(S): float(np.percentile(np.array(v) * 1e3, 50)) for S, v in
                                        sorted(sizes.items())},
           "latency_ms_p99_by_window": {str(S): float(np.percentile(np.array(v) * 1e3, 99)) for S, v in
                                        sorted(sizes.items())},
           "offered_subsets_per_s": float(offered),
           "served_converged_subsets_per_s": float(subsets / t_end), "converged_subsets": int(subsets),
           "makespan_s": t_end, "drain_after_last_arrival_s": t_end - last_arrival,
           "keeps_up": bool(t_end - last_arrival < 2.0),
           "queue_per_second": {"columns": ["t_s", "queued", "active", "resident_refs", "used_gb"], "rows": qlog},
           "registrations": reg["count"], "registration_ms_total": reg["ms"], "evictions": reg["evictions"],
           "launch_shapes": {str(N): {"threads_per_subset": v[0], "tile_side": v[1]} for N, v in shapes.items()},
           "sampled_parity": {"requests": len(kept), "max_duv_px": max(errs) if errs else None,
                              "max_dzncc": max(dz) if dz else None, "min_status_agree": min(agree) if agree else None},
           "error_vs_truth_rms_px_max_over_sample": max(terr) if terr else None}
    print(json.dumps(rec))
    srv.close()


def _event_ms(fn, reps):
    """Median over reps of the device time between events recorded on the
    current stream (the library's stream) around one call, and the last result."""
    import torch
    ts, r = [], None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r = fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), r


def _host_s(fn):
    t = time.perf_counter()
    r = fn()
    return time.perf_counter() - t, r


def extensions(args):
    """The entry points beyond the single-pair path, each timed on MI355X on a
    workload of the paper's kind, with the oracle timed beside it on a bounded
    sample (one host thread unless stated): multi-window FFT initial guess and
    the correlation it seeds, strain, the rigid shape, NSSD/SSD costs and
    Levenberg-Marquardt, multi-frame correlation with reference updating, and
    out-of-core (band-by-band) correlation from host memory."""
    import torch
    import oracle
    from oracle import chunked as OCH
    from oracle import sequence as OSQ
    from oracle import strain as OST
    from paper_2601_12941_amd import dic, synth
    t0 = time.perf_counter()
    rows = []

    def note(msg):
        print("# %6.1f s  %s" % (time.perf_counter() - t0, msg), file=sys.stderr, flush=True)

    def emit(rec):
        rows.append(rec)
        note(json.dumps(rec))

    eng = dic.Engine(0)
    # ---- multi-window FFT guess and the correlation it seeds: 2048^2 dense speckle,
    # translation ~0.15 image widths (far beyond any integer search radius)
    w = synth.workload("large", size=args.size)
    pair = w.pair()
    d_ref, d_def = dic.to_device_image(pair.ref), dic.to_device_image(pair.deformed)
    d_roi = torch.from_numpy(pair.roi).cuda()
    eng.set_reference(d_ref, d_roi, **w.params())
    ms, r = _event_ms(lambda: eng.multiwindow(d_def, max_disp=w.max_disp, subpixel=True), 5)
    nodes = int(r["valid"].sum().item())
    wo = synth.workload("large", size=384)
    po = wo.pair()
    sec, ro = _host_s(lambda: oracle.multiwindow(po.ref, po.deformed, po.roi, subset_size=wo.N, step=wo.step,
                                                 max_disp=wo.max_disp, subpixel=True))
    # algorithmic work: per window pair of side W, 20 W^2 log2 W flop of transforms, its
    # 2 W^2 pixels, and for windows above 64 samples (HBM batch buffers) 128 W^2 bytes
    # of complex traffic; level grids: 50 %-overlap tiles of the image, then the nodes
    nxn, nyn = eng.grid[0], eng.grid[1]
    flop, nbytes, nwin = 0.0, 0.0, 0
    for li, Wl in enumerate(r["levels"]):
        cnt = nxn * nyn if li == len(r["levels"]) - 1 else \
            ((w.W - Wl) // (Wl // 2) + 1) * ((w.H - Wl) // (Wl // 2) + 1)
        nwin += cnt
        flop += cnt * 20.0 * Wl * Wl * math.log2(Wl)
        nbytes += cnt * (2.0 * Wl * Wl + (128.0 * Wl * Wl if Wl > 64 else 0.0))
    emit({"row": "multiwindow", "workload": "%d^2 u8 dense speckle, translation (%.1f, %.1f) px + 1 %% / -0.5 %% "
          "strain, subset %d, step %d, max_disp %d, sub-pixel fit, MAD 2.0" % (
              w.W, 0.1526 * w.W, -0.0915 * w.W, w.N, w.step, w.max_disp),
          "levels": r["levels"], "ms": ms, "valid_nodes": nodes, "nodes_per_s": nodes / (ms / 1e3),
          "window_pairs": nwin, "algorithmic_gflop": flop / 1e9, "algorithmic_gb": nbytes / 1e9,
          "achieved_tflops": flop / (ms / 1e3) / 1e12, "achieved_GBps": nbytes / (ms / 1e3) / 1e9,
          "cpu_oracle": {"kind": "oracle", "cores": 1, "sample": "384^2 pair of the same recipe",
                         "nodes_per_s": float(ro["valid"].sum() / sec), "s": sec}})
    ms_mw, g = _event_ms(lambda: eng.correlate_mw(d_def, w.seeds, max_disp=w.max_disp), 3)
    conv = int((g["status"] == 0).sum().item())
    ms_plain, gp = _event_ms(lambda: eng.correlate(d_def, w.seeds), 1)
    emit({"row": "correlate_mw", "workload": "as multiwindow; affine, reliability-guided from the estimate",
          "ms": ms_mw, "converged": conv, "converged_per_s": conv / (ms_mw / 1e3),
          "plain_seed_search_converged": int((gp["status"] == 0).sum().item())})
    del d_ref, d_def, d_roi, pair

    # ---- the 2048^2 u8 affine workload: strain, variants, out-of-core
    w = synth.workload("c1", size=args.size)
    pair = w.pair()
    d_ref, d_def = dic.to_device_image(pair.ref), dic.to_device_image(pair.deformed)
    d_roi = torch.from_numpy(pair.roi).cuda()
    eng.set_reference(d_ref, d_roi, **w.params())
    base_ms, base = _event_ms(lambda: eng.correlate(d_def, w.seeds), 3)
    base_conv = int((base["status"] == 0).sum().item())
    wl = "%d^2 u8 speckle, affine field, subset %d, step %d" % (w.W, w.N, w.step)
    emit({"row": "znssd_affine_gn", "workload": wl, "ms": base_ms, "converged": base_conv,
          "converged_per_s": base_conv / (base_ms / 1e3)})
    ny, nx = base["status"].shape
    u, v, stt = base["p"][0].contiguous(), base["p"][1].contiguous(), base["status"].contiguous()
    us, vs, ss = base["p"][0].cpu().numpy(), base["p"][1].cpu().numpy(), base["status"].cpu().numpy()
    for win, basis, meas in ((5, "bilinear", "green_lagrange"), (9, "biquadratic", "hencky")):
        ms, _ = _event_ms(lambda: eng.strain(u, v, stt, step=w.step, window=win, basis=basis, measure=meas), 10)
        crop = (slice(ny // 2 - 48, ny // 2 + 48), slice(nx // 2 - 48, nx // 2 + 48))
        sec, _ = _host_s(lambda: OST.strain(us[crop], vs[crop], w.step, win, basis, meas, valid=ss[crop] == 0))
        nb = nx * ny * (4 + 4 + 1 + 7 * 4)
        emit({"row": "strain", "workload": "%s result grid %dx%d, window %d, %s, %s" % (wl, nx, ny, win, basis, meas),
              "ms": ms, "nodes_per_s": nx * ny / (ms / 1e3), "algorithmic_bytes": nb,
              "achieved_GBps": nb / (ms / 1e3) / 1e9,
              "cpu_oracle": {"kind": "oracle", "cores": 1, "sample": "96x96-node crop of the same grid",
                             "nodes_per_s": 96 * 96 / sec, "s": sec}})
    crop_w = synth.workload("c1", size=512)
    cpair = crop_w.pair()
    for name, over in (("rigid_znssd", dict(shape=2)), ("nssd_affine", dict(cost="nssd")),
                       ("ssd_affine", dict(cost="ssd")), ("znssd_affine_lm", dict(lm_lambda=1e-3)),
                       ("znssd_quadratic_gn", dict(shape=12))):
        prm = dict(w.params())
        prm.update(over)
        eng.set_reference(d_ref, d_roi, **prm)
        ms, g = _event_ms(lambda: eng.correlate(d_def, w.seeds), 3)
        conv = int((g["status"] == 0).sum().item())
        po = {k: v for k, v in crop_w.params().items() if k not in ("coef_fp16", "reduce_fp64", "threads_per_subset",
                                                                      "nan_unconverged", "tile_side")}
        po.update(over)
        sec, ro = _host_s(lambda: oracle.correlate(cpair.ref, cpair.deformed, cpair.roi, seeds=crop_w.seeds,
                                                   threads=1, **po))
        emit({"row": name, "workload": wl, "ms": ms, "converged": conv, "converged_per_s": conv / (ms / 1e3),
              "vs_znssd_affine_gn": base_ms / ms,
              "cpu_oracle": {"kind": "oracle", "cores": 1, "sample": "512^2 pair of the same recipe",
                             "converged_per_s": float((ro["status"] == 0).sum() / sec), "s": sec}})
    # out-of-core: host images, one band of 32 node rows (+16 halo rows) on the device at a time
    prm = dict(w.params())
    ref_h, def_h, roi_h = pair.ref, pair.deformed, pair.roi
    sec, g = _host_s(lambda: eng.correlate_chunked(ref_h, def_h, roi_h, seeds=w.seeds, band_rows=32, halo=16, **prm))
    sec2, g = _host_s(lambda: eng.correlate_chunked(ref_h, def_h, roi_h, seeds=w.seeds, band_rows=32, halo=16,
                                                    **prm))
    conv = int((g["status"] == 0).sum())
    po = {k: v for k, v in crop_w.params().items() if k not in ("coef_fp16", "reduce_fp64", "threads_per_subset",
                                                                  "nan_unconverged", "tile_side")}
    osec, ro = _host_s(lambda: OCH.correlate_chunked(cpair.ref, cpair.deformed, cpair.roi, seeds=crop_w.seeds,
                                                     band_rows=8, halo=16, **po))
    emit({"row": "chunked", "workload": wl + "; host images, bands of 32 node rows, halo 16", "s": min(sec, sec2),
          "converged": conv, "converged_per_s": conv / min(sec, sec2),
          "device_resident_ms": base_ms, "band_rows_on_device": 32 * w.step + w.N + 32,
          "cpu_oracle": {"kind": "oracle", "cores": 1, "sample": "512^2 pair, bands of 8 node rows",
                         "converged_per_s": float((ro["status"] == 0).sum() / osec), "s": osec}})
    del d_ref, d_def, d_roi

    # ---- sequence with reference updating: 1024^2, 8 frames of a growing stretch
    W, F = args.size // 2, 8
    X, Y, Sg, A = synth.draw_blobs(W, W, int(0.03 * W * W), (1.5, 3.0), (60, 200), 77)
    ref = synth._finish(synth._render_blobs(W, W, X, Y, Sg, A), 2.0, 78, 8)
    frames = []
    for k in range(F):
        fld = synth.field_affine(0.0, 0.0, dudx=0.03 * k, dvdy=0.03 * k, xc=W / 2, yc=W / 2)
        uu, vv = fld(X, Y)
        frames.append(synth._finish(synth._render_blobs(W, W, X + uu, Y + vv, Sg, A), 2.0, 79 + k, 8))
    roi = np.zeros((W, W), np.uint8)
    m = W // 5
    roi[m:W - m, m:W - m] = 1
    d_roi = torch.from_numpy(roi).cuda()
    prm = dict(subset_size=21, step=4, seed_radius=3)
    eng.set_reference(dic.to_device_image(ref), d_roi, **prm)
    d_frames = [dic.to_device_image(f) for f in frames]
    seeds = [(W / 2, W / 2, 0, 0)]
    ms, (outs, refs) = _event_ms(lambda: eng.correlate_sequence(d_frames, seeds, d_roi, min_converged=0.9,
                                                                min_zncc=0.999), 1)
    eng.set_reference(dic.to_device_image(ref), d_roi, **prm)
    ms, (outs, refs) = _event_ms(lambda: eng.correlate_sequence(d_frames, seeds, d_roi, min_converged=0.9,
                                                                min_zncc=0.999), 1)
    conv = [int((o["status"] == 0).sum().item()) for o in outs]
    Ws = 192
    Xs, Ys, Ss, As = synth.draw_blobs(Ws, Ws, int(0.03 * Ws * Ws), (1.5, 3.0), (60, 200), 77)
    refs_ = synth._finish(synth._render_blobs(Ws, Ws, Xs, Ys, Ss, As), 2.0, 78, 8)
    fr_s = []
    for k in range(4):
        fld = synth.field_affine(0.0, 0.0, dudx=0.04 * k, dvdy=0.04 * k, xc=Ws / 2, yc=Ws / 2)
        uu, vv = fld(Xs, Ys)
        fr_s.append(synth._finish(synth._render_blobs(Ws, Ws, Xs + uu, Ys + vv, Ss, As), 2.0, 79 + k, 8))
    roi_s = np.zeros((Ws, Ws), np.uint8)
    roi_s[40:Ws - 40, 40:Ws - 40] = 1
    osec, (oo, orf) = _host_s(lambda: OSQ.correlate_sequence(refs_, fr_s, roi_s, seeds=[(96, 96, 0, 0)],
                                                            min_converged=0.9, min_zncc=0.999, **prm))
    emit({"row": "sequence", "workload": "%d^2 u8 speckle, %d frames, stretch +3 %% per frame in x and y, "
          "subset 21, step 4, affine, update below 90 %% converged or mean ZNCC 0.999" % (W, F),
          "ms": ms, "frames_per_s": F / (ms / 1e3), "references": refs, "converged_per_frame": conv,
          "converged_per_s": sum(conv) / (ms / 1e3),
          "cpu_oracle": {"kind": "oracle", "cores": 1, "sample": "192^2, 4 frames of +4 % stretch",
                         "converged_per_s": float(sum((o["status"] == 0).sum() for o in oo) / osec), "s": osec}})
    eng.close()
    print(json.dumps({"workload": "entry points beyond the single-pair path", "rows": rows,
                      "host": host_info(), "s_total": time.perf_counter() - t0}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=32, help="deformed frames per batched step (at most 32)")
    ap.add_argument("--latency-runs", type=int, default=60, help="plain single-frame calls for p50/p99")
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--fp32-reductions", action="store_true")
    ap.add_argument("--tps", type=int, default=0, help="threads per subset, batched form (0: autotuned)")
    ap.add_argument("--plain-tps", type=int, default=0, help="threads per subset, plain form (0: autotuned)")
    ap.add_argument("--tile", type=int, default=0, help="LDS window side, batched form (0: autotuned with --tps 0)")
    ap.add_argument("--plain-tile", type=int, default=0, help="LDS window side, plain form")
    ap.add_argument("--tune-size", type=int, default=0,
                    help="side of the autotuner's pair (0: the benchmark's own pair)")
    ap.add_argument("--cpu-crop", type=int, default=2048,
                    help="oracle window on the host's CPU share (0 = skip; the image side = the whole pair, which "
                         "also gives the accuracy fields)")
    ap.add_argument("--single-crop", type=int, default=512, help="oracle window on one core (0 = skip)")
    ap.add_argument("--no-fp32-variant", action="store_true",
                    help="skip timing the FP32-reduction variant beside the FP64-reduction default")
    ap.add_argument("--workload", default="2048", choices=["2048", "gigapixel", "serve", "precision", "extensions", "roofs"],
                    help="2048: the 2048^2 batched/plain benchmark; gigapixel: the 32768^2 pair, repeated; "
                         "serve: the serving mix")
    ap.add_argument("--precision-size", type=int, default=2048, help="precision: image side")
    ap.add_argument("--giga-tps", type=int, default=0,
                    help="gigapixel: threads per subset (0: time 128/256 threads x windows N+5/N+9 on the pair)")
    ap.add_argument("--giga-tile", type=int, default=0, help="gigapixel: LDS window side with --giga-tps")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of Poisson arrivals")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: requests per second")
    ap.add_argument("--max-active", type=int, default=48, help="serve: requests on the device at once")
    ap.add_argument("--budget-gb", type=float, default=230.0,
                    help="serve: library HBM budget (of the 288 GB; the rest holds the rendered frames and outputs)")
    ap.add_argument("--chunk", type=int, default=8, help="serve: launch steps per server call")
    ap.add_argument("--parity-samples", type=int, default=8, help="serve: requests checked against the oracle")
    ap.add_argument("--summarize-trace", metavar="DIR", help="write the kernel-trace summary of a rocprofv3 run")
    ap.add_argument("--summary-out", default=os.path.join(ROOT, "profiles", "k_wave_2048_kernel_trace.md"))
    ap.add_argument("--trace-log", metavar="LOG", help="--summarize-trace: the profiled run's output (its JSON line)")
    ap.add_argument("--summarize-sq-stalls", metavar="SQ",
                    help="write the wave-cycle breakdown of the batched k_wave from a rocprofv3 --pmc run")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("SQ", "TRACE"),
                    help="write the SQ instruction-counter summary from a rocprofv3 --pmc run and a kernel trace")
    ap.add_argument("--summarize-l2", nargs=3, metavar=("BENCH", "COPY", "TRACE"),
                    help="write the L2 counter summary from two rocprofv3 --pmc runs and a kernel trace")
    ap.add_argument("--summarize-ext-trace", metavar="DIR",
                    help="write the kernel-trace summary of a profiled --workload extensions run")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the HBM counter summary and per-launch traffic from four rocprofv3 --pmc runs")
    ap.add_argument("--no-probes", action="store_true", help="skip the achievable-rate probes in the roofline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.summary_out, args.trace_log)
        return
    if args.summarize_sq:
        summarize_sq(*args.summarize_sq, os.path.join(ROOT, "profiles", "k_wave_2048_sq_counters.md"))
        return
    if args.summarize_sq_stalls:
        summarize_sq_stalls(args.summarize_sq_stalls, os.path.join(ROOT, "profiles", "k_wave_2048_sq_stalls.md"))
        return
    if args.summarize_l2:
        summarize_l2(*args.summarize_l2, os.path.join(ROOT, "profiles", "k_wave_2048_l2_counters.md"))
        return
    if args.summarize_ext_trace:
        summarize_ext_trace(args.summarize_ext_trace, args.summary_out)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, os.path.join(ROOT, "profiles", "k_wave_2048_hbm_counters.md"),
                      os.path.join(ROOT, "profiles", "k_wave_2048_batched_traffic.json"))
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        serve(args)
        return
    if args.workload == "precision":
        precision(args)
        return
    if args.workload == "gigapixel":
        gigapixel(args)
        return
    if args.workload == "extensions":
        extensions(args)
        return
    if args.workload == "roofs":
        from paper_2601_12941_amd import roofs
        print(json.dumps({"workload": "achievable-rate probes (include/dic_roofs.h)", **roofs.measure(),
                          "published": {"hbm_GBps": PEAK_HBM_GBPS, "fp32_TFLOPs": PEAK_FP32_TFLOPS,
                                        "fp64_TFLOPs": 78.6}, "host": host_info()}))
        return

    import torch
    from paper_2601_12941_amd import dic, synth

    w = synth.workload("c2", size=args.size)
    t0 = time.perf_counter()
    ref, frames, roi = render_frames(w, args.batch)
    print("# inputs rendered in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)

    # ---- launch shapes: the autotuner times every candidate on a smaller pair of
    # the same workload (same field formula and speckle statistics)
    tuned = {}
    if args.tps == 0 or args.plain_tps == 0:
        from paper_2601_12941_amd import autotune
        if args.tune_size in (0, args.size):
            proxy = (ref, frames, roi, w.seeds)     # the benchmark's own pair
            pname = "the %d^2 workload itself" % args.size
        else:
            wt = synth.workload("c2", size=args.tune_size)
            tref, tframes, troi = render_frames(wt, args.batch)
            proxy = (tref, tframes, troi, wt.seeds)
            pname = "%d^2 pair of the 2048^2 workload recipe" % args.tune_size

        def log(msg):
            print("# " + msg, file=sys.stderr, flush=True)
        for form, b in (("batched", args.batch), ("plain", 1)):
            if (args.tps if form == "batched" else args.plain_tps) == 0:
                tuned[form] = autotune.choose(w.N, w.step, w.shape, reduce_fp64=not args.fp32_reductions, batch=b,
                                              seed_radius=w.seed_radius,
                                              proxy=proxy, proxy_name=pname, log=log, use_cache=False)
    tps_b = args.tps or tuned["batched"]["threads_per_subset"]
    tile_b = args.tile if args.tps else tuned["batched"]["tile_side"]
    tps_p = args.plain_tps or tuned["plain"]["threads_per_subset"]
    tile_p = args.plain_tile if args.plain_tps else tuned["plain"]["tile_side"]

    dev = torch.device("cuda", 0)
    d_ref = dic.to_device_image(ref)
    d_frames = [dic.to_device_image(f) for f in frames]
    d_roi = torch.from_numpy(roi).to(dev)
    eng = dic.Engine(0)
    prm = w.params()
    prm.update(reduce_fp64=not args.fp32_reductions, threads_per_subset=tps_b, tile_side=tile_b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.set_reference(d_ref, d_roi, **prm)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    peng = dic.Engine(0)
    peng.set_reference(d_ref, d_roi, **{**prm, "threads_per_subset": tps_p, "tile_side": tile_p})
    seeds = w.seeds

    # ---- batched steps
    for _ in range(args.warmup):
        eng.correlate_batch(d_frames, seeds)
    torch.cuda.synchronize()
    conv = 0
    iters = 0
    kern_ms = 0.0
    launches = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bout = eng.correlate_batch(d_frames, seeds)
        st = eng.stats()
        conv += st["converged"]
        iters += st["iterations"]
        kern_ms += st["ms_wave_kernels"]
        launches += st["wave_launches"]
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    last = eng.stats()
    value = conv / t_batch
    batched_frame0 = {k: v.cpu().numpy() for k, v in bout[0].items()}
    del bout

    # ---- plain single-frame calls: throughput and pair latency
    def plain_runs(engine, runs):
        engine.correlate(d_frames[0], seeds)
        torch.cuda.synchronize()
        lat, pc, first = [], 0, None
        for i in range(runs):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            out = engine.correlate(d_frames[i % len(d_frames)], seeds)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
            pc += engine.stats()["converged"]
            if i == 0:
                first = {k: v.cpu().numpy() for k, v in out.items()}
        return pc / sum(lat), np.array(lat) * 1e3, first
    plain_rate, lat_ms, plain_frame0 = plain_runs(peng, args.latency_runs)

    # ---- the FP32-reduction variant of both forms, same launch shapes
    fp32 = None
    if not args.no_fp32_variant and not args.fp32_reductions:
        veng = dic.Engine(0)
        veng.set_reference(d_ref, d_roi, **{**prm, "reduce_fp64": False})
        vpeng = dic.Engine(0)
        vpeng.set_reference(d_ref, d_roi, **{**prm, "reduce_fp64": False, "threads_per_subset": tps_p,
                                              "tile_side": tile_p})
        veng.correlate_batch(d_frames, seeds)
        torch.cuda.synchronize()
        vsteps = max(1, min(args.steps, 5))
        vconv = 0
        t0 = time.perf_counter()
        for _ in range(vsteps):
            vout = veng.correlate_batch(d_frames, seeds)
            vconv += veng.stats()["converged"]
        torch.cuda.synchronize()
        vt = time.perf_counter() - t0
        v_frame0 = {k: v.cpu().numpy() for k, v in vout[0].items()}
        del vout
        vrate, vlat, vplain0 = plain_runs(vpeng, max(20, args.latency_runs // 3))
        fp32 = {"batched": {"value": vconv / vt, "unit": "converged subsets/s", "steps": vsteps,
                            "ms_per_step": vt / vsteps * 1e3},
                "plain": {"value": vrate, "unit": "converged subsets/s",
                          "latency_ms_p50": float(np.percentile(vlat, 50)),
                          "latency_ms_p99": float(np.percentile(vlat, 99)), "runs": len(vlat)},
                "_frames": (v_frame0, vplain0)}
        veng.close()
        vpeng.close()

    # ---- roofline of the IC-GN wave kernel (plain FP32 VALU arithmetic)
    N = w.N
    flops = FLOP_PER_PX_IT[w.shape] * N * N * iters
    avg_launch_ms = kern_ms / max(1, launches)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    # the committed counters describe the profiled launch shape only
    profiled = (args.batch == 32 and args.size == 2048 and last["threads_per_subset"] == PROFILE_SHAPES["tps"]
                and tile_b == PROFILE_SHAPES["tile"] and not args.fp32_reductions)
    traffic = profiled_traffic() if profiled else None
    roofline = {"bound": "alu", "kernel": "k_wave (IC-GN frontier wave)", "achieved": achieved,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": traffic,
                "flop_per_px_iter": FLOP_PER_PX_IT[w.shape], "avg_launch_us": avg_launch_ms * 1e3,
                "launches_per_step": launches / args.steps,
                "subsets_per_launch": conv / max(1, launches),
                "launch_chains": last["launch_chains"],
                "launch": "one wave step: the launches of every launch chain for one wave index, which run side "
                          "by side on their streams; avg_launch_us is the duration of a wave step"}
    # achievable denominators measured on this GPU beside the published peaks: FP32 FMA
    # issue as the library is built (no packed FP32) and HBM streaming reads
    if not args.no_probes:
        from paper_2601_12941_amd import roofs
        fma32 = roofs.fma(False)
        hbm = roofs.hbm_read()
        roofline["achievable"] = {"fma_f32_TFLOPs": fma32, "hbm_read_GBps": hbm,
                                  "probe": "dic_roof_fma / dic_roof_hbm_read (include/dic_roofs.h)"}
        roofline["frac_of_achievable"] = achieved / fma32
    if traffic:
        # the same launch against the HBM roof: counted bytes over the live launch time,
        # and the counted bytes over the compulsory ones (each frame's deformed image and
        # coefficients once, the reference arrays once per launch)
        gbps = traffic / (avg_launch_ms * 1e-3) / 1e9
        roofline["traffic_gbps"] = gbps
        roofline["traffic_frac_of_hbm"] = gbps / PEAK_HBM_GBPS
        roofline["traffic_bytes_per_subset"] = traffic / max(1.0, conv / max(1, launches))
        if "achievable" in roofline:
            roofline["traffic_frac_of_achievable_hbm"] = gbps / roofline["achievable"]["hbm_read_GBps"]

    cpu = None
    acc = None
    if args.cpu_crop > 0:
        cpu, o = cpu_baseline(ref, frames[0], roi, w, min(args.cpu_crop, args.size), args.single_crop)
        if min(args.cpu_crop, args.size) == args.size:
            from paper_2601_12941_amd import synth
            u, v, _ = synth.truth_at_nodes(w.field(), w.W, w.H, w.N, w.step)
            acc = {"batched_frame0": accuracy(batched_frame0, o, w, (u, v)),
                   "plain_frame0": accuracy(plain_frame0, o, w, (u, v)),
                   "oracle_vs_truth": accuracy(
                       {"p": o["p"], "zncc": o["zncc"], "status": o["status"], "wave": o["wave"]}, o, w,
                       (u, v))["vs_truth"]}
            if fp32 is not None:
                fb, fpl = fp32["_frames"]
                fp32["accuracy"] = {"batched_frame0": accuracy(fb, o, w, (u, v)),
                                    "plain_frame0": accuracy(fpl, o, w, (u, v))}
    if fp32 is not None:
        fp32.pop("_frames")

    rec = {
        "metric": "converged subsets/s at 2048^2 (batched vs plain, same GPU); p50/p99 pair latency",
        "value": value,
        "unit": "converged subsets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fp32_reductions else "f32 (f64 reductions and solve)",
        "data": "synthetic",
        "config": {"workload": "2048x2048 u16 12-bit speckle, sinusoidal u (lambda 10..300 px), subset 31, step 2, "
                               "affine, batched %d frames per step" % args.batch,
                   "size": args.size, "subset": N, "step": w.step, "nodes": last["nodes"], "active": last["active"],
                   "frames_per_step": args.batch, "threads_per_subset": last["threads_per_subset"],
                   "tile_side": tile_b},
        "plain": {"value": plain_rate, "unit": "converged subsets/s", "latency_ms_p50": float(np.percentile(lat_ms, 50)),
                  "latency_ms_p99": float(np.percentile(lat_ms, 99)), "runs": args.latency_runs,
                  "threads_per_subset": tps_p, "tile_side": tile_p},
        "batched_over_plain": value / plain_rate,
        "waves_per_frame": last["waves"],
        "iterations_per_subset": iters / max(1, conv),
        "converged_per_frame": last["converged"] / max(1, last["frames"]),
        "set_reference_ms": t_ref * 1e3,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": acc,
        "fp32_reductions": fp32,
        "autotune": {k: {"threads_per_subset": v["threads_per_subset"], "tile_side": v["tile_side"],
                         "proxy": v["proxy"],
                         "candidates": [[r["threads_per_subset"], r["tile_side"], round(r["rate"] / 1e6, 2)]
                                        for r in v["table"]]} for k, v in tuned.items()},
    }
    print(json.dumps(rec))
    eng.close()
    peng.close()


if __name__ == "__main__":
    main()
