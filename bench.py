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
their own launch shapes (threads per subset: 64 for the batched form, which
is throughput-bound; 128 for the plain form, which is latency-bound).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOP_PER_PX_IT = {6: 91.0, 12: 115.0}   # algorithmic flops per subset pixel per IC-GN iteration
PEAK_FP32_TFLOPS = 157.3                  # MI355X published FP32 vector peak


def render_frames(w, nframes):
    """Reference plus `nframes` deformed frames that differ only in their noise."""
    from paper_2601_12941_amd import synth
    X, Y, S, A = synth.draw_blobs(w.W, w.H, w.nblobs, w.sigma, w.amp, w.seed_blobs)
    ref_clean = synth._render_blobs(w.W, w.H, X, Y, S, A)
    f = w.field()
    u, v = f(X, Y)
    def_clean = synth._render_blobs(w.W, w.H, X + u, Y + v, S, A)
    ref = synth._finish(ref_clean, w.noise, w.seed_noise_ref, w.bits)
    frames = [synth._finish(def_clean, w.noise, w.seed_noise_def + i, w.bits) for i in range(nframes)]
    roi = synth.roi_from_field(w.W, w.H, f)
    return ref, frames, roi


def cpu_baseline(ref, deformed, roi, w, crop):
    """The FP64 oracle on the central crop x crop window of the same pair."""
    import oracle
    H, W = ref.shape
    y0, x0 = (H - crop) // 2, (W - crop) // 2
    sl = (slice(y0, y0 + crop), slice(x0, x0 + crop))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    prm = w.params()
    t0 = time.perf_counter()
    r = oracle.correlate(ref[sl], deformed[sl], roi[sl], seeds=[(crop / 2, crop / 2, 0, 0)], threads=threads, **prm)
    dt = time.perf_counter() - t0
    conv = int((r["status"] == 0).sum())
    return {"value": conv / dt, "unit": "converged subsets/s", "cores": threads, "kind": "oracle",
            "sample": "central %dx%d window of the same pair (%d converged subsets in %.1f s, WAVE order, "
                      "OpenMP over the nodes of each wave)" % (crop, crop, conv, dt)}


def profiled_traffic():
    """HBM bytes per batched k_wave launch from the committed FETCH_SIZE / WRITE_SIZE
    counter runs, if they were taken on the kernel source that is built now."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "k_wave_2048_batched_traffic.json")
    src = os.path.join(ROOT, "paper_2601_12941_amd", "csrc", "dic_kernels.hip")
    try:
        rec = json.load(open(rec_path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    return rec["traffic_bytes_per_launch"] if rec.get("source_sha256") == sha else None


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
    t0 = time.perf_counter()
    eng.set_reference(d_ref, d_roi, **w.params())
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
           "threads_per_subset": st["threads_per_subset"], "repeats": repeats,
           "latency_ms_p50": float(np.percentile(lat_ms, 50)), "latency_ms_p99": float(np.percentile(lat_ms, 99)),
           "converged_subsets_per_s": float(conv.sum() / np.median(lat)), "set_reference_ms": t_ref * 1e3,
           "render_s": t_render, "sampled_parity": {"nodes": used, "max_duv_px": float(max(errs)) if errs else None,
                                                     "max_dzncc": float(max(dz)) if dz else None},
           "error_vs_truth_px": {"rms": float(np.sqrt((err_truth ** 2).mean())), "max": float(err_truth.max())},
           "library_device_memory_gb": (free0 - free1) / 1e9,
           "input_device_memory_gb": (pair.ref.nbytes + pair.deformed.nbytes + pair.roi.nbytes) / 1e9}
    print(json.dumps(rec))
    eng.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16, help="deformed frames per batched step")
    ap.add_argument("--latency-runs", type=int, default=30, help="plain single-frame calls for p50/p99")
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--fp32-reductions", action="store_true")
    ap.add_argument("--tps", type=int, default=64, help="threads per subset, batched form")
    ap.add_argument("--plain-tps", type=int, default=128, help="threads per subset, plain form")
    ap.add_argument("--cpu-crop", type=int, default=2048, help="oracle sample window (0 = skip)")
    ap.add_argument("--workload", default="2048", choices=["2048", "gigapixel"],
                    help="2048: the 2048^2 batched/plain benchmark; gigapixel: the 32768^2 pair, repeated")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "gigapixel":
        gigapixel(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_12941_amd import dic, synth

    w = synth.workload("c2", size=args.size)
    t0 = time.perf_counter()
    ref, frames, roi = render_frames(w, args.batch)
    print("# inputs rendered in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    d_ref = dic.to_device_image(ref)
    d_frames = [dic.to_device_image(f) for f in frames]
    d_roi = torch.from_numpy(roi).to(dev)
    eng = dic.Engine(0)
    prm = w.params()
    prm.update(reduce_fp64=not args.fp32_reductions, threads_per_subset=args.tps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.set_reference(d_ref, d_roi, **prm)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    peng = dic.Engine(0)
    peng.set_reference(d_ref, d_roi, **{**prm, "threads_per_subset": args.plain_tps})
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
        eng.correlate_batch(d_frames, seeds)
        st = eng.stats()
        conv += st["converged"]
        iters += st["iterations"]
        kern_ms += st["ms_wave_kernels"]
        launches += st["wave_launches"]
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    last = eng.stats()
    value = conv / t_batch

    # ---- plain single-frame calls: throughput and pair latency
    peng.correlate(d_frames[0], seeds)
    torch.cuda.synchronize()
    lat = []
    pconv = 0
    for i in range(args.latency_runs):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        peng.correlate(d_frames[i % len(d_frames)], seeds)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
        pconv += peng.stats()["converged"]
    plain_rate = pconv / sum(lat)
    lat_ms = np.array(lat) * 1e3

    # ---- roofline of the IC-GN wave kernel (plain FP32 VALU arithmetic)
    N = w.N
    flops = FLOP_PER_PX_IT[w.shape] * N * N * iters
    avg_launch_ms = kern_ms / max(1, launches)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_wave (IC-GN frontier wave)", "achieved": achieved,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": profiled_traffic() if args.batch == 16 and args.size == 2048 else None,
                "flop_per_px_iter": FLOP_PER_PX_IT[w.shape], "avg_launch_us": avg_launch_ms * 1e3,
                "launches_per_step": launches / args.steps}

    cpu = None
    if args.cpu_crop > 0:
        cpu = cpu_baseline(ref, frames[0], roi, w, min(args.cpu_crop, args.size))

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
                   "frames_per_step": args.batch, "threads_per_subset": last["threads_per_subset"]},
        "plain": {"value": plain_rate, "unit": "converged subsets/s", "latency_ms_p50": float(np.percentile(lat_ms, 50)),
                  "latency_ms_p99": float(np.percentile(lat_ms, 99)), "runs": args.latency_runs,
                  "threads_per_subset": args.plain_tps},
        "batched_over_plain": value / plain_rate,
        "waves_per_frame": last["waves"],
        "iterations_per_subset": iters / max(1, conv),
        "converged_per_frame": last["converged"] / max(1, last["frames"]),
        "set_reference_ms": t_ref * 1e3,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))
    eng.close()
    peng.close()


if __name__ == "__main__":
    main()
