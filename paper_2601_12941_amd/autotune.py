"""Launch-shape autotuner: picks the subset-to-wavefront mapping (threads per
subset) and the LDS window side for a parameter set by timing the library on a
synthetic speckle pair of the same subset size, step and shape.

Every candidate runs through the same C ABI as production calls; the choice
with the highest converged-subsets rate wins.  Results are cached in a JSON
file keyed by device name and parameters (DIC_AUTOTUNE_CACHE, default
autotune_cache.json next to this module).
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, List, Optional

from . import dic, synth

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.environ.get("DIC_AUTOTUNE_CACHE", os.path.join(_HERE, "autotune_cache.json"))


def default_tile(N: int) -> int:
    return N + 9


def candidates(N: int, shape: int = 6):
    """(threads per subset, tile side) pairs worth timing for subset size N: the
    smallest window (1 sample of drift room per side), the library default (3) and
    a roomy one (7)."""
    tiles = sorted({t for t in (N + 5, default_tile(N), N + 17) if N + 5 <= t <= 96})
    out = []
    for tps in (16, 32, 64, 128, 256):
        if tps < 64 and (shape != 6 or N > 16):
            continue   # packed subsets: affine, N <= 16
        if tps < N:
            continue
        for ts in tiles:
            out.append((tps, ts))
    return out


def proxy_pair(N: int, step: int, size: int, frames: int, seed: int = 9001):
    """A u8 speckle reference and `frames` deformed frames under a mild affine
    field (translation about 1.3 px, gradients of a few 1e-3), with the
    density, blob sizes and noise of the 512^2 workload."""
    W = size
    field = synth.field_affine(1.3, -0.7, 0.004, 0.002, -0.003, 0.005, xc=W / 2.0, yc=W / 2.0)
    nblobs = int(round(synth.SERVE_DENSITY * W * W))
    X, Y, S, A = synth.draw_blobs(W, W, nblobs, (2.0, 4.0), (60.0, 200.0), seed)
    render = synth._render_blobs_large if W * W > synth._LARGE // 4 else synth._render_blobs
    ref = synth._finish(render(W, W, X, Y, S, A), 2.0, seed + 1, 8)
    u, v = field(X, Y)
    de = render(W, W, X + u, Y + v, S, A)
    defs = [synth._finish(de, 2.0, seed + 2 + f, 8) for f in range(frames)]
    roi = synth.roi_from_field(W, W, field, 8)
    return ref, defs, roi


def _key(N, step, shape, coef_fp16, reduce_fp64, batch, device_name):
    return "%s|N%d|s%d|np%d|h%d|f64%d|b%d" % (device_name, N, step, shape, int(coef_fp16), int(reduce_fp64), batch)


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    tmp = CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def choose(N: int, step: int, shape: int = 6, coef_fp16: bool = False, reduce_fp64: bool = True, batch: int = 1,
           seed_radius: int = 8, size: int = 1024, reps: int = 3, use_cache: bool = True,
           log: Optional[Callable[[str], None]] = None, proxy=None, proxy_name: Optional[str] = None) -> Dict:
    """Best (threads_per_subset, tile_side) for the parameter set, timed with
    `batch` frames per call (1 = the plain form).  `proxy` = (reference,
    [deformed frames], roi, seeds) replaces the default affine speckle pair.
    Returns the choice, its rate and every candidate's rate."""
    import torch
    name = torch.cuda.get_device_name(0)
    key = _key(N, step, shape, coef_fp16, reduce_fp64, batch, name) + ("|" + proxy_name if proxy_name else "")
    if use_cache:
        hit = _load().get(key)
        if hit:
            return dict(hit, cached=True)
    if proxy is None:
        ref, defs, roi = proxy_pair(N, step, size, batch)
        seeds = [(size / 2.0, size / 2.0, 0.0, 0.0)]
        desc = "%d^2 u8 speckle, affine field, %d frame(s)" % (size, batch)
    else:
        ref, defs, roi, seeds = proxy
        defs = defs[:batch]
        desc = proxy_name or "caller's pair"
    d_ref = dic.to_device_image(ref)
    d_defs = [dic.to_device_image(d) for d in defs]
    d_roi = torch.from_numpy(roi).cuda()
    table: List[Dict] = []
    eng = dic.Engine(0)
    try:
        for tps, ts in candidates(N, shape):
            try:
                eng.set_reference(d_ref, d_roi, subset_size=N, step=step, shape=shape, coef_fp16=coef_fp16,
                                  reduce_fp64=reduce_fp64, threads_per_subset=tps, tile_side=ts, seed_radius=seed_radius)
            except dic.DicError:
                continue
            run = (lambda: eng.correlate(d_defs[0], seeds)) if batch == 1 else \
                (lambda: eng.correlate_batch(d_defs, seeds))
            run()
            torch.cuda.synchronize()
            t = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                run()
                torch.cuda.synchronize()
                t.append(time.perf_counter() - t0)
            conv = eng.stats()["converged"]
            rate = conv / min(t)
            table.append(dict(threads_per_subset=tps, tile_side=ts, rate=rate, ms=min(t) * 1e3))
            if log:
                log("autotune N%d s%d b%d: %d threads, tile %d -> %.1fM subsets/s" % (N, step, batch, tps, ts,
                                                                                        rate / 1e6))
    finally:
        eng.close()
    if not table:
        raise RuntimeError("no launch shape is supported for subset %d" % N)
    best = max(table, key=lambda r: r["rate"])
    out = dict(threads_per_subset=best["threads_per_subset"], tile_side=best["tile_side"], rate=best["rate"],
               proxy=desc, table=table)
    if use_cache:
        d = _load()
        d[key] = out
        _store(d)
    return dict(out, cached=False)
