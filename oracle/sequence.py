"""FP64 reference of multi-frame correlation with reference updating (paper
Sec. 6: an automated reference-updating scheme, in which the reference moves
through the sequence of deformed images to follow large strains).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library's own
path.  Plain numpy over the oracle's own correlation (dic_oracle.c); it shares
no code with the GPU path.

Readings (the paper names the scheme and cites Pan et al. 2012):
  * quality of a frame's correlation against the current reference: the
    fraction of active nodes CONVERGED and the mean ZNCC over them; when either
    is below its threshold and the previous frame is not already the
    reference, the previous frame becomes the reference (same grid, ROI mask
    and parameters) and the frame is correlated again against it;
  * seeds: the user's seed positions; the guess is the user's (u0, v0) for the
    first frame against the original reference, (0, 0) for the first frame
    against an updated reference, and otherwise the previous frame's
    incremental displacement at the seed's node (the nearest active node)
    when that node converged;
  * every frame's result is expressed on the original reference's nodes
    (Lagrangian): with the current reference's accumulated displacement u_r
    and gradient G_r = [[p2, p3], [p4, p5]] at node X, the node sits at
    x = X + u_r(X) in the current reference; the incremental result is
    interpolated bilinearly at x over its node grid (only terms of non-zero
    weight), u = u_r + u_inc(x), and G = G_inc + G_r + G_inc G_r (the
    composition (I + G_inc)(I + G_r) - I); the ZNCC is interpolated the same
    way, iterations and wave index are those of the nearest node;
  * status: NOT_REACHED where the reference state is not CONVERGED or x falls
    outside the node grid; else the first non-CONVERGED status among the
    weighted nodes (order (i0, j0), (i0+1, j0), (i0, j0+1), (i0+1, j0+1)), or
    CONVERGED;
  * rigid and affine shapes (quadratic terms are not composed).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

CONVERGED, NOT_REACHED = 0, 1


def accumulate(ref_state, inc, N, step, npar):
    """Result of a frame on the original nodes from the current reference's
    accumulated state (None: the original reference) and the frame's
    incremental result against it.  Dicts of p [12][ny][nx], zncc, iters,
    status, wave (oracle.correlate's layout)."""
    ny, nx = inc["status"].shape
    h = (N - 1) // 2
    out = dict(p=np.zeros_like(inc["p"]), zncc=np.zeros((ny, nx)), iters=np.zeros((ny, nx), np.int32),
               status=np.full((ny, nx), NOT_REACHED, np.int32), wave=np.full((ny, nx), -1, np.int32))
    for j in range(ny):
        for i in range(nx):
            if ref_state is None:
                ur = vr = 0.0
                Gr = np.zeros((2, 2))
                if inc["status"][j, i] == 2:          # outside the ROI on the original grid
                    out["status"][j, i] = 2
                    continue
            else:
                if ref_state["status"][j, i] != CONVERGED:
                    out["status"][j, i] = 2 if ref_state["status"][j, i] == 2 else NOT_REACHED
                    continue
                ur, vr = ref_state["p"][0, j, i], ref_state["p"][1, j, i]
                Gr = np.array([[ref_state["p"][2, j, i], ref_state["p"][3, j, i]],
                               [ref_state["p"][4, j, i], ref_state["p"][5, j, i]]]) if npar >= 6 else np.zeros((2, 2))
            x = h + i * step + ur
            y = h + j * step + vr
            fx, fy = (x - h) / step, (y - h) / step
            i0, j0 = math.floor(fx), math.floor(fy)
            ax, ay = fx - i0, fy - j0
            # the cell's far column / row is needed only where it carries weight
            if i0 < 0 or j0 < 0 or i0 > nx - 1 or j0 > ny - 1 or (ax > 0 and i0 + 1 > nx - 1) or \
                    (ay > 0 and j0 + 1 > ny - 1):
                continue
            terms = [(j0, i0, (1 - ax) * (1 - ay)), (j0, i0 + 1, ax * (1 - ay)), (j0 + 1, i0, (1 - ax) * ay),
                     (j0 + 1, i0 + 1, ax * ay)]
            terms = [(jj, ii, wgt) for jj, ii, wgt in terms if wgt > 0.0]
            st = CONVERGED
            for jj, ii, _ in terms:
                if inc["status"][jj, ii] != CONVERGED:
                    st = int(inc["status"][jj, ii])
                    break

            def interp(a):
                return sum(wgt * a[jj, ii] for jj, ii, wgt in terms)
            ui, vi = interp(inc["p"][0]), interp(inc["p"][1])
            out["p"][0, j, i] = ur + ui
            out["p"][1, j, i] = vr + vi
            if npar >= 6:
                Gi = np.array([[interp(inc["p"][2]), interp(inc["p"][3])], [interp(inc["p"][4]), interp(inc["p"][5])]])
                G = Gi + Gr + Gi @ Gr
                out["p"][2, j, i], out["p"][3, j, i] = G[0, 0], G[0, 1]
                out["p"][4, j, i], out["p"][5, j, i] = G[1, 0], G[1, 1]
            out["zncc"][j, i] = interp(inc["zncc"])
            ri = min(max(int(math.floor(fx + 0.5)), 0), nx - 1)
            rj = min(max(int(math.floor(fy + 0.5)), 0), ny - 1)
            out["iters"][j, i] = inc["iters"][rj, ri]
            out["wave"][j, i] = inc["wave"][rj, ri]
            out["status"][j, i] = st
    return out


def snap(x, y, status, N, step):
    """Nearest active node to (x, y) (Euclidean; ties to smaller y, then x), as (j, i)."""
    h = (N - 1) // 2
    ny, nx = status.shape
    X, Y = np.meshgrid(h + step * np.arange(nx, dtype=float), h + step * np.arange(ny, dtype=float))
    d = (X - x) ** 2 + (Y - y) ** 2
    d[status == 2] = np.inf
    k = int(np.argmin(d))           # first minimum in row-major order: smaller y, then x
    return k // nx, k % nx


def quality(res):
    """(fraction of active nodes CONVERGED, mean ZNCC over them)."""
    act = res["status"] != 2
    conv = res["status"] == CONVERGED
    frac = conv.sum() / max(1, act.sum())
    return frac, (res["zncc"][conv].mean() if conv.any() else 0.0)


def correlate_sequence(ref, frames, roi, *, seeds, min_converged=0.95, min_zncc=0.9, update=True, threads=1,
                       **params):
    """Every frame on the original nodes; returns (results, reference index of
    each frame: -1 = the original reference)."""
    N, step, npar = params["subset_size"], params["step"], params.get("shape", 6)
    cur_img, cur = ref, -1
    state = None
    prev_inc = None
    results, refs = [], []
    for t, fr in enumerate(frames):
        def run(guess_from_prev):
            sd = []
            for (x, y, u0, v0) in seeds:
                gu, gv = (u0, v0) if cur == -1 and t == 0 else (0.0, 0.0)
                if guess_from_prev and prev_inc is not None:
                    j, i = snap(x, y, prev_inc["status"], N, step)
                    if prev_inc["status"][j, i] == CONVERGED:
                        gu, gv = prev_inc["p"][0, j, i], prev_inc["p"][1, j, i]
                sd.append((x, y, gu, gv))
            return oracle.correlate(cur_img, fr, roi, seeds=sd, threads=threads, **params)
        inc = run(True)
        frac, mz = quality(inc)
        if update and (frac < min_converged or mz < min_zncc) and t >= 1 and cur != t - 1:
            cur_img, cur = frames[t - 1], t - 1
            state = results[t - 1]
            prev_inc = None
            inc = run(False)
        results.append(accumulate(state, inc, N, step, npar))
        refs.append(cur)
        prev_inc = inc
    return results, refs
