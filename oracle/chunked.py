"""FP64 reference of out-of-core correlation (paper Sec. 6: the images are
partitioned into chunks that are loaded one at a time, so that a pair larger
than the available memory can still be correlated).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library's own
path.  Plain numpy over the oracle's own correlation (dic_oracle.c); it shares
no code with the GPU path.

The paper names the partitioning but not its rules; the reading taken here:
  * the node grid of the whole pair (subset N, step s) is cut into bands of
    `band_rows` node rows; band b covers node rows [b*band_rows, ...);
  * a band's window is the pixel rows its subsets cover, widened by `halo`
    rows on both sides (clipped to the image) with its top moved down to a
    multiple of s, so that the window's node grid is a part of the whole
    grid; the ROI inside the window is the given one restricted to the band's
    own pixel rows, so the window's active nodes are exactly the band's;
  * each window pair is correlated as a pair of its own (its own spline
    prefilter, bounds and propagation); the band's node rows are copied out;
  * the first band is the one holding the node row nearest to the first seed;
    then the bands below it in order, then the bands above it in order;
  * a band's seeds are the given seeds whose nearest node row is in the band
    and, for all but the first band, seeds on the band's node row next to the
    finished neighbour: of the neighbour's CONVERGED nodes across the
    boundary (columns c_0 < c_1 < ... < c_{n-1}), k = min(boundary_seeds, n)
    are taken, the q-th at c[floor(q n / k) + floor(n / (2k))], each guessed
    with that node's (u, v);
  * then a second sweep back toward the first band (from the last band
    upward to the one after the first, and from the top band downward to the
    one before it): a band with no CONVERGED node is correlated again from
    its given seeds and its other neighbour's boundary row (a band behind an
    ROI gap, reached only from a seed further out);
  * a band without a usable seed keeps its active nodes NOT_REACHED.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

CONVERGED, NOT_REACHED, NOT_IN_ROI = 0, 1, 2


def _nearest_row(y, h, step, ny):
    r = (y - h) / step
    if r <= 0.0:
        return 0
    if r >= ny - 1:
        return ny - 1
    return int(math.floor(r + 0.5))


def correlate_chunked(ref, deformed, roi=None, *, seeds, band_rows, halo, boundary_seeds=8, threads=1, **params):
    """Whole-grid result (oracle.correlate's layout) from band-by-band
    correlation of window pairs."""
    ref = np.asarray(ref)
    deformed = np.asarray(deformed)
    H, W = ref.shape
    N, s = params["subset_size"], params["step"]
    h = (N - 1) // 2
    nx, ny = (W - N) // s + 1, (H - N) // s + 1
    roi_full = np.ones((H, W), np.uint8) if roi is None else (np.asarray(roi) != 0).astype(np.uint8)
    out = dict(p=np.zeros((12, ny, nx)), zncc=np.zeros((ny, nx)), iters=np.zeros((ny, nx), np.int32),
               status=np.full((ny, nx), NOT_IN_ROI, np.int32), wave=np.full((ny, nx), -1, np.int32),
               subset_size=N, step=s)
    seeds = [tuple(float(a) for a in sd) + (0.0,) * (4 - len(sd)) for sd in seeds]
    nbands = -(-ny // band_rows)
    b0 = _nearest_row(seeds[0][1], h, s, ny) // band_rows

    def run_band(b, side):
        """Correlate band b from its given seeds and, when side is 'above' or
        'below', from the converged nodes across that boundary."""
        j0, j1 = b * band_rows, min(ny, (b + 1) * band_rows)
        y_top, y_bot = j0 * s, (j1 - 1) * s + N - 1
        ya = (max(0, y_top - halo) // s) * s
        yb = min(H - 1, y_bot + halo)
        jw = ya // s                                     # window node row k is grid row jw + k
        win_roi = np.zeros((yb - ya + 1, W), np.uint8)
        win_roi[y_top - ya:y_bot - ya + 1] = roi_full[y_top:y_bot + 1]
        # the band's active nodes: every subset pixel inside the ROI
        for j in range(j0, j1):
            for i in range(nx):
                if roi_full[j * s:j * s + N, i * s:i * s + N].all():
                    out["status"][j, i] = NOT_REACHED
        sd = [(x, y - ya, u0, v0) for (x, y, u0, v0) in seeds if j0 <= _nearest_row(y, h, s, ny) < j1]
        if side is not None:
            jr, jn = (j0, j0 - 1) if side == "above" else (j1 - 1, j1)
            cols = [i for i in range(nx) if out["status"][jn, i] == CONVERGED]
            n = len(cols)
            k = min(boundary_seeds, n)
            for q in range(k):
                i = cols[(q * n) // k + n // (2 * k)]
                sd.append((float(h + i * s), float(h + jr * s - ya), float(out["p"][0, jn, i]),
                           float(out["p"][1, jn, i])))
        if not sd:
            return
        try:
            r = oracle.correlate(ref[ya:yb + 1], deformed[ya:yb + 1], win_roi, seeds=sd, threads=threads, **params)
        except ValueError:                               # no seed on an active node of the band
            return
        for key in ("zncc", "iters", "status", "wave"):
            out[key][j0:j1] = r[key][j0 - jw:j1 - jw]
        out["p"][:, j0:j1] = r["p"][:, j0 - jw:j1 - jw]

    def converged(b):
        return bool((out["status"][b * band_rows:(b + 1) * band_rows] == CONVERGED).any())

    # first sweep: outward from the first seed's band
    run_band(b0, None)
    for b in range(b0 + 1, nbands):
        run_band(b, "above")
    for b in range(b0 - 1, -1, -1):
        run_band(b, "below")
    # second sweep, back toward the first band: bands still without a converged
    # node, seeded across their other boundary
    for b in range(nbands - 2, b0, -1):
        if not converged(b):
            run_band(b, "below")
    for b in range(1, b0):
        if not converged(b):
            run_band(b, "above")
    out["u"], out["v"] = out["p"][0], out["p"][1]
    return out
