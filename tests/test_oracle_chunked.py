"""Pins of the out-of-core (band-by-band) oracle (paper Sec. 6, images
partitioned into chunks): one band covering the grid is exactly the whole-pair
correlation; with many bands and a halo covering the motion every converged
node agrees with the whole-pair correlation to well within the convergence
threshold's reach, in both propagation directions; without a halo the
subsets whose warped pixels leave their band's window are exactly the ones
marked OUT_OF_BOUNDS; given seeds reach bands that no boundary can."""
import numpy as np
import pytest

import oracle
from oracle import ST
from oracle import chunked as CH
from paper_2601_12941_amd import synth

PRM = dict(subset_size=21, step=4, seed_radius=4, tol=1e-4)


def _pair(field, W=200, H=232, seed=31):
    return synth.make_pair(W, H, int(0.03 * W * H), (1.5, 3.0), (60, 200), field, 2.0, 8, seed, seed + 1, seed + 2)


def _converged_agree(c, f, tol=1e-3):
    both = (c["status"] == ST["CONVERGED"]) & (f["status"] == ST["CONVERGED"])
    act = f["status"] != ST["NOT_IN_ROI"]
    h = (PRM["subset_size"] - 1) / 2
    d = np.max(np.abs(c["p"][:6] - f["p"][:6])[:, both] * np.array([1, 1, h, h, h, h])[:, None], axis=0)
    return both.sum() / act.sum(), float(d.max())


def test_one_band_is_the_whole_pair():
    pair = _pair(synth.field_affine(1.3, -2.2, 0.01, 0.0, 0.0, -0.008, 100, 116))
    seeds = [(100, 116, 1, -2)]
    full = oracle.correlate(pair.ref, pair.deformed, pair.roi, seeds=seeds, threads=8, **PRM)
    ny = full["status"].shape[0]
    c = CH.correlate_chunked(pair.ref, pair.deformed, pair.roi, seeds=seeds, band_rows=ny, halo=300, threads=8,
                             **PRM)
    for k in ("p", "zncc", "iters", "status", "wave"):
        assert np.array_equal(c[k], full[k]), k


@pytest.mark.parametrize("seed_y", [20, 116, 210])
def test_bands_agree_with_the_whole_pair(seed_y):
    # vertical motion up to ~2.5 px; halo 12 rows covers it and the spline's reach;
    # seeds at the top, middle and bottom: bands run downward, both ways, upward
    pair = _pair(synth.field_affine(0.8, 1.2, 0.006, 0.002, -0.004, 0.01, 100, 116))
    seeds = [(100, seed_y, 1, 1)]
    full = oracle.correlate(pair.ref, pair.deformed, pair.roi, seeds=seeds, threads=8, **PRM)
    c = CH.correlate_chunked(pair.ref, pair.deformed, pair.roi, seeds=seeds, band_rows=7, halo=12,
                             boundary_seeds=4, threads=8, **PRM)
    assert np.array_equal(c["status"] == ST["NOT_IN_ROI"], full["status"] == ST["NOT_IN_ROI"])
    frac, dmax = _converged_agree(c, full)
    print("bands vs whole pair:", frac, dmax)
    assert frac > 0.99
    # both stop within |dp| < tol of the same fixed point, from different guesses
    assert dmax < 2e-3
    # the wave index restarts in each band: it is smaller than in one pass somewhere
    both = (c["status"] == 0) & (full["status"] == 0)
    assert (c["wave"][both] < full["wave"][both]).any()


def test_without_halo_the_band_edges_leave_the_window():
    # a downward translation of 3 px: with no halo a band's last node row reads
    # 3 rows past its window (OUT_OF_BOUNDS) unless the window ends at the image's
    # edge, and no boundary seed crosses it, so every band gets a seed of its own;
    # every other node matches the whole pair
    pair = _pair(synth.field_affine(0.0, 3.0))
    br, h, s = 6, 10, 4
    full = oracle.correlate(pair.ref, pair.deformed, pair.roi, seeds=[(100, 30, 0, 3)], threads=8, **PRM)
    ny = full["status"].shape[0]
    seeds = [(100, h + s * (br * b + 2), 0, 3) for b in range(-(-ny // br))]
    c = CH.correlate_chunked(pair.ref, pair.deformed, pair.roi, seeds=seeds, band_rows=br, halo=0, threads=8,
                             **PRM)
    act = full["status"] == ST["CONVERGED"]
    last_rows = np.zeros_like(act)
    last_rows[br - 1::br] = True
    last_rows[ny - 1] = False                         # the last band's window ends at the image's edge
    assert (last_rows & act).sum() > 100
    assert np.all(c["status"][last_rows & act] == ST["OUT_OF_BOUNDS"])
    rest = act & ~last_rows
    assert np.all(c["status"][rest] == ST["CONVERGED"])
    # away from the window's edges the values match; a band's first node row and
    # the row above its last sample the deformed spline within 3 rows of the
    # window's edge, where the window's own prefilter differs from the image's
    interior = np.zeros_like(act)
    interior[np.arange(ny) % br <= br - 3] = True
    interior[br::br] = False
    assert np.abs(c["p"][:2] - full["p"][:2])[:, rest & interior].max() < 2e-3
    # one seed only: the band below the first cannot be seeded across an edge row
    # that did not converge, so it and every band after it stay NOT_REACHED
    one = CH.correlate_chunked(pair.ref, pair.deformed, pair.roi, seeds=seeds[:1], band_rows=br, halo=0,
                               threads=8, **PRM)
    assert np.all(one["status"][br:][act[br:]] == ST["NOT_REACHED"])


def test_given_seeds_reach_bands_behind_an_roi_gap():
    # the ROI is cut by a band of 30 empty rows: no boundary carries a seed across it
    pair = _pair(synth.field_affine(-1.0, 0.5, 0.004, 0.0, 0.0, 0.004, 100, 116))
    roi = pair.roi.copy()
    roi[100:130] = 0
    top, bottom = (100, 40, -1, 0), (100, 190, -1, 1)
    one = CH.correlate_chunked(pair.ref, pair.deformed, roi, seeds=[top], band_rows=5, halo=10, threads=8, **PRM)
    two = CH.correlate_chunked(pair.ref, pair.deformed, roi, seeds=[top, bottom], band_rows=5, halo=10, threads=8,
                               **PRM)
    full = oracle.correlate(pair.ref, pair.deformed, roi, seeds=[top, bottom], threads=8, **PRM)
    below = np.zeros_like(one["status"], bool)
    below[(130 - 0) // 4:] = True
    act = one["status"] != ST["NOT_IN_ROI"]
    assert np.all(one["status"][below & act] == ST["NOT_REACHED"])
    frac, dmax = _converged_agree(two, full)
    assert frac > 0.99 and dmax < 2e-3
