"""Pins of the multi-window FFT oracle (paper Sec. 2.2, Eq. (1); Sec. 4's MAD
outlier removal): the transform against numpy.fft, Eq. (1) on circular and
windowed integer shifts, the 3-point Gaussian fit on exact Gaussians, the
window schedule of the paper's example, the MAD pass against numpy medians,
and whole-image estimates of large displacements against the field."""
import numpy as np
import pytest

import oracle
from paper_2601_12941_amd import synth

from test_oracle_icgn import speckle


@pytest.mark.parametrize("W", [2, 8, 32, 128])
def test_fft2_against_numpy(W):
    rng = np.random.default_rng(W)
    a = rng.normal(size=(W, W)) + 1j * rng.normal(size=(W, W))
    np.testing.assert_allclose(oracle.fft2(a), np.fft.fft2(a), rtol=0, atol=1e-10 * W * W)
    np.testing.assert_allclose(oracle.fft2(a, inverse=True), np.fft.ifft2(a) * W * W, rtol=0, atol=1e-10 * W * W)


@pytest.mark.parametrize("dx, dy", [(3, -5), (-7, 0), (15, 16), (0, 0)])
def test_phase_correlation_of_a_circular_shift_is_a_delta(dx, dy):
    # g(x) = f(x - d) circularly: F conj(G) / |F||G| = exp(i k d), its inverse a unit
    # delta at -d; the peak reports q = -d (wrapped into [-W/2, W/2))
    W = 32
    f = np.random.default_rng(1).normal(size=(W, W))
    g = np.roll(np.roll(f, dy, axis=0), dx, axis=1)
    r = oracle.phase_corr(f, g)
    qx, qy, margin = oracle.map_peak(r)
    wrap = lambda q: (q + W // 2) % W - W // 2
    assert (qx, qy) == (wrap(-dx), wrap(-dy))
    assert abs(r.max() - 1.0) < 1e-12 and margin > 0.99


def test_gaussian_fit_is_exact_on_gaussians():
    for e in (-0.43, -0.1, 0.0, 0.27, 0.49):
        a, b, c = (np.exp(-((x - e) ** 2) / 1.7) for x in (-1.0, 0.0, 1.0))
        assert abs(oracle.gauss3(a, b, c) - e) < 1e-12
    # parabolic fallback with a non-positive side, exact on parabolas
    e = 0.2
    a, b, c = (1.0 - (x - e) ** 2 for x in (-1.0, 0.0, 1.0))
    assert a < 0 and abs(oracle.gauss3(a, b, c) - e) < 1e-12
    assert oracle.gauss3(1.0, 1.0, 1.0) == 0.0        # degenerate: no shift


def test_window_schedule_of_the_paper_example():
    # maximum displacement 800 px and subset 17: powers of two from 1024 down, the
    # node level at the smallest power of two holding the subset (32)
    assert oracle.mw_levels(800, 17, 4096, 4096) == ([1024, 512, 256, 128, 64], 32)
    assert oracle.mw_levels(2000, 31, 32000, 32000) == ([2048, 1024, 512, 256, 128, 64], 32)
    assert oracle.mw_levels(512, 31, 4096, 4096) == ([1024, 512, 256, 128, 64], 32)   # "above" 512
    assert oracle.mw_levels(800, 17, 600, 900) == ([512, 256, 128, 64], 32)           # capped by the image
    assert oracle.mw_levels(10, 31, 256, 256) == ([], 32)
    assert oracle.mw_levels(10, 33, 48, 48)[1] == 0                                   # no room for a window


def test_mad_pass_against_numpy_medians():
    rng = np.random.default_rng(4)
    u = np.round(5 + 0.3 * np.arange(12)[None, :] + rng.normal(0, 0.4, (9, 12))).astype(np.int32)
    v = np.round(-3 + rng.normal(0, 0.4, (9, 12))).astype(np.int32)
    u[4, 6] += 40
    v[2, 3] -= 25
    fu, fv, rep = oracle.mad_filter(u, v, thr=2.0)
    assert rep[4, 6] and rep[2, 3]
    for j, i in zip(*np.nonzero(rep)):
        nb = [(jj, ii) for jj in range(j - 1, j + 2) for ii in range(i - 1, i + 2)
              if (jj, ii) != (j, i) and 0 <= jj < 9 and 0 <= ii < 12]
        mu = np.median([u[p] for p in nb])
        mv = np.median([v[p] for p in nb])
        assert fu[j, i] == int(np.sign(mu) * np.floor(abs(mu) + 0.5))
        assert fv[j, i] == int(np.sign(mv) * np.floor(abs(mv) + 0.5))
    # every unreplaced entry passes the test against numpy's medians
    for j in range(9):
        for i in range(12):
            if rep[j, i]:
                continue
            nb = np.array([(u[jj, ii], v[jj, ii]) for jj in range(j - 1, j + 2) for ii in range(i - 1, i + 2)
                           if (jj, ii) != (j, i) and 0 <= jj < 9 and 0 <= ii < 12], float)
            med = np.median(nb, axis=0)
            mad = np.median(np.abs(nb - med), axis=0)
            assert np.all(np.abs(np.array([u[j, i], v[j, i]]) - med) <= 2.0 * (mad + 1.0))
    assert rep.sum() <= 6


@pytest.mark.parametrize("t", [(150.0, -80.0), (-37.0, 211.0)])
def test_large_integer_translation_is_recovered_exactly(t):
    # an integer translation far beyond any subset: every node's estimate is exact.
    # (Eq. (1)'s map is circular: a level resolves shifts up to half its window,
    # so the maximum displacement given is about twice the actual one, as in the
    # paper's SEM run.)
    W = 512
    ref, _ = speckle(W + 512, dens=0.02, sigma=(1.5, 3.0), seed=31)
    ox, oy = 256, 256
    de = ref[oy - int(t[1]):oy - int(t[1]) + W, ox - int(t[0]):ox - int(t[0]) + W]
    ref = ref[oy:oy + W, ox:ox + W]
    f = synth.field_affine(*t)
    roi = synth.roi_from_field(W, W, f)
    r = oracle.multiwindow(ref, de, roi, subset_size=21, step=8, max_disp=300)
    assert r["levels"] == [512, 256, 128, 64, 32]
    ok = r["valid"]
    assert ok.sum() > 100
    assert np.all(r["u"][ok] == t[0]) and np.all(r["v"][ok] == t[1])


def test_subpixel_estimate_of_a_rendered_affine_field():
    # a rendered (not shifted) speckle with a large translation and 1 % strain: the
    # integer mode is within a pixel everywhere; the Gaussian sub-pixel mode moves
    # each estimate toward the field (the sharp phase-correlation peak makes the
    # 3-point fit underestimate the fraction: peak locking), about halving the error
    W = 384
    f = synth.field_affine(120.4, -60.7, dudx=0.01, dvdy=-0.005, xc=W / 2, yc=W / 2)
    ref, de = speckle(W, dens=0.03, sigma=(1.5, 3.0), seed=17, field=f)
    roi = synth.roi_from_field(W, W, f)
    u, v, _ = synth.truth_at_nodes(f, W, W, 31, 10)
    r0 = oracle.multiwindow(ref, de, roi, subset_size=31, step=10, max_disp=250)
    r1 = oracle.multiwindow(ref, de, roi, subset_size=31, step=10, max_disp=250, subpixel=True)
    ok = r0["valid"]
    assert ok.sum() > 200
    # the node window's centre is 0.5 px above-left of the node; strain <= 1 % moves it < 0.01 px
    assert np.abs(r0["u"] - u)[ok].max() <= 1.0 and np.abs(r0["v"] - v)[ok].max() <= 1.0
    e0 = np.hypot(r0["u"] - u, r0["v"] - v)[ok]
    e1 = np.hypot(r1["u"] - u, r1["v"] - v)[ok]
    assert np.median(e1) < 0.6 * np.median(e0) and np.percentile(e1, 99) < 0.5
    # the fit moves from the integer peak toward the true position
    res = (u - r0["u"])[ok]
    big = np.abs(res) > 0.15
    assert np.all(np.sign((r1["u"] - r0["u"])[ok][big]) == np.sign(res[big]))


def test_mad_removes_a_wrong_window_at_the_node_level():
    # a patch of the deformed image replaced by unrelated speckle: those windows'
    # peaks are random, and the MAD pass brings isolated ones back to their neighbours
    W = 256
    f = synth.field_affine(40.0, 25.0)
    ref, de = speckle(W, dens=0.03, sigma=(1.5, 3.0), seed=5, field=f)
    other, _ = speckle(W, dens=0.03, sigma=(1.5, 3.0), seed=99)
    de = de.copy()
    de[150:166, 150:166] = other[150:166, 150:166]
    roi = synth.roi_from_field(W, W, f)
    a = oracle.multiwindow(ref, de, roi, subset_size=15, step=8, max_disp=100, mad_threshold=0.0)
    b = oracle.multiwindow(ref, de, roi, subset_size=15, step=8, max_disp=100)
    ok = a["valid"]
    bad_a = ((np.abs(a["u"] - 40) > 1) | (np.abs(a["v"] - 25) > 1)) & ok
    bad_b = ((np.abs(b["u"] - 40) > 1) | (np.abs(b["v"] - 25) > 1)) & ok
    assert bad_b.sum() < bad_a.sum()
