"""Pins of the oracle's other costs (SSD, Eq. (2); NSSD, Eq. (3)), the rigid
shape of Eq. (5) in the full correlation, and Levenberg-Marquardt damping
(Sec. 2.2): exact integer shifts, the intensity changes each cost is and is
not invariant to, brute-force grid minimisation of each cost through scipy's
interpolation, the damped solve's limits, and LM reaching Gauss-Newton's
fixed point."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from oracle import ST
from paper_2601_12941_amd import synth

from test_oracle_icgn import speckle


@pytest.mark.parametrize("cost", ["ssd", "nssd"])
@pytest.mark.parametrize("npar", [2, 6, 12])
def test_integer_shift_recovered_exactly(cost, npar):
    ref, _ = speckle(128, seed=12)
    dx, dy = 3, -2
    de = np.roll(np.roll(ref, dy, axis=0), dx, axis=1)
    p0 = np.zeros(npar)
    p0[:2] = [2.6, -1.5]
    p, z, it, st = oracle.icgn(ref, de, 64, 64, p0, 21, npar, tol=1e-12, max_iter=100, cost=cost)
    assert st == ST["CONVERGED"]
    assert abs(p[0] - dx) <= 1e-9 and abs(p[1] - dy) <= 1e-9 and np.abs(p[2:]).max(initial=0) <= 1e-9
    assert abs(z - 1.0) <= 1e-12


@pytest.mark.parametrize("cost", ["ssd", "nssd"])
def test_zero_displacement_is_exactly_zero(cost):
    ref, _ = speckle(64)
    p, z, it, st = oracle.icgn(ref, ref, 32, 30, np.zeros(6), 21, 6, cost=cost)
    assert st == ST["CONVERGED"] and it == 1 and np.all(p == 0.0) and z == 1.0


def test_invariances_of_each_cost():
    # Sec. 2.2: NSSD is invariant to a scale of the deformed intensities, ZNSSD to
    # scale and offset, SSD to neither (its fixed point moves)
    ref, de = speckle(96, field=synth.field_affine(0.37, -0.21), noise=1.0)
    args = (48, 48, [0, 0, 0, 0, 0, 0], 21, 6)
    kw = dict(tol=1e-10, max_iter=200)
    base = {c: oracle.icgn(ref, de, *args, cost=c, **kw)[0] for c in ("znssd", "nssd", "ssd")}
    scaled = {c: oracle.icgn(ref, 1.7 * de, *args, cost=c, **kw)[0] for c in ("znssd", "nssd", "ssd")}
    shifted = {c: oracle.icgn(ref, 1.7 * de + 30.0, *args, cost=c, **kw)[0] for c in ("znssd", "nssd", "ssd")}
    assert np.abs(scaled["znssd"] - base["znssd"]).max() <= 1e-8
    assert np.abs(shifted["znssd"] - base["znssd"]).max() <= 1e-8
    assert np.abs(scaled["nssd"] - base["nssd"]).max() <= 1e-8
    assert np.abs(shifted["nssd"] - base["nssd"]).max() > 1e-4
    assert np.abs(scaled["ssd"] - base["ssd"]).max() > 1e-4


def _cost_grid(fc, gc, xc, yc, N, us, vs, cost):
    """Eq. (2) or Eq. (3) on a (u, v) grid with scipy's cubic spline (rigid shape)."""
    h = N // 2
    dy, dx = np.mgrid[-h:h + 1, -h:h + 1]
    f = ndi.map_coordinates(fc, [yc + dy.ravel(), xc + dx.ravel()], order=3, mode="mirror", prefilter=False)
    U, V = np.meshgrid(us, vs)
    xs = xc + dx.ravel()[None, :] + U.ravel()[:, None]
    ys = yc + dy.ravel()[None, :] + V.ravel()[:, None]
    g = ndi.map_coordinates(gc, [ys.ravel(), xs.ravel()], order=3, mode="mirror", prefilter=False).reshape(xs.shape)
    if cost == "ssd":
        c = ((f[None, :] - g) ** 2).sum(1)
    else:
        c = ((f[None, :] / np.linalg.norm(f) - g / np.linalg.norm(g, axis=1, keepdims=True)) ** 2).sum(1)
    k = c.argmin()
    return U.ravel()[k], V.ravel()[k], c.min()


@pytest.mark.parametrize("cost", ["ssd", "nssd"])
@pytest.mark.parametrize("N,xc,yc", [(7, 32, 32), (9, 44, 25)])
def test_brute_force_grid_minimum(cost, N, xc, yc):
    # noise-free shift: the IC fixed point is the minimiser of the cost itself
    ref, de = speckle(64, field=synth.field_affine(0.37, -0.21))
    p, z, it, st = oracle.icgn(ref, de, xc, yc, [0, 0], N, 2, tol=1e-10, max_iter=100, cost=cost)
    assert st == ST["CONVERGED"]
    fc = ndi.spline_filter(ref, order=3, mode="mirror")
    gc = ndi.spline_filter(de, order=3, mode="mirror")
    g1 = np.arange(-0.5, 0.5001, 0.01)
    u1, v1, _ = _cost_grid(fc, gc, xc, yc, N, p[0] + g1, p[1] + g1, cost)
    g2 = np.arange(-0.02, 0.02001, 0.001)
    u2, v2, _ = _cost_grid(fc, gc, xc, yc, N, u1 + g2, v1 + g2, cost)
    assert abs(u2 - p[0]) <= 1.5e-3 and abs(v2 - p[1]) <= 1.5e-3


def test_damped_step_limits():
    # one iteration from the same start: the LM increment solves (H + lam diag H) dp = -b,
    # so it tends to the Gauss-Newton increment as lam -> 0, shrinks monotonically with
    # lam, and lam dp tends to the fixed vector -diag(H)^-1 b as lam grows (rigid
    # shape: p1 = p0 - dp)
    ref, de = speckle(96, field=synth.field_affine(0.37, -0.21), noise=1.0)
    p0 = np.array([0.1, 0.05])

    def step(lam):
        p, _, _, st = oracle.icgn(ref, de, 48, 48, p0, 21, 2, tol=1e-14, max_iter=1, lm_lambda=lam)
        assert st == ST["MAX_ITER"]
        return p0 - p
    gn = step(0.0)
    d = {lam: step(lam) for lam in (1e-9, 1e-2, 1.0, 1e2, 1e6, 1e7)}
    np.testing.assert_allclose(d[1e-9], gn, rtol=1e-7)
    norms = [np.linalg.norm(d[k]) for k in sorted(d)]
    assert all(a > b for a, b in zip(norms, norms[1:]))
    np.testing.assert_allclose(1e6 * d[1e6], 1e7 * d[1e7], rtol=2e-6)
    assert np.dot(gn, d[1e6]) > 0


@pytest.mark.parametrize("cost", ["znssd", "nssd", "ssd"])
def test_lm_reaches_the_gauss_newton_fixed_point(cost):
    # an integer shift is an exact zero-residual point of every cost: the damped
    # iteration ends there, as Gauss-Newton does
    ref, _ = speckle(128, seed=12)
    de = np.roll(np.roll(ref, -2, axis=0), 3, axis=1)
    kw = dict(tol=1e-10, max_iter=300, cost=cost)
    start = [2.55, -1.6, 0, 0, 0, 0]
    a = oracle.icgn(ref, de, 64, 64, start, 21, 6, **kw)
    b = oracle.icgn(ref, de, 64, 64, start, 21, 6, lm_lambda=1.0, **kw)
    assert a[3] == b[3] == ST["CONVERGED"]
    assert np.abs(a[0] - [3, -2, 0, 0, 0, 0]).max() <= 1e-9 and np.abs(b[0] - [3, -2, 0, 0, 0, 0]).max() <= 1e-9
    assert b[2] >= a[2]          # damping costs iterations
    # with noise and a rendered (not interpolated) deformation the IC fixed point is
    # only near the cost's minimiser; the damped iteration, whose merit is the
    # undamped increment, ends at Gauss-Newton's fixed point all the same
    ref, de = speckle(128, field=synth.field_affine(1.3, -0.8, dudx=0.01, dvdy=-0.008), noise=1.0)
    for c in ("znssd", "nssd", "ssd"):
        kw["cost"] = c
        a = oracle.icgn(ref, de, 64, 64, [0.4, -0.2, 0, 0, 0, 0], 21, 6, **kw)
        b = oracle.icgn(ref, de, 64, 64, [0.4, -0.2, 0, 0, 0, 0], 21, 6, lm_lambda=1.0, **kw)
        assert a[3] == b[3] == ST["CONVERGED"]
        assert np.abs(a[0][:2] - b[0][:2]).max() <= 1e-8


def test_rigid_correlation_of_a_translation_field():
    # the rigid shape through the whole reliability-guided correlation
    W = 160
    f = synth.field_affine(2.3, -1.4)
    ref, de = speckle(W, dens=0.02, sigma=(2.0, 3.5), seed=21, field=f)
    roi = synth.roi_from_field(W, W, f)
    for cost in ("znssd", "nssd", "ssd"):
        r = oracle.correlate(ref, de, roi, subset_size=21, step=6, shape=2, seeds=[(80, 80, 2, -1)], seed_radius=3,
                             cost=cost)
        ok = r["status"] == ST["CONVERGED"]
        assert ok.sum() == (r["status"] != ST["NOT_IN_ROI"]).sum()
        assert np.abs(r["u"][ok] - 2.3).max() < 0.01 and np.abs(r["v"][ok] + 1.4).max() < 0.01
        assert np.all(r["p"][2:, ok] == 0.0)
