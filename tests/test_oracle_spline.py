"""Pins of the oracle's cubic B-spline prefilter and evaluation (Sec. 2.2,
"bicubic b-spline") against definitions that do not go through the oracle:
a dense linear solve of the interpolation condition, scipy's spline routines,
the closed-form impulse response, polynomial reproduction and finite
differences."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle


def _mirror_system(n):
    """Dense matrix of (c[k-1] + 4 c[k] + c[k+1]) / 6 with c[-1]=c[1], c[n]=c[n-2]."""
    A = np.zeros((n, n))
    for k in range(n):
        for d, w in ((-1, 1.0), (0, 4.0), (1, 1.0)):
            j = k + d
            if j < 0:
                j = -j
            if j > n - 1:
                j = 2 * (n - 1) - j
            A[k, j] += w / 6.0
    return A


@pytest.mark.parametrize("n", [2, 3, 5, 16, 77, 512])
def test_prefilter_line_solves_interpolation_condition(n):
    rng = np.random.default_rng(n)
    s = rng.uniform(-100, 300, n)
    c = oracle.prefilter_line(s)
    ref = np.linalg.solve(_mirror_system(n), s)
    assert np.abs(c - ref).max() <= 1e-12 * np.abs(ref).max()


def test_prefilter_2d_matches_scipy_mirror():
    rng = np.random.default_rng(1)
    img = rng.uniform(0, 4095, (53, 71))
    c = oracle.prefilter(img)
    cs = ndi.spline_filter(img, order=3, mode="mirror")
    assert np.abs(c - cs).max() <= 1e-12 * np.abs(cs).max()


def test_prefilter_impulse_response_closed_form():
    # interior response to a unit impulse: h[k] = sqrt(3) (sqrt(3) - 2)^|k|
    n = 301
    s = np.zeros(n)
    s[150] = 1.0
    c = oracle.prefilter_line(s)
    k = np.arange(-20, 21)
    h = np.sqrt(3.0) * (np.sqrt(3.0) - 2.0) ** np.abs(k)
    assert np.abs(c[150 + k] - h).max() <= 1e-14


def test_eval_matches_scipy_map_coordinates():
    rng = np.random.default_rng(2)
    img = rng.uniform(0, 255, (40, 57))
    c = oracle.prefilter(img)
    x = np.concatenate([rng.uniform(0, 56, 500), [0.0, 56.0, 0.25, 55.9]])
    y = np.concatenate([rng.uniform(0, 39, 500), [0.0, 39.0, 38.7, 0.1]])
    v, _, _ = oracle.evaluate(c, x, y)
    vs = ndi.map_coordinates(img, [y, x], order=3, mode="mirror")
    assert np.abs(v - vs).max() <= 1e-11


def test_eval_reproduces_samples_at_integer_pixels():
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 255, (23, 31))
    c = oracle.prefilter(img)
    yy, xx = np.mgrid[0:23, 0:31]
    v, _, _ = oracle.evaluate(c, xx.ravel().astype(float), yy.ravel().astype(float))
    assert np.abs(v - img.ravel()).max() <= 1e-11


def _cubic_image(W, H):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)

    def f(x, y):
        return (40 + 3.0 * x - 2.0 * y + 0.05 * x * x - 0.03 * x * y + 0.02 * y * y
                + 1e-3 * x ** 3 - 2e-3 * x * x * y + 5e-4 * y ** 3 + 1e-5 * x ** 3 * y ** 3 / 100)

    def fx(x, y):
        return 3.0 + 0.1 * x - 0.03 * y + 3e-3 * x * x - 4e-3 * x * y + 3e-5 * x * x * y ** 3 / 100

    def fy(x, y):
        return -2.0 - 0.03 * x + 0.04 * y - 2e-3 * x * x + 1.5e-3 * y * y + 3e-5 * x ** 3 * y * y / 100
    return f(xx, yy), f, fx, fy


def test_eval_reproduces_tensor_cubic_polynomials_in_interior():
    # a cubic B-spline reproduces polynomials of degree <= 3 in each variable;
    # the mirror boundary only leaks in as |sqrt(3)-2|^distance
    img, f, fx, fy = _cubic_image(96, 96)
    c = oracle.prefilter(img)
    rng = np.random.default_rng(4)
    x = rng.uniform(38, 58, 300)
    y = rng.uniform(38, 58, 300)
    v, gx, gy = oracle.evaluate(c, x, y)
    scale = np.abs(img).max()
    assert np.abs(v - f(x, y)).max() <= 1e-11 * scale
    assert np.abs(gx - fx(x, y)).max() <= 1e-10 * scale
    assert np.abs(gy - fy(x, y)).max() <= 1e-10 * scale


def test_eval_derivative_matches_finite_difference():
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 255, (30, 30))
    c = oracle.prefilter(img)
    x = rng.uniform(2, 27, 200)
    y = rng.uniform(2, 27, 200)
    e = 1e-5
    _, gx, gy = oracle.evaluate(c, x, y)
    fxp, _, _ = oracle.evaluate(c, x + e, y)
    fxm, _, _ = oracle.evaluate(c, x - e, y)
    fyp, _, _ = oracle.evaluate(c, x, y + e)
    fym, _, _ = oracle.evaluate(c, x, y - e)
    assert np.abs(gx - (fxp - fxm) / (2 * e)).max() <= 1e-5
    assert np.abs(gy - (fyp - fym) / (2 * e)).max() <= 1e-5
