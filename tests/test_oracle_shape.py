"""Pins of the oracle's shape-function algebra (Eq. (5)): the
inverse-compositional update p <- p o dp^{-1} and the guess transfer between
neighbouring nodes, checked by evaluating warps as point maps (numpy linear
solves / Newton inversion), independent of the oracle's closed forms."""
import numpy as np
import pytest

import oracle


def warp(p, dx, dy):
    """Eq. (5) with x, y read as offsets from the subset centre."""
    p = np.concatenate([np.asarray(p, float), np.zeros(12 - len(p))])
    X = dx + p[0] + p[2] * dx + p[3] * dy + p[6] * dx * dx + p[7] * dx * dy + p[8] * dy * dy
    Y = dy + p[1] + p[4] * dx + p[5] * dy + p[9] * dx * dx + p[10] * dx * dy + p[11] * dy * dy
    return X, Y


def inverse_point(p, X, Y):
    """Solve warp(p, x, y) = (X, Y) for (x, y) by Newton iteration."""
    p = np.concatenate([np.asarray(p, float), np.zeros(12 - len(p))])
    x, y = np.array(X, float), np.array(Y, float)
    for _ in range(60):
        fx, fy = warp(p, x, y)
        rx, ry = fx - X, fy - Y
        a = 1 + p[2] + 2 * p[6] * x + p[7] * y
        b = p[3] + p[7] * x + 2 * p[8] * y
        c = p[4] + 2 * p[9] * x + p[10] * y
        d = 1 + p[5] + p[10] * x + 2 * p[11] * y
        det = a * d - b * c
        x = x - (d * rx - b * ry) / det
        y = y - (-c * rx + a * ry) / det
    return x, y


def rand_p(rng, n, scale=1.0):
    p = np.zeros(n)
    p[:2] = rng.uniform(-3, 3, 2) * scale
    if n >= 6:
        p[2:6] = rng.uniform(-0.05, 0.05, 4) * scale
    if n >= 12:
        p[6:12] = rng.uniform(-2e-3, 2e-3, 6) * scale
    return p


@pytest.mark.parametrize("n", [2, 6, 12])
def test_compose_with_zero_increment_is_identity(n):
    rng = np.random.default_rng(n)
    p = rand_p(rng, n)
    assert np.abs(oracle.compose(p, np.zeros(n), n) - p).max() <= 1e-16


@pytest.mark.parametrize("n", [2, 6])
def test_compose_self_inverse_gives_identity_warp(n):
    rng = np.random.default_rng(10 + n)
    p = rand_p(rng, n)
    assert np.abs(oracle.compose(p, p, n)).max() <= 1e-14


@pytest.mark.parametrize("n", [2, 6])
def test_compose_is_exact_point_composition_rigid_affine(n):
    rng = np.random.default_rng(20 + n)
    for _ in range(20):
        p, dp = rand_p(rng, n), rand_p(rng, n, 0.3)
        q = oracle.compose(p, dp, n)
        X, Y = rng.uniform(-15, 15, 50), rng.uniform(-15, 15, 50)
        # p o dp^{-1} (X, Y) = p(dp^{-1}(X, Y)), dp^{-1} by a 2x2 linear solve
        A = np.array([[1 + (dp[2] if n > 2 else 0), dp[3] if n > 2 else 0],
                      [dp[4] if n > 2 else 0, 1 + (dp[5] if n > 2 else 0)]])
        xy = np.linalg.solve(A, np.vstack([X - dp[0], Y - dp[1]]))
        ex, ey = warp(p, xy[0], xy[1])
        qx, qy = warp(q, X, Y)
        assert max(np.abs(qx - ex).max(), np.abs(qy - ey).max()) <= 1e-12


def test_compose_quadratic_exact_for_affine_increment():
    # quadratic o affine^{-1} is quadratic: the lifted rule must be exact
    rng = np.random.default_rng(30)
    for _ in range(20):
        p = rand_p(rng, 12)
        dp = np.zeros(12)
        dp[:6] = rand_p(rng, 6, 0.3)
        q = oracle.compose(p, dp, 12)
        X, Y = rng.uniform(-15, 15, 50), rng.uniform(-15, 15, 50)
        x, y = inverse_point(dp, X, Y)
        ex, ey = warp(p, x, y)
        qx, qy = warp(q, X, Y)
        assert max(np.abs(qx - ex).max(), np.abs(qy - ey).max()) <= 1e-10


def test_compose_quadratic_first_order_in_increment():
    # affine p, general quadratic increment eps*d: p o (eps d)^{-1} is a
    # quadratic up to O(eps^2), and the lifted rule must agree with it to
    # O(eps^2) (first-order exact): the error shrinks ~100x per 10x in eps.
    # (With a quadratic p the exact composition carries O(eps) cubic terms
    # that no quadratic represents, so only its affine-increment case is exact.)
    rng = np.random.default_rng(31)
    p = np.zeros(12)
    p[:6] = rand_p(rng, 6)
    d = rand_p(rng, 12)
    X, Y = rng.uniform(-10, 10, 200), rng.uniform(-10, 10, 200)
    errs = []
    for eps in (1e-1, 1e-2, 1e-3):
        q = oracle.compose(p, eps * d, 12)
        x, y = inverse_point(eps * d, X, Y)
        ex, ey = warp(p, x, y)
        qx, qy = warp(q, X, Y)
        errs.append(max(np.abs(qx - ex).max(), np.abs(qy - ey).max()))
    assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 30


def test_ic_update_sign_convention():
    # content moved by +d: at p = 0 the increment is -d (dp = -H^-1 J^T r) and
    # the composed update gives p = +d
    p = oracle.compose(np.zeros(2), np.array([-0.4, 0.7]), 2)
    assert np.allclose(p, [0.4, -0.7])


@pytest.mark.parametrize("n", [2, 6, 12])
def test_guess_transfer_reexpands_the_neighbour_warp(n):
    # the neighbour's displacement field evaluated at delta + offset equals the
    # transferred shape evaluated at offset (exact for polynomial shapes up to
    # the order the shape carries)
    rng = np.random.default_rng(40 + n)
    pm = rand_p(rng, n)
    for ddx, ddy in ((5, 0), (-5, 0), (0, 5), (0, -5)):
        q = oracle.transfer_guess(pm, n, ddx, ddy)
        ox, oy = rng.uniform(-10, 10, 40), rng.uniform(-10, 10, 40)
        mx, my = warp(pm, ox + ddx, oy + ddy)
        qx, qy = warp(q, ox, oy)
        if n == 2:
            # rigid: displacement copied
            assert np.allclose(q, pm)
            continue
        assert np.abs((mx - ddx) - qx).max() <= 1e-12 and np.abs((my - ddy) - qy).max() <= 1e-12


def test_guess_copy_mode():
    pm = np.array([1.0, 2.0, 0.1, 0.0, 0.0, -0.1])
    assert np.array_equal(oracle.transfer_guess(pm, 6, 5, 0, mode="copy"), pm)
