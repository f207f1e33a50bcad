"""FP64 reference of the strain post-processing (paper Sec. 2.3).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library's own
path.  Plain numpy: one least-squares fit per window (numpy.linalg.lstsq) and
one symmetric eigendecomposition per node (numpy.linalg.eigh) for the matrix
square roots and logarithms.  It shares no code with the GPU path (which
applies precomputed fit weights and closed-form 2x2 matrix functions).

What it computes:
  * Eq. (8)-(9): over a square window of N x N displacement nodes centred on a
    node, fit u_x and u_y by linear least squares in a polynomial basis of the
    local node offsets (x, y) in pixels (offset times the grid step);
    reading of the bases: bilinear = [1, x, y, xy] and biquadratic = the full
    tensor product [1, x, y, xy, x^2, y^2, x^2 y, x y^2, x^2 y^2] (4 and 9
    "window elements"; the printed lists drop the xy term);
  * Eq. (6): F = I + grad u from the fitted polynomials' derivatives at the
    window centre (x = y = 0);
  * the five strain measures listed in Sec. 2.3: Green-Lagrange
    (F^T F - I)/2, Hencky ln sqrt(F^T F), Euler-Almansi (I - (F F^T)^-1)/2,
    Biot right sqrt(F^T F) - I, Biot left sqrt(F F^T) - I;
  * Eq. (7): the virtual strain gauge VSG = (N - 1) s + w.
Reading where the paper is silent: a node gets a strain only if its whole
window lies inside the grid and every node of it holds a valid displacement
(CONVERGED status, finite u and v); every other node is NaN.
"""
from __future__ import annotations

import numpy as np

BASES = {"bilinear": 4, "biquadratic": 9}
MEASURES = ("green_lagrange", "hencky", "euler_almansi", "biot_right", "biot_left")


def vsg(window: int, step: int, subset_size: int) -> int:
    """Eq. (7): virtual strain gauge size in pixels."""
    return (window - 1) * step + subset_size


def basis_row(x, y, basis: str):
    """Eq. (9) basis terms at local offsets (x, y) (arrays), as columns."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    one = np.ones_like(x)
    if basis == "bilinear":
        return np.stack([one, x, y, x * y], axis=-1)
    if basis == "biquadratic":
        return np.stack([one, x, y, x * y, x * x, y * y, x * x * y, x * y * y, x * x * y * y], axis=-1)
    raise ValueError(basis)


def deformation_gradient(u, v, step: int, window: int, basis: str = "bilinear", valid=None):
    """F [2][2][ny][nx] from displacement fields u, v [ny][nx] on a grid of the
    given step (Eq. (6) and (8)); NaN where the window is incomplete."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    ny, nx = u.shape
    ok = np.isfinite(u) & np.isfinite(v)
    if valid is not None:
        ok &= np.asarray(valid, bool)
    r = (window - 1) // 2
    off = np.arange(-r, r + 1) * float(step)
    X, Y = np.meshgrid(off, off)            # X varies along columns (x), Y along rows (y)
    A = basis_row(X.ravel(), Y.ravel(), basis)
    F = np.full((2, 2, ny, nx), np.nan)
    for j in range(r, ny - r):
        for i in range(r, nx - r):
            win = (slice(j - r, j + r + 1), slice(i - r, i + r + 1))
            if not ok[win].all():
                continue
            cu = np.linalg.lstsq(A, u[win].ravel(), rcond=None)[0]
            cv = np.linalg.lstsq(A, v[win].ravel(), rcond=None)[0]
            # d/dx and d/dy of the basis at the origin pick the x and y coefficients
            F[0, 0, j, i] = 1.0 + cu[1]
            F[0, 1, j, i] = cu[2]
            F[1, 0, j, i] = cv[1]
            F[1, 1, j, i] = 1.0 + cv[2]
    return F


def _sym_fn(M, fn):
    """fn applied to a symmetric positive-definite 2x2 matrix through its eigenbasis."""
    lam, V = np.linalg.eigh(M)
    return (V * fn(lam)) @ V.T


def strain_tensor(F, measure: str):
    """One strain measure of a single 2x2 deformation gradient (Sec. 2.3)."""
    F = np.asarray(F, np.float64)
    I = np.eye(2)
    if measure == "green_lagrange":
        return 0.5 * (F.T @ F - I)
    if measure == "hencky":
        return _sym_fn(F.T @ F, lambda l: np.log(np.sqrt(l)))
    if measure == "euler_almansi":
        return 0.5 * (I - np.linalg.inv(F @ F.T))
    if measure == "biot_right":
        return _sym_fn(F.T @ F, np.sqrt) - I
    if measure == "biot_left":
        return _sym_fn(F @ F.T, np.sqrt) - I
    raise ValueError(measure)


def strain(u, v, step: int, window: int, basis: str = "bilinear", measure: str = "green_lagrange", valid=None):
    """Deformation gradient [2][2][ny][nx] and strain (xx, xy, yy) [3][ny][nx]."""
    F = deformation_gradient(u, v, step, window, basis, valid)
    ny, nx = F.shape[2:]
    eps = np.full((3, ny, nx), np.nan)
    for j in range(ny):
        for i in range(nx):
            f = F[:, :, j, i]
            if not np.isfinite(f).all():
                continue
            e = strain_tensor(f, measure)
            eps[:, j, i] = e[0, 0], e[0, 1], e[1, 1]
    return F, eps
