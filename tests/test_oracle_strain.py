"""Pins of the strain oracle (paper Sec. 2.3, Eq. (6)-(9)) against closed
forms: polynomial displacement fields each basis reproduces exactly, strain
measures of stretches, rotations and simple shear, and scipy's matrix square
root and logarithm (a different algorithm from the oracle's eigenbasis)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import strain as S


def _grid(nx, ny, step, fu, fv):
    X, Y = np.meshgrid(np.arange(nx) * float(step), np.arange(ny) * float(step))
    return fu(X, Y), fv(X, Y), X, Y


def test_vsg_is_eq7():
    assert S.vsg(5, 2, 31) == 39
    assert S.vsg(9, 15, 31) == 151
    assert S.vsg(1, 7, 21) == 21


@pytest.mark.parametrize("step", [1, 3])
def test_bilinear_reproduces_bilinear_fields(step):
    # u = a + b x + c y + d x y: the bilinear fit is exact, grad u at a node is (b + d y, c + d x)
    a, b, c, d = 0.7, 0.013, -0.021, 4e-4
    u, v, X, Y = _grid(12, 10, step, lambda X, Y: a + b * X + c * Y + d * X * Y,
                       lambda X, Y: -0.2 + 0.005 * X + 0.017 * Y - 3e-4 * X * Y)
    F = S.deformation_gradient(u, v, step, 5, "bilinear")
    r = 2
    sl = (slice(r, -r), slice(r, -r))
    np.testing.assert_allclose(F[0, 0][sl], 1 + b + d * Y[sl], rtol=0, atol=1e-12)
    np.testing.assert_allclose(F[0, 1][sl], c + d * X[sl], rtol=0, atol=1e-12)
    np.testing.assert_allclose(F[1, 0][sl], 0.005 - 3e-4 * Y[sl], rtol=0, atol=1e-12)
    np.testing.assert_allclose(F[1, 1][sl], 1 + 0.017 - 3e-4 * X[sl], rtol=0, atol=1e-12)
    # an incomplete window (grid edge) gives no value
    assert np.isnan(F[:, :, :r, :]).all() and np.isnan(F[:, :, :, -r:]).all()


def test_biquadratic_reproduces_biquadratic_fields():
    # every term of the 9-term tensor basis, and derivatives by hand at each node
    k = np.array([0.3, 0.01, -0.02, 1e-3, 2e-3, -1.5e-3, 1e-5, -2e-5, 3e-7])

    def fu(X, Y):
        return (k[0] + k[1] * X + k[2] * Y + k[3] * X * Y + k[4] * X * X + k[5] * Y * Y + k[6] * X * X * Y
                + k[7] * X * Y * Y + k[8] * X * X * Y * Y)
    u, v, X, Y = _grid(11, 11, 2, fu, lambda X, Y: -fu(Y, X))
    F = S.deformation_gradient(u, v, 2, 7, "biquadratic")
    dudx = k[1] + k[3] * Y + 2 * k[4] * X + 2 * k[6] * X * Y + k[7] * Y * Y + 2 * k[8] * X * Y * Y
    dudy = k[2] + k[3] * X + 2 * k[5] * Y + k[6] * X * X + 2 * k[7] * X * Y + 2 * k[8] * X * X * Y
    sl = (slice(3, -3), slice(3, -3))
    np.testing.assert_allclose(F[0, 0][sl], 1 + dudx[sl], atol=1e-10)
    np.testing.assert_allclose(F[0, 1][sl], dudy[sl], atol=1e-10)
    # v(x, y) = -u(y, x): dv/dx = -dudy(y, x), dv/dy = -dudx(y, x)
    np.testing.assert_allclose(F[1, 0][sl], -dudy.T[sl], atol=1e-10)
    np.testing.assert_allclose(F[1, 1][sl], 1 - dudx.T[sl], atol=1e-10)


def test_bilinear_smooths_a_quadratic_term_out_symmetrically():
    # on a full symmetric window the x^2 term is orthogonal to x and y, so the
    # bilinear fit's derivative at the centre is the exact one
    u, v, X, Y = _grid(9, 9, 1, lambda X, Y: 0.02 * X + 1e-3 * (X - 4) ** 2, lambda X, Y: 0.0 * X)
    F = S.deformation_gradient(u, v, 1, 5, "bilinear")
    np.testing.assert_allclose(F[0, 0][2:-2, 2:-2], 1 + 0.02 + 2e-3 * (X[2:-2, 2:-2] - 4), atol=1e-12)


def test_invalid_nodes_blank_their_windows():
    u, v, _, _ = _grid(9, 9, 1, lambda X, Y: 0.01 * X, lambda X, Y: 0.0 * X)
    valid = np.ones_like(u, bool)
    valid[4, 4] = False
    F = S.deformation_gradient(u, v, 1, 3, "bilinear", valid)
    assert np.isnan(F[0, 0, 3:6, 3:6]).all()
    assert np.isfinite(F[0, 0, 2, 2]) and np.isfinite(F[0, 0, 6, 6])
    u[1, 1] = np.nan
    F = S.deformation_gradient(u, v, 1, 3, "bilinear")
    assert np.isnan(F[0, 0, 1, 1]) and np.isnan(F[0, 0, 2, 2]) and np.isfinite(F[0, 0, 3, 3])


@pytest.mark.parametrize("lam1, lam2", [(1.1, 0.95), (1.0, 1.0), (1.3, 1.3), (0.8, 1.05)])
def test_stretch_closed_forms(lam1, lam2):
    F = np.diag([lam1, lam2])
    L = np.array([lam1, lam2])
    exp = {"green_lagrange": 0.5 * (L ** 2 - 1), "hencky": np.log(L), "euler_almansi": 0.5 * (1 - 1 / L ** 2),
           "biot_right": L - 1, "biot_left": L - 1}
    for m in S.MEASURES:
        np.testing.assert_allclose(S.strain_tensor(F, m), np.diag(exp[m]), atol=1e-14, err_msg=m)


@pytest.mark.parametrize("theta", [0.0, 0.3, -1.1])
def test_rotation_alone_strains_nothing_and_biot_sees_the_stretch(theta):
    c, s = np.cos(theta), np.sin(theta)
    R = np.array([[c, -s], [s, c]])
    for m in S.MEASURES:
        np.testing.assert_allclose(S.strain_tensor(R, m), 0.0, atol=1e-14, err_msg=m)
    U = np.array([[1.08, 0.03], [0.03, 0.97]])   # right stretch
    F = R @ U
    np.testing.assert_allclose(S.strain_tensor(F, "biot_right"), U - np.eye(2), atol=1e-13)
    np.testing.assert_allclose(S.strain_tensor(F, "biot_left"), R @ U @ R.T - np.eye(2), atol=1e-13)
    np.testing.assert_allclose(S.strain_tensor(F, "green_lagrange"), 0.5 * (U @ U - np.eye(2)), atol=1e-13)


@pytest.mark.parametrize("g", [0.0, 0.05, 0.4])
def test_simple_shear_closed_forms(g):
    F = np.array([[1.0, g], [0.0, 1.0]])
    np.testing.assert_allclose(S.strain_tensor(F, "green_lagrange"), [[0, g / 2], [g / 2, g * g / 2]], atol=1e-15)
    np.testing.assert_allclose(S.strain_tensor(F, "euler_almansi"), [[0, g / 2], [g / 2, -g * g / 2]], atol=1e-15)
    # Hencky: eigenvalues of C = F^T F are ((2+g^2) +- g sqrt(4+g^2))/2, the log
    # stretches +-asinh(g/2); the trace of ln U is ln det U = 0
    H = S.strain_tensor(F, "hencky")
    assert abs(np.trace(H)) < 1e-14
    np.testing.assert_allclose(np.linalg.eigvalsh(H), [-np.arcsinh(g / 2), np.arcsinh(g / 2)], atol=1e-14)


def test_matrix_functions_against_scipy():
    rng = np.random.default_rng(3)
    for _ in range(20):
        F = np.eye(2) + rng.uniform(-0.2, 0.2, (2, 2))
        C, B = F.T @ F, F @ F.T
        np.testing.assert_allclose(S.strain_tensor(F, "biot_right"), scipy.linalg.sqrtm(C).real - np.eye(2),
                                   atol=1e-12)
        np.testing.assert_allclose(S.strain_tensor(F, "biot_left"), scipy.linalg.sqrtm(B).real - np.eye(2),
                                   atol=1e-12)
        np.testing.assert_allclose(S.strain_tensor(F, "hencky"), 0.5 * scipy.linalg.logm(C).real, atol=1e-12)


def test_strain_of_a_uniform_affine_field():
    # u = 0.02 x + 0.01 y, v = -0.005 x + 0.03 y: every complete window gives the same F
    u, v, _, _ = _grid(8, 7, 4, lambda X, Y: 0.02 * X + 0.01 * Y, lambda X, Y: -0.005 * X + 0.03 * Y)
    F, eps = S.strain(u, v, 4, 3, "biquadratic", "green_lagrange")
    F0 = np.array([[1.02, 0.01], [-0.005, 1.03]])
    E0 = 0.5 * (F0.T @ F0 - np.eye(2))
    np.testing.assert_allclose(eps[0, 1:-1, 1:-1], E0[0, 0], atol=1e-12)
    np.testing.assert_allclose(eps[1, 1:-1, 1:-1], E0[0, 1], atol=1e-12)
    np.testing.assert_allclose(eps[2, 1:-1, 1:-1], E0[1, 1], atol=1e-12)
    assert np.isnan(eps[:, 0]).all()
