"""Pins of the sequence oracle (paper Sec. 6, reference updating): the
Lagrangian accumulation reproduces the composition of two affine maps exactly
(bilinear interpolation is exact on affine fields), is the identity against
the original reference, and marks what it cannot reach; the update rule fires
on a quality drop and the accumulated result follows a large stretch."""
import numpy as np

import oracle
from oracle import sequence as S
from paper_2601_12941_amd import synth

from test_oracle_icgn import speckle


def _field_result(nx, ny, N, step, A, b, npar=6):
    """A result dict holding the affine displacement u(X) = A X + b at the nodes."""
    h = (N - 1) // 2
    X, Y = np.meshgrid(h + step * np.arange(nx, dtype=float), h + step * np.arange(ny, dtype=float))
    p = np.zeros((12, ny, nx))
    p[0] = A[0, 0] * X + A[0, 1] * Y + b[0]
    p[1] = A[1, 0] * X + A[1, 1] * Y + b[1]
    if npar >= 6:
        p[2], p[3], p[4], p[5] = A[0, 0], A[0, 1], A[1, 0], A[1, 1]
    return dict(p=p, zncc=np.full((ny, nx), 0.99), iters=np.full((ny, nx), 3, np.int32),
                status=np.zeros((ny, nx), np.int32), wave=np.zeros((ny, nx), np.int32)), X, Y


def test_accumulation_composes_affine_maps_exactly():
    # reference state: X -> X + A1 X + b1; increment on the same grid: x -> x + A2 x + b2
    N, step, nx, ny = 21, 5, 40, 30
    A1, b1 = np.array([[0.02, 0.01], [-0.005, 0.03]]), np.array([3.3, -2.1])
    A2, b2 = np.array([[-0.01, 0.004], [0.006, 0.015]]), np.array([-1.2, 0.7])
    ref, X, Y = _field_result(nx, ny, N, step, A1, b1)
    inc, _, _ = _field_result(nx, ny, N, step, A2, b2)
    out = S.accumulate(ref, inc, N, step, 6)
    # total map: X -> (I + A2)(X + A1 X + b1) + b2
    x1 = X + A1[0, 0] * X + A1[0, 1] * Y + b1[0]
    y1 = Y + A1[1, 0] * X + A1[1, 1] * Y + b1[1]
    ut = x1 + A2[0, 0] * x1 + A2[0, 1] * y1 + b2[0] - X
    vt = y1 + A2[1, 0] * x1 + A2[1, 1] * y1 + b2[1] - Y
    ok = out["status"] == 0
    assert ok.sum() > 0.8 * nx * ny
    np.testing.assert_allclose(out["p"][0][ok], ut[ok], atol=1e-9)
    np.testing.assert_allclose(out["p"][1][ok], vt[ok], atol=1e-9)
    G = (np.eye(2) + A2) @ (np.eye(2) + A1) - np.eye(2)
    for k, (a, b) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        np.testing.assert_allclose(out["p"][2 + k][ok], G[a, b], atol=1e-12)
    # nodes carried off the increment's grid are not reached
    assert np.all(out["status"][~ok] == S.NOT_REACHED)
    x1n, y1n = (x1 - 10) / step, (y1 - 10) / step
    outside = (x1n < 0) | (y1n < 0) | (x1n > nx - 1) | (y1n > ny - 1)
    assert np.array_equal(~ok, outside)


def test_accumulation_against_the_original_reference_is_the_identity():
    N, step, nx, ny = 15, 4, 12, 9
    inc, _, _ = _field_result(nx, ny, N, step, np.array([[0.01, 0.0], [0.0, -0.02]]), np.array([1.5, 2.5]))
    inc["status"][3, 4] = 3
    inc["status"][0, 0] = 2
    inc["p"][:, 3, 4] = np.nan
    out = S.accumulate(None, inc, N, step, 6)
    assert np.array_equal(out["status"], inc["status"])
    act = inc["status"] != 2
    for k in ("zncc", "iters", "wave"):
        assert np.array_equal(out[k][act], inc[k][act]), k
    np.testing.assert_array_equal(out["p"][:6, act], inc["p"][:6, act])


def test_unconverged_reference_nodes_are_not_reached():
    N, step, nx, ny = 15, 4, 10, 10
    ref, _, _ = _field_result(nx, ny, N, step, np.zeros((2, 2)), np.array([0.5, 0.5]))
    ref["status"][5, 5] = 3
    inc, _, _ = _field_result(nx, ny, N, step, np.zeros((2, 2)), np.array([1.0, 0.0]))
    inc["status"][2, 2] = 4
    out = S.accumulate(ref, inc, N, step, 6)
    assert out["status"][5, 5] == S.NOT_REACHED
    # node (1, 1) sits at (1.125, 1.125) cells: its cell's far corner (2, 2) is LOW_ZNCC
    assert out["status"][1, 1] == 4
    assert out["status"][3, 3] == 0 and abs(out["p"][0, 3, 3] - 1.5) < 1e-12


def test_sequence_updates_the_reference_under_a_large_stretch():
    # frames stretched by 0, 4, 8, ... 20 % about the centre (rendered speckle): with a
    # ZNCC threshold the reference moves along the sequence, and the accumulated
    # displacement follows the field
    W = 192
    X, Y, Sg, A = synth.draw_blobs(W, W, int(0.03 * W * W), (1.5, 3.0), (60, 200), 77)
    ref = synth._render_blobs(W, W, X, Y, Sg, A)
    frames, fields = [], []
    for k in range(6):
        f = synth.field_affine(0.0, 0.0, dudx=0.04 * k, dvdy=0.04 * k, xc=W / 2, yc=W / 2)
        u, v = f(X, Y)
        frames.append(synth._render_blobs(W, W, X + u, Y + v, Sg, A))
        fields.append(f)
    roi = np.zeros((W, W), np.uint8)
    roi[40:152, 40:152] = 1
    prm = dict(subset_size=21, step=4, shape=6, seed_radius=3)
    res, refs = S.correlate_sequence(ref, frames, roi, seeds=[(96, 96, 0, 0)], min_converged=0.9, min_zncc=0.999,
                                     **prm)
    assert refs[0] == -1 and refs[-1] >= 1 and refs == sorted(refs)
    res0, refs0 = S.correlate_sequence(ref, frames, roi, seeds=[(96, 96, 0, 0)], update=False, **prm)
    assert refs0 == [-1] * 6
    # the rendered blobs keep their shape under the stretch, an error that grows with
    # the strain alike with and without updates; the updates keep the correlation
    # against the current reference near 1 where the original reference decorrelates
    for r, r0, f in zip(res, res0, fields):
        ok, ok0 = r["status"] == 0, r0["status"] == 0
        assert ok.sum() > 300
        u, v, _ = synth.truth_at_nodes(f, W, W, 21, 4)
        e = np.hypot(r["p"][0] - u, r["p"][1] - v)[ok]
        e0 = np.hypot(r0["p"][0] - u, r0["p"][1] - v)[ok0]
        assert np.sqrt(np.mean(e ** 2)) <= 1.2 * np.sqrt(np.mean(e0 ** 2)) + 0.005
    assert S.quality(res[-1])[1] > 0.999 > S.quality(res0[-1])[1]
    print("reference of each frame:", refs)
