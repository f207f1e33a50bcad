"""GPU parity of the strain step (dic_strain through the C ABI) against the
FP64 strain oracle, element by element, on seeded displacement grids: every
window size, both bases, all five measures, invalid nodes, degenerate grids;
and the whole chain (correlation, then strain) against the ground-truth
strain of a quadratic field."""
import numpy as np
import pytest

from oracle import strain as S
from paper_2601_12941_amd import dic, synth

pytestmark = pytest.mark.gpu

# F and the strains are written in FP32 after FP64 arithmetic: the bar is a few
# FP32 units of F (~1) and far below any strain resolution DIC reaches
TOL = 1e-6


def _gpu(eng, u, v, status, step, window, basis, measure):
    import torch
    tu, tv = torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda()
    ts = torch.from_numpy(status).cuda() if status is not None else None
    out = eng.strain(tu, tv, ts, step=step, window=window, basis=basis, measure=measure)
    torch.cuda.synchronize()
    return out["F"].cpu().numpy(), out["eps"].cpu().numpy()


def _check(Fg, eg, Fo, eo):
    Fo4 = Fo.reshape(4, *Fo.shape[2:])
    assert np.array_equal(np.isnan(Fg), np.isnan(Fo4)), "valid-node maps differ (F)"
    assert np.array_equal(np.isnan(eg), np.isnan(eo)), "valid-node maps differ (strain)"
    ok = ~np.isnan(Fo4)
    if ok.any():
        assert np.abs(Fg[ok] - Fo4[ok]).max() <= TOL
        ok3 = ~np.isnan(eo)
        assert np.abs(eg[ok3] - eo[ok3]).max() <= TOL


@pytest.mark.parametrize("window", [3, 5, 9, 15])
@pytest.mark.parametrize("basis", ["bilinear", "biquadratic"])
def test_strain_parity_every_measure(window, basis):
    eng = dic.Engine(0)
    u, v, st = synth.displacement_grid(83, 61, 3, "smooth", noise=2e-3, invalid=0.01, seed=window)
    valid = st == 0
    print("GPU case: strain", window, basis, flush=True)
    for measure in S.MEASURES:
        Fo, eo = S.strain(u.astype(np.float64), v.astype(np.float64), 3, window, basis, measure, valid)
        Fg, eg = _gpu(eng, u, v, st, 3, window, basis, measure)
        _check(Fg, eg, Fo, eo)
    eng.close()


@pytest.mark.parametrize("kind", ["rotation", "shear"])
def test_strain_parity_large_rotation_and_shear(kind):
    # finite rotation and shear: the measures differ from each other at first order
    eng = dic.Engine(0)
    u, v, st = synth.displacement_grid(40, 33, 5, kind, seed=1)
    for measure in S.MEASURES:
        Fo, eo = S.strain(u.astype(np.float64), v.astype(np.float64), 5, 5, "bilinear", measure)
        Fg, eg = _gpu(eng, u, v, None, 5, 5, "bilinear", measure)
        _check(Fg, eg, Fo, eo)
    eng.close()


def test_strain_degenerate_grids():
    eng = dic.Engine(0)
    # exactly one complete window; then a grid narrower than the window (all NaN)
    u, v, st = synth.displacement_grid(7, 7, 2, "smooth", seed=2)
    Fo, eo = S.strain(u.astype(np.float64), v.astype(np.float64), 2, 7, "biquadratic", "hencky")
    Fg, eg = _gpu(eng, u, v, st, 2, 7, "biquadratic", "hencky")
    _check(Fg, eg, Fo, eo)
    assert np.isfinite(Fg[:, 3, 3]).all() and int(np.isfinite(Fg[0]).sum()) == 1
    u, v, st = synth.displacement_grid(4, 30, 2, "smooth", seed=3)
    Fg, eg = _gpu(eng, u, v, st, 2, 5, "bilinear", "green_lagrange")
    assert np.isnan(Fg).all() and np.isnan(eg).all()
    # NaN displacements (the library's nan_unconverged output) count as invalid without a status array
    u, v, _ = synth.displacement_grid(20, 20, 2, "smooth", seed=4)
    u[9, 9] = np.nan
    Fo, eo = S.strain(u.astype(np.float64), v.astype(np.float64), 2, 3, "bilinear", "biot_left")
    Fg, eg = _gpu(eng, u, v, None, 2, 3, "bilinear", "biot_left")
    _check(Fg, eg, Fo, eo)
    # bad arguments
    import torch
    t = torch.zeros((10, 10), dtype=torch.float32, device="cuda")
    for kw in (dict(window=4), dict(window=17), dict(basis="cubic")):
        with pytest.raises((dic.DicError, KeyError)):
            eng.strain(t, t, step=2, **kw)
    assert dic.dic_vsg(5, 2, 31) == S.vsg(5, 2, 31) == 39
    eng.close()


def test_correlation_then_strain_against_the_field():
    # the whole chain on the quadratic-field recipe (u8, subset 21, step 4): the
    # Green-Lagrange strain from the GPU's displacements, a 9-node bilinear window,
    # against the field's exact strain at the nodes
    import torch
    w = synth.workload("c3", size=384, N=21, shape=6)
    pair = w.pair()
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(pair.ref), torch.from_numpy(pair.roi).cuda(), **w.params())
    out = eng.correlate(dic.to_device_image(pair.deformed), w.seeds)
    res = eng.strain(out["p"][0].contiguous(), out["p"][1].contiguous(), out["status"], step=w.step, window=9,
                     basis="bilinear", measure="green_lagrange")
    torch.cuda.synchronize()
    eps = res["eps"].cpu().numpy()
    u, v, (ux, uy, vx, vy) = synth.truth_at_nodes(pair.field, w.W, w.H, w.N, w.step)
    exx = ux + 0.5 * (ux * ux + vx * vx)
    ok = np.isfinite(eps[0])
    assert ok.sum() > 1000
    # displacement noise ~0.01 px over a 32-px window half-width: ~1e-3 strain noise
    assert np.abs(eps[0][ok] - exx[ok]).mean() < 2e-3
    eng.close()
