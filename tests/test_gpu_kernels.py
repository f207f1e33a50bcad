"""Kernel-level GPU parity through the C ABI: the reference precompute
(prefilter coefficients, interpolant and gradient at every pixel, read back
with dic_reference_arrays) against the FP64 oracle's prefilter and
evaluation; and single subsets started from an identical shape (seeds with a
zero search radius at integer guesses) against the oracle's IC-GN from the
same start, for every shape and cost."""
import numpy as np
import pytest

import oracle
from oracle import ST
from paper_2601_12941_amd import dic, synth

pytestmark = pytest.mark.gpu


def _image(kind, W=131, H=97, seed=3):
    X, Y, S, A = synth.draw_blobs(W, H, int(0.012 * W * H), (2.0, 4.0), (60.0, 200.0), seed)
    img = synth._render_blobs(W, H, X, Y, S, A)
    if kind == "u8":
        return synth._finish(img, 2.0, seed + 1, 8)
    if kind == "u16":
        return synth._finish(img * 16.0, 4.0, seed + 1, 12)
    return (img + np.random.default_rng(seed).normal(0.0, 2.0, img.shape)).astype(np.float32)


@pytest.mark.parametrize("kind", ["u8", "u16", "f32"])
def test_reference_precompute_against_the_oracle(kind):
    import torch
    img = _image(kind)
    H, W = img.shape
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(img), None, subset_size=21, step=5)
    print("GPU case: reference arrays", kind, img.shape, flush=True)
    arr = eng.reference_arrays()
    torch.cuda.synchronize()
    coef = arr["coef"].cpu().numpy().astype(np.float64) * 36.0   # stored as 1/36 of the coefficients
    c_o = oracle.prefilter(img.astype(np.float64))
    scale = float(np.abs(img).max())
    assert np.abs(coef - c_o).max() <= 3e-6 * scale, np.abs(coef - c_o).max() / scale
    yy, xx = np.mgrid[0:H, 0:W]
    v, gx, gy = oracle.evaluate(c_o, xx.ravel().astype(float), yy.ravel().astype(float))
    for name, o in (("f", v), ("fx", gx), ("fy", gy)):
        g = arr[name].cpu().numpy().astype(np.float64).ravel()
        err = np.abs(g - o).max() / scale
        print(name, err, flush=True)
        assert err <= 4e-6, (name, err)
    # the interpolant reproduces the samples
    assert np.abs(arr["f"].cpu().numpy() - img.astype(np.float64)).max() <= 4e-6 * scale
    eng.close()


@pytest.mark.parametrize("shape, cost, lm", [(6, "znssd", 0.0), (12, "znssd", 0.0), (2, "znssd", 0.0),
                                             (6, "nssd", 0.0), (6, "ssd", 0.0), (6, "znssd", 1e-2)])
def test_single_subsets_from_an_identical_start(shape, cost, lm):
    import torch
    w = synth.workload("c1", size=256)
    pair = w.pair()
    prm = dict(subset_size=21, step=5, shape=shape, cost=cost, lm_lambda=lm, seed_radius=0, tol=1e-4)
    u, v, _ = synth.truth_at_nodes(pair.field, w.W, w.H, 21, 5)
    rng = np.random.default_rng(5)
    ny, nx = u.shape
    pick = [(int(j), int(i)) for j, i in zip(rng.integers(4, ny - 4, 24), rng.integers(4, nx - 4, 24))]
    pick = sorted(set(pick))
    seeds = [(10 + 5 * i, 10 + 5 * j, float(np.round(u[j, i])), float(np.round(v[j, i]))) for j, i in pick]
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(pair.ref), torch.from_numpy(pair.roi).cuda(), **prm)
    print("GPU case: single subsets", shape, cost, lm, len(seeds), flush=True)
    g = {k: t.cpu().numpy() for k, t in eng.correlate(dic.to_device_image(pair.deformed), seeds).items()}
    eng.close()
    h = 10.0
    scale = np.array([1, 1] + [h] * 4 + [h * h] * 6)[:shape]
    same_it = 0
    for (j, i), sd in zip(pick, seeds):
        assert g["wave"][j, i] == 0
        p0 = np.zeros(shape)
        p0[0], p0[1] = sd[2], sd[3]
        po, zo, ito, sto = oracle.icgn(pair.ref, pair.deformed, sd[0], sd[1], p0, 21, shape, tol=1e-4, max_iter=50,
                                       cost=cost, lm_lambda=lm)
        assert g["status"][j, i] == sto, (j, i, g["status"][j, i], sto)
        if sto != ST["CONVERGED"]:
            continue
        d = np.abs(g["p"][:shape, j, i] - po[:shape]) * scale
        assert d.max() <= 1e-3, (j, i, d)
        assert abs(g["zncc"][j, i] - zo) <= 1e-5
        same_it += int(g["iters"][j, i] == ito)
    print("iterations equal on", same_it, "of", len(pick), flush=True)
    assert same_it >= 0.9 * len(pick)
