"""GPU parity on reduced-size versions of every workload recipe (same speckle
statistics, fields, subset sizes and steps), the quadratic shape, FP16
coefficient storage, several seeds, every node status, the error paths of
the C ABI, and sampled parity at the full 2048^2 size."""
import numpy as np
import pytest

import oracle
from oracle import ST
from paper_2601_12941_amd import dic, synth

from gpu_common import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2_512():
    w = synth.workload("c2", size=512)
    pair = w.pair()
    return w, pair, oracle_run(pair, w)


# (threads per subset, window side): the library default (128 threads, 8-row
# register block), and the benchmark's batched shape (64 threads, 16-row block,
# the software-pipelined pixel loop, the smallest window)
@pytest.mark.parametrize("shape_args", [{}, dict(threads_per_subset=64, tile_side=36)])
def test_sine_field_12bit_parity(c2_512, shape_args):
    # 12-bit speckle, u = 0.5 sin(2 pi x / lambda(y)) with lambda 10..300 px over
    # the image height, subset 31, step 2
    w, pair, o = c2_512
    g, _ = gpu_run(pair, w, **shape_args)
    compare(g, o)
    assert g["stats"]["seed_du"] == int(o["seed_nodes"][0, 1]) and g["stats"]["seed_dv"] == int(o["seed_nodes"][0, 2])


@pytest.mark.parametrize("N, shape, tps", [(23, 6, 64), (35, 12, 128), (41, 6, 128), (51, 6, 256), (51, 12, 256)])
def test_pipelined_blocks_parity(N, shape, tps):
    # subsets that fill an 11-, 12- or 14-row register block exactly (the
    # software-pipelined pixel loop): 23 pixels at 64 threads and 35 at 128 (12
    # rows), 41 at 128 (14 rows), 51 at 256 (11 rows), affine and quadratic
    w = synth.workload("c3", size=384, N=N, shape=shape)
    pair = w.pair()
    g, _ = gpu_run(pair, w, threads_per_subset=tps)
    o = oracle_run(pair, w)
    compare(g, o, npar=shape)


@pytest.mark.parametrize("N, tps, tile", [(51, 256, 68), (61, 256, 96), (21, 64, 38)])
def test_window_sides_and_lds_pitch_parity(N, tps, tile):
    # windows wider than one 64-lane staging request (68 and 96 samples: two
    # requests per row), a padded LDS row pitch (68 at N 51 -> 83, 38 at N 21 ->
    # 53) and a window too large to pad (96 at N 61: pitch 96)
    w = synth.workload("c3", size=384, N=N, shape=6)
    pair = w.pair()
    g, _ = gpu_run(pair, w, threads_per_subset=tps, tile_side=tile)
    o = oracle_run(pair, w)
    compare(g, o)


@pytest.mark.parametrize("N", [21, 41])
@pytest.mark.parametrize("shape", [6, 12])
def test_quadratic_field_parity(N, shape):
    # u8, u = 1e-5 x~^2 + 0.3 + 0.02 x~, v = -2e-5 x~ y~ + 0.2 + 0.02 y~ about the centre, step 4
    w = synth.workload("c3", size=384, N=N, shape=shape)
    pair = w.pair()
    g, _ = gpu_run(pair, w)
    o = oracle_run(pair, w)
    compare(g, o, npar=shape)


@pytest.mark.parametrize("shape", [6, 12])
def test_fp16_coefficients_error_is_reported(shape):
    # FP16 storage of the deformed coefficients is an approximation: report its
    # error against the FP64 oracle (8-bit data: a few 1e-3 px)
    w = synth.workload("c3", size=384, shape=shape)
    pair = w.pair()
    g, _ = gpu_run(pair, w, coef_fp16=True)
    o = oracle_run(pair, w)
    rep = compare(g, o, npar=shape, tol_uv=2e-2, tol_zncc=2e-4, status_agree=0.99)
    print("fp16 coefficient error vs oracle:", rep)


def test_bump_field_many_seeds_parity():
    # rigid shift (3.41, -7.92) plus a Gaussian bump in u, subset 41, step 20, 16 seeds
    w = synth.workload("c4", size=1024)
    pair = w.pair()
    g, _ = gpu_run(pair, w)
    o = oracle_run(pair, w)
    rep = compare(g, o)
    assert (g["wave"] == 0).sum() == len(o["seed_nodes"]) == 16
    assert rep["wave_equal"] == 1.0


def test_guess_copy_mode_parity():
    w = synth.workload("c1", size=256)
    pair = w.pair()
    g, _ = gpu_run(pair, w, guess="copy")
    compare(g, oracle_run(pair, w, guess="copy"))


# ------------------------------------------------------------------ statuses
def _small_pair(field=None, size=160):
    w = synth.workload("c1", size=size)
    if field is not None:
        pair = synth.make_pair(w.W, w.H, w.nblobs, w.sigma, w.amp, field, w.noise, w.bits, w.seed_blobs,
                               w.seed_noise_ref, w.seed_noise_def)
    else:
        pair = w.pair()
    return w, pair


def test_statuses_out_of_bounds_and_not_reached():
    # no ROI trimming: nodes near the right edge are pushed out of the image
    w, pair = _small_pair(synth.field_affine(6.3, 0.4))
    pair.roi = np.ones_like(pair.roi)
    g, _ = gpu_run(pair, w)
    o = oracle_run(pair, w)
    compare(g, o)
    assert (g["status"] == ST["OUT_OF_BOUNDS"]).sum() > 0


def test_statuses_flat_and_max_iter_and_low_zncc():
    # flat patches wide enough that some subsets (and their interpolation
    # support, which rings ~0.27^distance around speckle) lie well inside
    # one seed in textured speckle, one inside each flat patch (nodes that are
    # flat are otherwise walled off by partly flat neighbours that fail)
    w = synth.workload("c1", size=256, seeds=[(200, 200, 0, 0), (100, 100, 0, 0), (70, 200, 0, 0)])
    pair = w.pair()
    ref = pair.ref.copy()
    ref[60:150, 60:150] = 90
    de = pair.deformed.copy()
    de[150:250, 20:120] = 30
    pair.ref, pair.deformed = ref, de
    g, _ = gpu_run(pair, w)
    o = oracle_run(pair, w)
    compare(g, o, status_agree=0.995)
    assert (g["status"] == ST["FLAT_REF"]).sum() > 0 and (g["status"] == ST["FLAT_DEF"]).sum() > 0
    w2, pair2 = _small_pair()
    g2, _ = gpu_run(pair2, w2, max_iter=2)
    compare(g2, oracle_run(pair2, w2, max_iter=2))
    assert (g2["status"] == ST["MAX_ITER"]).sum() > 0
    g3, _ = gpu_run(pair2, w2, zncc_min=0.998)
    compare(g3, oracle_run(pair2, w2, zncc_min=0.998))
    assert (g3["status"] == ST["LOW_ZNCC"]).sum() > 0


def test_status_nan_from_float_pixels():
    w, pair = _small_pair()
    ref = pair.ref.astype(np.float32)
    de = pair.deformed.astype(np.float32)
    de[70, 75] = np.nan
    pair.ref, pair.deformed = ref, de
    g, _ = gpu_run(pair, w)
    o = oracle_run(pair, w)
    assert np.array_equal(g["status"] == ST["NAN"], o["status"] == ST["NAN"])
    assert (g["status"] == ST["NAN"]).sum() > 0


def test_nan_unconverged_flag():
    w, pair = _small_pair(synth.field_affine(6.3, 0.4))
    pair.roi = np.ones_like(pair.roi)
    g, _ = gpu_run(pair, w, nan_unconverged=True)
    bad = g["status"] != ST["CONVERGED"]
    assert bad.any()
    assert np.all(np.isnan(g["p"][:, bad])) and np.all(np.isfinite(g["p"][:, ~bad]))


# ------------------------------------------------------------------ errors
def test_error_paths():
    import torch
    w, pair = _small_pair()
    eng = dic.Engine(0)
    ref = dic.to_device_image(pair.ref)
    with pytest.raises(dic.DicError) as e:
        eng.grid = (10, 10, 0, 0, 1)
        eng.shape = 6
        eng.correlate(ref, w.seeds)
    assert e.value.code == dic.DIC_E_STATE
    prm = w.params()
    with pytest.raises(dic.DicError) as e:
        eng.set_reference(ref, None, **{**prm, "subset_size": 20})
    assert e.value.code == dic.DIC_E_INVAL
    with pytest.raises(dic.DicError) as e:
        eng.set_reference(ref, None, **{**prm, "shape": 12, "subset_size": 25, "threads_per_subset": 64})
    assert e.value.code == dic.DIC_E_UNSUPPORTED
    with pytest.raises(dic.DicError) as e:
        eng.set_reference(ref, None, **{**prm, "shape": 2, "threads_per_subset": 64})
    assert e.value.code == dic.DIC_E_INVAL
    with pytest.raises(dic.DicError) as e:
        eng.set_reference(ref, None, **{**prm, "cost": "ssd", "lm_lambda": -1.0})
    assert e.value.code == dic.DIC_E_INVAL
    eng.set_reference(ref, torch.from_numpy(pair.roi).cuda(), **prm)
    with pytest.raises(dic.DicError) as e:
        eng.correlate(dic.to_device_image(pair.deformed[:-1]), w.seeds)
    assert e.value.code == dic.DIC_E_INVAL
    empty = torch.zeros_like(torch.from_numpy(pair.roi)).cuda()
    eng.set_reference(ref, empty, **prm)
    with pytest.raises(dic.DicError) as e:
        eng.correlate(dic.to_device_image(pair.deformed), w.seeds)
    assert e.value.code == dic.DIC_E_NOSEED
    # the context stays usable after these errors
    eng.set_reference(ref, torch.from_numpy(pair.roi).cuda(), **prm)
    out = eng.correlate(dic.to_device_image(pair.deformed), w.seeds)
    assert int((out["status"] == 0).sum()) > 0
    eng.close()


# ------------------------------------------------------------------ full size
def test_full_size_2048_batched_parity():
    # The full 2048^2 12-bit pair, element by element against the FP64 oracle run
    # on the whole pair (WAVE order), in the benchmark's launch configuration: a
    # batched launch of 16 noise realisations (frames pinned to XCD groups), 64
    # threads per subset, a 36-sample window.  Frame 0 is the oracle's pair; every
    # Eq. (5) parameter, the ZNCC, the status and the wave index are compared.
    import torch
    w = synth.workload("c2")
    ref, frames, roi = synth.noise_frames(w, 16)
    eng = dic.Engine(0)
    print("GPU case: 2048^2 batched, 16 frames, 64 threads, window 36", flush=True)
    eng.set_reference(dic.to_device_image(ref), torch.from_numpy(roi).cuda(),
                      **{**w.params(), "threads_per_subset": 64, "tile_side": 36})
    outs = eng.correlate_batch([dic.to_device_image(f) for f in frames], w.seeds)
    torch.cuda.synchronize()
    st = eng.stats()
    g = {k: v.cpu().numpy() for k, v in outs[0].items()}
    o = oracle.correlate(ref, frames[0], roi, seeds=w.seeds, threads=16, **{
        k: v for k, v in w.params().items() if k not in ("coef_fp16", "reduce_fp64", "threads_per_subset",
                                                          "nan_unconverged", "tile_side")})
    rep = compare(g, o)
    assert st["waves"] > 900 and rep["both_converged"] > 0.99 * rep["active"]
    # frames 1..15 converge as well (their own noise, same field)
    for out in outs[1:]:
        assert int((out["status"] == 0).sum()) > 0.99 * rep["active"]
    eng.close()
