"""Edge cases of the entry points around the path, through the C ABI against
the oracle: out-of-core correlation of float pixels with no ROI and with
one-node-row bands; the multi-window guess on float pixels."""
import numpy as np
import pytest

import oracle
from oracle import chunked as CH
from paper_2601_12941_amd import dic, synth

from gpu_common import compare

pytestmark = pytest.mark.gpu


def _float_pair(W, H, field, seed):
    X, Y, S, A = synth.draw_blobs(W, H, int(0.03 * W * H), (1.5, 3.0), (60.0, 200.0), seed)
    ref = synth._render_blobs(W, H, X, Y, S, A)
    u, v = field(X, Y)
    de = synth._render_blobs(W, H, X + u, Y + v, S, A)
    rng = np.random.default_rng(seed + 1)
    ref = (ref + rng.normal(0.0, 1.5, ref.shape)).astype(np.float32)
    de = (de + rng.normal(0.0, 1.5, de.shape)).astype(np.float32)
    return ref, de


@pytest.mark.parametrize("band_rows, halo", [(6, 12), (1, 10)])
def test_chunked_float_pixels_without_roi(band_rows, halo):
    # no ROI: every subset inside the image is active; bands of one node row are
    # their own first and last rows
    ref, de = _float_pair(160, 136, synth.field_affine(0.6, -0.9, 0.004, 0.0, 0.0, 0.006, 80, 68), 41)
    prm = dict(subset_size=17, step=4, seed_radius=4)
    seeds = [(80, 68, 1, -1)]
    eng = dic.Engine(0)
    print("GPU case: chunked f32 no ROI", band_rows, halo, flush=True)
    g = eng.correlate_chunked(ref, de, None, seeds=seeds, band_rows=band_rows, halo=halo, boundary_seeds=6, **prm)
    eng.close()
    o = CH.correlate_chunked(ref, de, None, seeds=seeds, band_rows=band_rows, halo=halo, boundary_seeds=6,
                             threads=8, **prm)
    rep = compare(g, o)
    assert rep["both_converged"] > 0.9 * rep["active"]


def test_multiwindow_float_pixels():
    import torch
    W = 384
    f = synth.field_affine(0.1526 * W, -0.0915 * W, dudx=0.01, dvdy=-0.005, xc=W / 2.0, yc=W / 2.0)
    ref, de = _float_pair(W, W, f, 61)
    roi = synth.roi_from_field(W, W, f)
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(ref), torch.from_numpy(roi).cuda(), subset_size=31, step=8)
    print("GPU case: multiwindow f32", W, flush=True)
    r = eng.multiwindow(dic.to_device_image(de), max_disp=120, subpixel=True)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}
    eng.close()
    o = oracle.multiwindow(ref, de, roi, subset_size=31, step=8, max_disp=120, subpixel=True)
    assert g["levels"] == o["levels"]
    assert np.array_equal(g["valid"].astype(bool), o["valid"])
    ok = o["valid"]
    same = (np.round(g["u"]) == np.round(o["u"])) & (np.round(g["v"]) == np.round(o["v"]))
    assert same[ok].mean() >= 0.995
    both = ok & same
    assert np.maximum(np.abs(g["u"] - o["u"]), np.abs(g["v"] - o["v"]))[both].max() <= 5e-3


def test_widest_reference_within_32_bit_offsets():
    """The wave kernel addresses a subset's reference rows (interpolant and gradient
    interleaved, 12 bytes per pixel) with 32-bit offsets from the subset's corner.
    A reference whose 31 rows pass 2^31 bytes is refused before any work; one just
    inside is correlated against itself, so every active subset's rows reach
    offsets within 4 % of 2^31, and every one of them must converge to exactly
    zero displacement (an identical deformed subset gives a zero increment, Eq. (5)
    with p = 0, ZNCC 1)."""
    import torch
    N, H, step = 31, 40, 15
    rng = np.random.default_rng(2601)
    for W, accepted in ((5_800_000, False), (5_760_000, True)):
        assert (12 * W * N > 2**31 - 1) != accepted   # both widths are multiples of 64
        img = torch.from_numpy(rng.integers(0, 256, size=(H, W), dtype=np.uint8)).cuda()
        eng = dic.Engine(0)
        try:
            if not accepted:
                with pytest.raises(dic.DicError) as e:
                    eng.set_reference(img, subset_size=N, step=step)
                assert e.value.code == dic.DIC_E_INVAL
                continue
            nx, ny = eng.set_reference(img, subset_size=N, step=step)[:2]
            assert ny == 1
            h = (N - 1) // 2
            seeds = [(h + step * int(i), h, 0.0, 0.0) for i in np.linspace(1, nx - 2, 64)]
            out = eng.correlate(img, seeds)
            torch.cuda.synchronize()
            st = out["status"].cpu().numpy()
            p = out["p"].cpu().numpy()
            zn = out["zncc"].cpu().numpy()
            assert np.all(st == 0)
            assert np.all(p == 0.0)
            assert np.all(zn == 1.0)
        finally:
            eng.close()
            del img
            torch.cuda.empty_cache()
