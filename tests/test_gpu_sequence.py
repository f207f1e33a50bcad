"""GPU parity of multi-frame correlation with reference updating
(dic_correlate_sequence through the C ABI) against the sequence oracle on the
same seeded frames: the same reference chosen for every frame, every frame's
accumulated result node by node; the first frame bitwise equal to a plain
correlation; and the argument checks."""
import numpy as np
import pytest

from oracle import sequence as S
from paper_2601_12941_amd import dic, synth

from gpu_common import compare

pytestmark = pytest.mark.gpu


def _stretch_sequence(W=192, frames=6, per=0.04, seed=77):
    X, Y, Sg, A = synth.draw_blobs(W, W, int(0.03 * W * W), (1.5, 3.0), (60, 200), seed)
    ref = synth._finish(synth._render_blobs(W, W, X, Y, Sg, A), 2.0, seed + 1, 8)
    out = []
    for k in range(frames):
        f = synth.field_affine(0.0, 0.0, dudx=per * k, dvdy=per * k, xc=W / 2, yc=W / 2)
        u, v = f(X, Y)
        out.append(synth._finish(synth._render_blobs(W, W, X + u, Y + v, Sg, A), 2.0, seed + 2 + k, 8))
    roi = np.zeros((W, W), np.uint8)
    roi[40:W - 40, 40:W - 40] = 1
    return ref, out, roi


@pytest.mark.parametrize("shape", [2, 6])
def test_sequence_with_updates_parity(shape):
    import torch
    ref, frames, roi = _stretch_sequence()
    prm = dict(subset_size=21, step=4, shape=shape, seed_radius=3)
    seeds = [(96, 96, 0, 0)]
    eng = dic.Engine(0)
    d_roi = torch.from_numpy(roi).cuda()
    eng.set_reference(dic.to_device_image(ref), d_roi, **prm)
    print("GPU case: sequence, shape", shape, flush=True)
    outs, refs = eng.correlate_sequence([dic.to_device_image(f) for f in frames], seeds, d_roi,
                                        min_converged=0.9, min_zncc=0.999)
    torch.cuda.synchronize()
    o, orefs = S.correlate_sequence(ref, frames, roi, seeds=seeds, min_converged=0.9, min_zncc=0.999, threads=8,
                                    **prm)
    print("references:", refs, orefs, flush=True)
    assert refs == orefs and refs[-1] >= 1
    for g, r in zip(outs, o):
        g = {k: v.cpu().numpy() for k, v in g.items()}
        r = dict(r, subset_size=21, step=4)
        compare(g, r, npar=shape, wave_agree=0.99)
    eng.close()


def test_sequence_without_updates_starts_as_a_plain_correlation():
    import torch
    ref, frames, roi = _stretch_sequence(frames=3, per=0.01)
    prm = dict(subset_size=21, step=4, seed_radius=3)
    eng = dic.Engine(0)
    d_roi = torch.from_numpy(roi).cuda()
    eng.set_reference(dic.to_device_image(ref), d_roi, **prm)
    plain = eng.correlate(dic.to_device_image(frames[0]), [(96, 96, 0, 0)])
    outs, refs = eng.correlate_sequence([dic.to_device_image(f) for f in frames], [(96, 96, 0, 0)], d_roi,
                                        update=False)
    torch.cuda.synchronize()
    assert refs == [-1, -1, -1]
    for k in plain:
        assert torch.equal(plain[k], outs[0][k]), k
    o, _ = S.correlate_sequence(ref, frames, roi, seeds=[(96, 96, 0, 0)], update=False, threads=8, **prm)
    for g, r in zip(outs, o):
        compare({k: v.cpu().numpy() for k, v in g.items()}, dict(r, subset_size=21, step=4))
    eng.close()


def test_sequence_argument_checks():
    import torch
    ref, frames, roi = _stretch_sequence(frames=2)
    eng = dic.Engine(0)
    d_roi = torch.from_numpy(roi).cuda()
    eng.set_reference(dic.to_device_image(ref), d_roi, subset_size=21, step=4, shape=12)
    with pytest.raises(dic.DicError) as e:
        eng.correlate_sequence([dic.to_device_image(f) for f in frames], [(96, 96, 0, 0)], d_roi)
    assert e.value.code == dic.DIC_E_UNSUPPORTED
    eng.set_reference(dic.to_device_image(ref), d_roi, subset_size=21, step=4)
    with pytest.raises(dic.DicError) as e:
        eng.correlate_sequence([dic.to_device_image(frames[0][:-1])], [(96, 96, 0, 0)], d_roi)
    assert e.value.code == dic.DIC_E_INVAL
    eng.close()
