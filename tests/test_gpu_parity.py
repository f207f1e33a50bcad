"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs, element by element, plus the properties that hold at any
size (exact zero displacement, determinism, batch == plain)."""
import numpy as np
import pytest

from oracle import ST
from paper_2601_12941_amd import synth

from gpu_common import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    w = synth.workload("c1")
    return w, w.pair()


def test_c1_full_size_parity(c1):
    # 512^2 u8, subset 21, step 5, affine: 99^2 nodes, several tiles, ragged edges
    w, pair = c1
    g, _ = gpu_run(pair, w)
    o = oracle_run(pair, w)
    rep = compare(g, o)
    assert rep["both_converged"] > 9000
    assert g["stats"]["converged"] == int((g["status"] == ST["CONVERGED"]).sum())


def test_c1_fp32_reductions_parity(c1):
    w, pair = c1
    g, _ = gpu_run(pair, w, reduce_fp64=False)
    compare(g, oracle_run(pair, w))


@pytest.mark.parametrize("tps", [64, 128, 256])
def test_c1_every_workgroup_size_parity(c1, tps):
    w, pair = c1
    g, _ = gpu_run(pair, w, threads_per_subset=tps)
    compare(g, oracle_run(pair, w))


def test_zero_displacement_is_exactly_zero():
    w = synth.workload("c1", size=160)
    pair = w.pair()
    pair.deformed = pair.ref.copy()
    g, _ = gpu_run(pair, w)
    act = g["status"] != ST["NOT_IN_ROI"]
    assert np.all(g["status"][act] == ST["CONVERGED"])
    assert np.all(g["p"][:, act] == 0.0)
    assert np.all(g["iters"][act] == 1)
    # equal reference and deformed sums give a ratio of 1 and a ZNCC of exactly 1
    assert np.all(g["zncc"][act] == 1.0)


def test_repeat_runs_are_bitwise_identical(c1):
    w, pair = c1
    a, eng = gpu_run(pair, w)
    b, _ = gpu_run(pair, w, engine=eng)
    for k in ("p", "zncc", "iters", "status", "wave"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("nframes", [3, 8, 16, 32, 40, 64])
def test_batch_equals_plain(nframes):
    # 8, 16 and 32 frames take the kernel's frame-to-XCD affinity (every 8th frame on
    # one XCD group), 3 frames the plain grid stride; both must give every frame
    # bitwise the results of its own plain call
    import torch
    from paper_2601_12941_amd import dic
    w = synth.workload("c1", size=256)
    ref, frames, roi = synth.noise_frames(w, nframes)
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(ref), torch.from_numpy(roi).cuda(), **w.params())
    plain = [eng.correlate(dic.to_device_image(f), w.seeds) for f in frames]
    batch = eng.correlate_batch([dic.to_device_image(f) for f in frames], w.seeds)
    st = eng.stats()
    # 16, 32 and 64 frames, and any count above 32 (one launch carries at most 32),
    # run as two launch chains of half the frames on two streams; a second call
    # reuses the frame buffers the first call's chains wrote
    assert st["frames"] == nframes and st["launch_chains"] == (2 if nframes % 16 == 0 or nframes > 32 else 1)
    again = eng.correlate_batch([dic.to_device_image(f) for f in frames], w.seeds)
    torch.cuda.synchronize()
    for a, b, c in zip(plain, batch, again):
        for k in a:
            assert torch.equal(a[k], b[k]), k
            assert torch.equal(a[k], c[k]), k


def test_batch_chains_that_end_apart_equal_plain():
    # 16 frames in two launch chains whose frontiers end at different waves: the first
    # chain's frames are seeded at the centre, the second chain's near a corner (about
    # twice the waves), so the first chain stops while the second still launches waves
    # and look-ahead launches; every frame must equal its own plain call
    import torch
    from paper_2601_12941_amd import dic
    w = synth.workload("c1", size=256)
    ref, frames, roi = synth.noise_frames(w, 16)
    centre, corner = [(128.0, 128.0, 0.0, 0.0)], [(40.0, 40.0, 0.0, 0.0)]
    seeds = [centre if f < 8 else corner for f in range(16)]
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(ref), torch.from_numpy(roi).cuda(), **w.params())
    plain, waves = [], []
    for f, fr in enumerate(frames):
        plain.append(eng.correlate(dic.to_device_image(fr), seeds[f]))
        waves.append(eng.stats()["waves"])
    assert max(waves[8:]) > max(waves[:8]) + 10
    batch = eng.correlate_batch([dic.to_device_image(f) for f in frames], seeds)
    st = eng.stats()
    assert st["launch_chains"] == 2 and st["waves"] == max(waves)
    torch.cuda.synchronize()
    for a, b in zip(plain, batch):
        for k in a:
            assert torch.equal(a[k], b[k]), k


def test_batch_frame_limit():
    import torch
    from paper_2601_12941_amd import dic
    w = synth.workload("c1", size=128)
    pair = w.pair()
    eng = dic.Engine(0)
    eng.set_reference(dic.to_device_image(pair.ref), torch.from_numpy(pair.roi).cuda(), **w.params())
    d = dic.to_device_image(pair.deformed)
    with pytest.raises(dic.DicError) as e:
        eng.correlate_batch([d] * 65, w.seeds)
    assert e.value.code == dic.DIC_E_INVAL
    eng.close()
