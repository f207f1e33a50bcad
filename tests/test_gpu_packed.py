"""Packed subsets on the GPU: with 16 or 32 threads per subset, four or two
small subsets share one wavefront. Same parity bar against the FP64 oracle,
the exact zero for identical images, and batch == plain."""
import numpy as np
import pytest
import torch

from paper_2601_12941_amd import dic, synth
from gpu_common import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    # the 512^2 u8 recipe at 256^2 with 15-pixel subsets on a 3-pixel step
    w = synth.workload("c1", size=256, N=15, step=3)
    return w, w.pair()


@pytest.mark.parametrize("tps", [16, 32])
def test_packed_parity(small, tps):
    w, pair = small
    g, eng = gpu_run(pair, w, threads_per_subset=tps)
    assert g["stats"]["threads_per_subset"] == tps
    compare(g, oracle_run(pair, w))
    eng.close()


@pytest.mark.parametrize("N,tps", [(9, 16), (9, 32), (5, 32), (13, 16)])
def test_packed_other_sizes_parity(N, tps):
    w = synth.workload("c1", size=192, N=N, step=4)
    pair = w.pair()
    g, eng = gpu_run(pair, w, threads_per_subset=tps)
    compare(g, oracle_run(pair, w))
    eng.close()


def test_packed_exact_zero_and_batch():
    w = synth.workload("c1", size=192, N=15, step=3)
    pair = w.pair()
    ref = dic.to_device_image(pair.ref)
    de = dic.to_device_image(pair.deformed)
    roi = torch.from_numpy(np.ascontiguousarray(pair.roi)).cuda()
    eng = dic.Engine(0)
    eng.set_reference(ref, roi, **w.params(), threads_per_subset=16)
    z = eng.correlate(ref, [(96.0, 96.0, 0.0, 0.0)])
    torch.cuda.synchronize()
    st = z["status"].cpu().numpy()
    conv = st == 0
    assert conv.sum() > 0.9 * (st != 2).sum()
    assert np.all(z["p"].cpu().numpy()[:, conv] == 0.0)
    assert np.all(z["zncc"].cpu().numpy()[conv] == 1.0)
    plain = eng.correlate(de, w.seeds)
    torch.cuda.synchronize()
    plain = {k: v.cpu().numpy() for k, v in plain.items()}
    batch = eng.correlate_batch([de, de, de], w.seeds)
    torch.cuda.synchronize()
    for b in batch:
        for k in ("p", "zncc", "iters", "status", "wave"):
            assert np.array_equal(b[k].cpu().numpy(), plain[k], equal_nan=True), k
    eng.close()


def test_packed_rejects_quadratic_and_large_subsets():
    w = synth.workload("c1", size=128, N=21)
    pair = w.pair()
    eng = dic.Engine(0)
    ref = dic.to_device_image(pair.ref)
    with pytest.raises(dic.DicError):
        eng.set_reference(ref, None, **w.params(), threads_per_subset=16)   # N 21 > 16
    w15 = synth.workload("c1", size=128, N=15, shape=12)
    with pytest.raises(dic.DicError) as e:
        eng.set_reference(ref, None, **w15.params(), threads_per_subset=32)
    assert e.value.code == dic.DIC_E_UNSUPPORTED
    eng.close()
