"""dic_correlate_noalloc through the C ABI against dic_correlate: two calls in
a row (the second on a smaller input) give bitwise the same results, a
reference whose scratch exceeds the array is refused before any work, and the
context stays usable afterwards."""
import numpy as np
import pytest

from paper_2601_12941_amd import dic, synth

pytestmark = pytest.mark.gpu


def _setup(eng, size, seed_shift=0):
    import torch
    w = synth.workload("c1", size=size)
    ref, frames, roi = synth.noise_frames(w, 1 + seed_shift)
    eng.set_reference(dic.to_device_image(ref), torch.from_numpy(roi).cuda(), **w.params())
    return w, dic.to_device_image(frames[-1])


def _equal(a, b):
    import torch
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_noalloc_equals_correlate_on_two_calls_then_a_smaller_input():
    import torch
    assert dic.dic_noalloc_scratch_bytes() == 64 << 20
    eng = dic.Engine(0)
    print("GPU case: noalloc 256^2 c1", flush=True)
    w, de = _setup(eng, 256)
    plain = eng.correlate(de, w.seeds)
    first = eng.correlate_noalloc(de, w.seeds)
    torch.cuda.synchronize()
    _equal(plain, first)
    assert int((first["status"] == 0).sum()) > 0.9 * eng.stats()["active"]
    print("GPU case: noalloc 160^2 c1 (smaller input)", flush=True)
    w2, de2 = _setup(eng, 160, seed_shift=1)
    plain2 = eng.correlate(de2, w2.seeds)
    second = eng.correlate_noalloc(de2, w2.seeds)
    torch.cuda.synchronize()
    _equal(plain2, second)
    assert int((second["status"] == 0).sum()) > 0.9 * eng.stats()["active"]
    eng.close()


def test_noalloc_contexts_share_the_array_in_turn():
    # two contexts on one device use the one array one after the other; each call
    # clears what it needs, so the results do not depend on the previous call
    import torch
    a, b = dic.Engine(0), dic.Engine(0)
    wa, da = _setup(a, 256)
    wb, db = _setup(b, 192)
    ra = a.correlate(da, wa.seeds)
    rb = b.correlate(db, wb.seeds)
    print("GPU case: noalloc a, b, a", flush=True)
    na1 = a.correlate_noalloc(da, wa.seeds)
    nb = b.correlate_noalloc(db, wb.seeds)
    na2 = a.correlate_noalloc(da, wa.seeds)
    torch.cuda.synchronize()
    _equal(ra, na1)
    _equal(rb, nb)
    _equal(ra, na2)
    a.close()
    b.close()


def test_noalloc_refuses_a_reference_above_the_limit():
    # 2900^2 at step 2 with subset 21: 1440^2 nodes need ~75 MB of scratch
    import torch
    eng = dic.Engine(0)
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(2900, 2900), dtype=np.uint8)
    d = dic.to_device_image(img)
    print("GPU case: noalloc oversize 2900^2", flush=True)
    eng.set_reference(d, None, subset_size=21, step=2)
    with pytest.raises(dic.DicError) as e:
        eng.correlate_noalloc(d, [(1450, 1450, 0, 0)])
    assert e.value.code == dic.DIC_E_INVAL and "scratch" in str(e.value)
    # still usable, with the same reference and with a smaller one
    w, de = _setup(eng, 160)
    _equal(eng.correlate(de, w.seeds), eng.correlate_noalloc(de, w.seeds))
    torch.cuda.synchronize()
    eng.close()
