"""The C ABI without a GPU: the built library loads, exports every function
include/dic.h declares, the binding's struct layouts match the header's, and
calls that need no device fail cleanly."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2601_12941_amd import dic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dic.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(dic_[a-z_]+)\s*\(", txt, flags=re.M)


def test_header_declares_the_binding_names():
    assert sorted(declared_functions()) == sorted(dic.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dic.LIB_PATH):
        pytest.skip("library not built")
    L = dic.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", dic.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(r"\bT %s\b" % name, out), name


def _c_layout():
    prog = r"""
#include <stddef.h>
#include <stdio.h>
#include "dic.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("dic_image %zu\n", sizeof(dic_image));
  F(dic_image, width) F(dic_image, height) F(dic_image, pitch_bytes) F(dic_image, pixel) F(dic_image, data)
  printf("dic_params %zu\n", sizeof(dic_params));
  F(dic_params, subset_size) F(dic_params, step) F(dic_params, shape) F(dic_params, max_iter) F(dic_params, tol)
  F(dic_params, zncc_min) F(dic_params, seed_radius) F(dic_params, guess_mode) F(dic_params, coef_fp16)
  F(dic_params, reduce_fp64) F(dic_params, nan_unconverged) F(dic_params, threads_per_subset)
  F(dic_params, tile_side) F(dic_params, cost) F(dic_params, lm_lambda)
  printf("dic_mw_params %zu\n", sizeof(dic_mw_params));
  F(dic_mw_params, max_disp) F(dic_mw_params, subpixel) F(dic_mw_params, mad_threshold)
  printf("dic_seq_params %zu\n", sizeof(dic_seq_params));
  F(dic_seq_params, update) F(dic_seq_params, min_converged) F(dic_seq_params, min_zncc)
  printf("dic_strain_params %zu\n", sizeof(dic_strain_params));
  F(dic_strain_params, window) F(dic_strain_params, basis) F(dic_strain_params, measure)
  printf("dic_chunk_params %zu\n", sizeof(dic_chunk_params));
  F(dic_chunk_params, band_rows) F(dic_chunk_params, halo) F(dic_chunk_params, boundary_seeds)
  printf("dic_seed %zu\n", sizeof(dic_seed));
  printf("dic_result %zu\n", sizeof(dic_result));
  F(dic_result, p) F(dic_result, zncc) F(dic_result, iters) F(dic_result, status) F(dic_result, wave)
  printf("dic_stats %zu\n", sizeof(dic_stats));
  F(dic_stats, waves) F(dic_stats, ms_total) F(dic_stats, ms_wave_kernels) F(dic_stats, wave_launches) F(dic_stats, launch_chains)
  printf("dic_server_params %zu\n", sizeof(dic_server_params));
  F(dic_server_params, max_active) F(dic_server_params, hbm_budget_bytes)
  printf("dic_server_stats %zu\n", sizeof(dic_server_stats));
  F(dic_server_stats, submitted) F(dic_server_stats, admitted) F(dic_server_stats, completed)
  F(dic_server_stats, active) F(dic_server_stats, waiting) F(dic_server_stats, steps)
  F(dic_server_stats, used_bytes) F(dic_server_stats, pool_bytes)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True).stdout
    return dict(line.rsplit(" ", 1) for line in out.strip().splitlines())


def test_struct_layouts_match_header():
    lay = {k: int(v) for k, v in _c_layout().items()}
    for name, cls in (("dic_image", dic.DicImage), ("dic_params", dic.DicParams), ("dic_seed", dic.DicSeed),
                      ("dic_result", dic.DicResult), ("dic_stats", dic.DicStats),
                      ("dic_server_params", dic.DicServerParams), ("dic_server_stats", dic.DicServerStats),
                      ("dic_mw_params", dic.DicMwParams), ("dic_seq_params", dic.DicSeqParams),
                      ("dic_strain_params", dic.DicStrainParams), ("dic_chunk_params", dic.DicChunkParams)):
        assert lay[name] == C.sizeof(cls), name
        for field, _ in cls._fields_:
            key = "%s.%s" % (name, field)
            if key in lay:
                assert lay[key] == getattr(cls, field).offset, key


def test_calls_without_a_device_fail_cleanly():
    if not os.path.exists(dic.LIB_PATH):
        pytest.skip("library not built")
    L = dic.load_library()
    assert L.dic_create(None, 0, None) == dic.DIC_E_INVAL
    assert L.dic_destroy(None) == dic.DIC_E_INVAL
    assert L.dic_get_stats(None, None) == dic.DIC_E_INVAL
    assert L.dic_correlate(None, None, None, 0, None) == dic.DIC_E_INVAL
    assert dic.load_library().dic_last_error(None) == b"null context"
    assert L.dic_server_create(None, 0, None, None) == dic.DIC_E_INVAL
    prm = dic.DicServerParams(0, 1e9)
    srv = C.c_void_p()
    assert L.dic_server_create(C.byref(srv), 0, None, C.byref(prm)) == dic.DIC_E_INVAL
    assert L.dic_server_step(None, 1) == dic.DIC_E_INVAL
    assert L.dic_server_poll(None, 1, None, None, None) == dic.DIC_E_INVAL
    assert L.dic_server_get_stats(None, None) == dic.DIC_E_INVAL
    assert L.dic_server_forget(None, 1) == dic.DIC_E_INVAL
    assert L.dic_server_destroy(None) == dic.DIC_E_INVAL
    assert L.dic_server_last_error(None) == b"null server"


def test_node_grid_counts_the_subsets_that_fit():
    # host-only call: nodes sit at h + i*step (h = (N-1)/2) while the N x N subset
    # stays inside the image, i.e. centres in [h, W-1-h]
    if not os.path.exists(dic.LIB_PATH):
        pytest.skip("library not built")
    for W, H, N, s in ((64, 48, 21, 5), (65, 47, 21, 4), (21, 21, 21, 7), (40, 90, 15, 1), (2048, 2048, 31, 2)):
        h = (N - 1) // 2
        assert dic.dic_node_grid(W, H, N, s) == (len(range(h, W - h, s)), len(range(h, H - h, s)))
    with pytest.raises(dic.DicError):
        dic.dic_node_grid(20, 40, 21, 2)
    with pytest.raises(dic.DicError):
        dic.dic_node_grid(40, 40, 21, 0)


def test_probe_library_exports_its_header():
    from paper_2601_12941_amd import build
    if not os.path.exists(build.ROOFS_LIB):
        pytest.skip("library not built")
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "dic_roofs.h")).read(), flags=re.S)
    names = re.findall(r"^\s*double\s+(dic_roof_[a-z_0-9]+)\s*\(", txt, flags=re.M)
    assert len(names) == 5
    out = subprocess.run(["nm", "-D", "--defined-only", build.ROOFS_LIB], capture_output=True, text=True).stdout
    for name in names:
        assert re.search(r"\bT %s\b" % name, out), name


def test_missing_library_raises(tmp_path, monkeypatch):
    monkeypatch.setattr(dic, "_lib", None)
    with pytest.raises(RuntimeError):
        dic.load_library(str(tmp_path / "nope.so"))
