"""Binding of the device-rate probes (include/dic_roofs.h, libdicroofs.so):
the achievable HBM, cache, LDS and FMA rates the benchmark quotes beside the
published peaks.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

from .build import ROOFS_LIB

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(ROOFS_LIB):
            raise RuntimeError("%s is not built (python -m paper_2601_12941_amd.build)" % ROOFS_LIB)
        L = C.CDLL(ROOFS_LIB)
        for n, args in (("dic_roof_hbm_read", [C.c_int64, C.c_int]), ("dic_roof_hbm_copy", [C.c_int64, C.c_int]),
                        ("dic_roof_cache_read", [C.c_int64, C.c_int64, C.c_int, C.c_int]),
                        ("dic_roof_lds_read", [C.c_int, C.c_int]), ("dic_roof_fma", [C.c_int, C.c_int, C.c_int])):
            f = getattr(L, n)
            f.argtypes = args
            f.restype = C.c_double
        _lib = L
    return _lib


def _rate(v, what):
    if v < 0:
        raise RuntimeError("probe %s failed" % what)
    return v


def hbm_read(nbytes=4 << 30, reps=5):
    return _rate(_load().dic_roof_hbm_read(nbytes, reps), "hbm_read")


def hbm_copy(nbytes=2 << 30, reps=5):
    return _rate(_load().dic_roof_hbm_copy(nbytes, reps), "hbm_copy")


def cache_read(footprint, chunk, inner=1, reps=5):
    return _rate(_load().dic_roof_cache_read(footprint, chunk, inner, reps), "cache_read")


def lds_read(iters=256, reps=5):
    return _rate(_load().dic_roof_lds_read(iters, reps), "lds_read")


def fma(fp64=False, iters=4096, reps=5):
    return _rate(_load().dic_roof_fma(1 if fp64 else 0, iters, reps), "fma")


def measure():
    """All probes with their default sizes: a dict of rates."""
    return {
        "hbm_read_GBps": hbm_read(),
        "hbm_copy_GBps": hbm_copy(),
        "l2_read_GBps": cache_read(2 << 20, 2 << 20, inner=4),
        "infinity_cache_64MiB_read_GBps": cache_read(64 << 20, 1 << 20, inner=2),
        "infinity_cache_192MiB_read_GBps": cache_read(192 << 20, 1 << 20, inner=2),
        "lds_read_GBps": lds_read(),
        "fma_f32_TFLOPs": fma(False),
        "fma_f64_TFLOPs": fma(True),
    }
