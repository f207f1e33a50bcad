"""Python binding of the C ABI in include/dic.h (libdicmi.so).

Argument marshalling only: every step of the correlation runs in the HIP
library.  PyTorch supplies device memory and the stream.  The entry points
keep the C names (dic_create, dic_set_reference, dic_grid_shape,
dic_correlate, dic_correlate_batch, dic_get_stats, dic_destroy,
dic_last_error, and the dic_server_* serving calls); `Engine` and `Server`
wrap them for torch tensors.

There is no fallback: if the library is missing or cannot be loaded, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdicmi.so")

DIC_OK, DIC_E_INVAL, DIC_E_NOMEM, DIC_E_DEVICE, DIC_E_STATE, DIC_E_NOSEED, DIC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_STATE", -5: "E_NOSEED",
                -6: "E_UNSUPPORTED"}
PIX_U8, PIX_U16, PIX_F32 = 0, 1, 2
COST = {"znssd": 0, "nssd": 1, "ssd": 2}
SHAPE_RIGID, SHAPE_AFFINE, SHAPE_QUADRATIC = 2, 6, 12
NODE = dict(CONVERGED=0, NOT_REACHED=1, NOT_IN_ROI=2, MAX_ITER=3, LOW_ZNCC=4, OUT_OF_BOUNDS=5, FLAT_REF=6,
            FLAT_DEF=7, SINGULAR=8, NAN=9)

# exported names, in the order include/dic.h declares them
EXPORTS = ["dic_create", "dic_set_reference", "dic_grid_shape", "dic_reference_arrays", "dic_node_grid",
           "dic_correlate",
           "dic_correlate_batch", "dic_correlate_noalloc", "dic_noalloc_scratch_bytes", "dic_get_stats",
           "dic_destroy", "dic_last_error", "dic_multiwindow", "dic_correlate_mw", "dic_correlate_sequence",
           "dic_correlate_chunked", "dic_strain", "dic_vsg", "dic_server_create", "dic_server_add_reference",
           "dic_server_remove_reference", "dic_server_submit", "dic_server_step", "dic_server_poll",
           "dic_server_forget", "dic_server_get_stats", "dic_server_destroy", "dic_server_last_error"]


class DicImage(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pitch_bytes", C.c_int64), ("pixel", C.c_int32),
                ("data", C.c_void_p)]


class DicParams(C.Structure):
    _fields_ = [("subset_size", C.c_int32), ("step", C.c_int32), ("shape", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("zncc_min", C.c_double), ("seed_radius", C.c_int32),
                ("guess_mode", C.c_int32), ("coef_fp16", C.c_int32), ("reduce_fp64", C.c_int32),
                ("nan_unconverged", C.c_int32), ("threads_per_subset", C.c_int32), ("tile_side", C.c_int32),
                ("cost", C.c_int32), ("lm_lambda", C.c_double)]


class DicSeed(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("u0", C.c_double), ("v0", C.c_double)]


class DicResult(C.Structure):
    _fields_ = [("p", C.c_void_p), ("zncc", C.c_void_p), ("iters", C.c_void_p), ("status", C.c_void_p),
                ("wave", C.c_void_p)]


class DicStats(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("active", C.c_int64), ("computed", C.c_int64), ("converged", C.c_int64),
                ("iterations", C.c_int64), ("waves", C.c_int32), ("frames", C.c_int32),
                ("threads_per_subset", C.c_int32), ("seed_du", C.c_int32), ("seed_dv", C.c_int32),
                ("ms_total", C.c_double), ("ms_icgn", C.c_double), ("ms_prefilter", C.c_double),
                ("ms_wave_kernels", C.c_double), ("wave_launches", C.c_int32), ("launch_chains", C.c_int32)]


class DicMwParams(C.Structure):
    _fields_ = [("max_disp", C.c_int32), ("subpixel", C.c_int32), ("mad_threshold", C.c_double)]


class DicSeqParams(C.Structure):
    _fields_ = [("update", C.c_int32), ("min_converged", C.c_double), ("min_zncc", C.c_double)]


class DicChunkParams(C.Structure):
    _fields_ = [("band_rows", C.c_int32), ("halo", C.c_int32), ("boundary_seeds", C.c_int32)]


class DicStrainParams(C.Structure):
    _fields_ = [("window", C.c_int32), ("basis", C.c_int32), ("measure", C.c_int32)]


STRAIN_BASIS = {"bilinear": 4, "biquadratic": 9}
STRAIN_MEASURE = {"green_lagrange": 0, "hencky": 1, "euler_almansi": 2, "biot_right": 3, "biot_left": 4}


class DicServerParams(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("hbm_budget_bytes", C.c_double)]


class DicServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("active", C.c_int32), ("waiting", C.c_int32), ("steps", C.c_int64), ("used_bytes", C.c_double),
                ("pool_bytes", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdicmi.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("the HIP library %s is not built; run paper_2601_12941_amd.build.build()" % path)
    # PyTorch ships its own HIP runtime under another file name; loading it first
    # makes the library bind to that same runtime instead of a second copy
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    P = C.POINTER
    L.dic_create.argtypes = [P(C.c_void_p), C.c_int, C.c_void_p]
    L.dic_set_reference.argtypes = [C.c_void_p, P(DicImage), C.c_void_p, P(DicParams)]
    L.dic_grid_shape.argtypes = [C.c_void_p] + [P(C.c_int32)] * 5
    L.dic_node_grid.argtypes = [C.c_int32] * 4 + [P(C.c_int32)] * 2
    L.dic_reference_arrays.argtypes = [C.c_void_p] * 5
    L.dic_correlate.argtypes = [C.c_void_p, P(DicImage), P(DicSeed), C.c_int32, P(DicResult)]
    L.dic_correlate_batch.argtypes = [C.c_void_p, P(DicImage), C.c_int32, P(DicSeed), C.c_int32, P(DicResult)]
    L.dic_correlate_noalloc.argtypes = [C.c_void_p, P(DicImage), P(DicSeed), C.c_int32, P(DicResult)]
    L.dic_noalloc_scratch_bytes.argtypes = []
    L.dic_get_stats.argtypes = [C.c_void_p, P(DicStats)]
    L.dic_strain.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                             P(DicStrainParams), C.c_void_p, C.c_void_p]
    L.dic_vsg.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.dic_multiwindow.argtypes = [C.c_void_p, P(DicImage), P(DicMwParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, P(C.c_int32)]
    L.dic_correlate_mw.argtypes = [C.c_void_p, P(DicImage), P(DicSeed), C.c_int32, P(DicMwParams), P(DicResult)]
    L.dic_correlate_sequence.argtypes = [C.c_void_p, P(DicImage), C.c_int32, C.c_void_p, P(DicSeed), C.c_int32,
                                         P(DicSeqParams), P(DicResult), P(C.c_int32)]
    L.dic_correlate_chunked.argtypes = [C.c_void_p, P(DicImage), P(DicImage), C.c_void_p, P(DicParams), P(DicSeed),
                                        C.c_int32, P(DicChunkParams), P(DicResult)]
    L.dic_destroy.argtypes = [C.c_void_p]
    L.dic_last_error.argtypes = [C.c_void_p]
    L.dic_last_error.restype = C.c_char_p
    L.dic_server_create.argtypes = [P(C.c_void_p), C.c_int, C.c_void_p, P(DicServerParams)]
    L.dic_server_add_reference.argtypes = [C.c_void_p, P(DicImage), C.c_void_p, P(DicParams), P(C.c_int32)]
    L.dic_server_remove_reference.argtypes = [C.c_void_p, C.c_int32]
    L.dic_server_submit.argtypes = [C.c_void_p, C.c_int32, P(DicImage), P(DicSeed), C.c_int32, P(DicResult),
                                    P(C.c_int64)]
    L.dic_server_step.argtypes = [C.c_void_p, C.c_int32]
    L.dic_server_poll.argtypes = [C.c_void_p, C.c_int64, P(C.c_int32), P(C.c_int32), P(DicStats)]
    L.dic_server_forget.argtypes = [C.c_void_p, C.c_int64]
    L.dic_server_get_stats.argtypes = [C.c_void_p, P(DicServerStats)]
    L.dic_server_destroy.argtypes = [C.c_void_p]
    L.dic_server_last_error.argtypes = [C.c_void_p]
    L.dic_server_last_error.restype = C.c_char_p
    for n in EXPORTS:
        if not n.endswith("last_error"):
            getattr(L, n).restype = C.c_int
    L.dic_noalloc_scratch_bytes.restype = C.c_int64
    L.dic_vsg.restype = C.c_int32
    _lib = L
    return L


class DicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


# ---- C-named entry points -------------------------------------------------
def dic_create(device: int = 0, stream: Optional[int] = None) -> C.c_void_p:
    ctx = C.c_void_p()
    rc = load_library().dic_create(C.byref(ctx), int(device), C.c_void_p(stream or 0))
    if rc != DIC_OK:
        raise DicError(rc, "dic_create failed")
    return ctx


def dic_last_error(ctx) -> str:
    m = load_library().dic_last_error(ctx)
    return m.decode() if m else ""


def _check(ctx, rc):
    if rc != DIC_OK:
        raise DicError(rc, dic_last_error(ctx))


def dic_set_reference(ctx, image: DicImage, roi_ptr: int, params: DicParams):
    _check(ctx, load_library().dic_set_reference(ctx, C.byref(image), C.c_void_p(roi_ptr or 0), C.byref(params)))


def dic_grid_shape(ctx):
    v = [C.c_int32() for _ in range(5)]
    _check(ctx, load_library().dic_grid_shape(ctx, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def dic_correlate(ctx, image: DicImage, seeds: Sequence[DicSeed], result: DicResult):
    arr = (DicSeed * len(seeds))(*seeds)
    _check(ctx, load_library().dic_correlate(ctx, C.byref(image), arr, len(seeds), C.byref(result)))


def dic_correlate_batch(ctx, images: Sequence[DicImage], seeds: Sequence[DicSeed], nseeds: int,
                        results: Sequence[DicResult]):
    ims = (DicImage * len(images))(*images)
    sds = (DicSeed * len(seeds))(*seeds)
    res = (DicResult * len(results))(*results)
    _check(ctx, load_library().dic_correlate_batch(ctx, ims, len(images), sds, nseeds, res))


def dic_correlate_noalloc(ctx, image: DicImage, seeds: Sequence[DicSeed], result: DicResult):
    arr = (DicSeed * len(seeds))(*seeds)
    _check(ctx, load_library().dic_correlate_noalloc(ctx, C.byref(image), arr, len(seeds), C.byref(result)))


def dic_noalloc_scratch_bytes() -> int:
    return int(load_library().dic_noalloc_scratch_bytes())


def dic_strain(ctx, u_ptr: int, v_ptr: int, status_ptr: int, nx: int, ny: int, step: int,
               params: DicStrainParams, F_ptr: int, eps_ptr: int):
    _check(ctx, load_library().dic_strain(ctx, C.c_void_p(u_ptr), C.c_void_p(v_ptr), C.c_void_p(status_ptr or 0),
                                          int(nx), int(ny), int(step), C.byref(params), C.c_void_p(F_ptr),
                                          C.c_void_p(eps_ptr)))


def dic_multiwindow(ctx, image: DicImage, params: DicMwParams, u_ptr: int, v_ptr: int, valid_ptr: int):
    lv = (C.c_int32 * 32)()
    n = C.c_int32()
    _check(ctx, load_library().dic_multiwindow(ctx, C.byref(image), C.byref(params), C.c_void_p(u_ptr),
                                               C.c_void_p(v_ptr), C.c_void_p(valid_ptr), lv, C.byref(n)))
    return [lv[i] for i in range(n.value)]


def dic_correlate_mw(ctx, image: DicImage, seeds: Sequence[DicSeed], params: DicMwParams, result: DicResult):
    arr = (DicSeed * len(seeds))(*seeds)
    _check(ctx, load_library().dic_correlate_mw(ctx, C.byref(image), arr, len(seeds), C.byref(params),
                                                C.byref(result)))


def dic_correlate_sequence(ctx, images: Sequence[DicImage], roi_ptr: int, seeds: Sequence[DicSeed],
                           params: DicSeqParams, results: Sequence[DicResult]):
    ims = (DicImage * len(images))(*images)
    sds = (DicSeed * len(seeds))(*seeds)
    res = (DicResult * len(results))(*results)
    refs = (C.c_int32 * len(images))()
    _check(ctx, load_library().dic_correlate_sequence(ctx, ims, len(images), C.c_void_p(roi_ptr or 0), sds,
                                                      len(seeds), C.byref(params), res, refs))
    return list(refs)


def dic_correlate_chunked(ctx, ref: DicImage, deformed: DicImage, roi_host_ptr: int, params: DicParams,
                          seeds: Sequence[DicSeed], chunk: DicChunkParams, result: DicResult):
    sds = (DicSeed * len(seeds))(*seeds)
    _check(ctx, load_library().dic_correlate_chunked(ctx, C.byref(ref), C.byref(deformed),
                                                     C.c_void_p(roi_host_ptr or 0), C.byref(params), sds, len(seeds),
                                                     C.byref(chunk), C.byref(result)))


def dic_vsg(window: int, step: int, subset_size: int) -> int:
    return int(load_library().dic_vsg(int(window), int(step), int(subset_size)))


def dic_get_stats(ctx) -> dict:
    s = DicStats()
    _check(ctx, load_library().dic_get_stats(ctx, C.byref(s)))
    return {k: getattr(s, k) for k, _ in DicStats._fields_}


def dic_destroy(ctx):
    load_library().dic_destroy(ctx)


def dic_server_create(device: int, stream: Optional[int], max_active: int, hbm_budget_bytes: float) -> C.c_void_p:
    srv = C.c_void_p()
    prm = DicServerParams(int(max_active), float(hbm_budget_bytes))
    rc = load_library().dic_server_create(C.byref(srv), int(device), C.c_void_p(stream or 0), C.byref(prm))
    if rc != DIC_OK:
        raise DicError(rc, "dic_server_create failed")
    return srv


def dic_server_last_error(srv) -> str:
    m = load_library().dic_server_last_error(srv)
    return m.decode() if m else ""


def _scheck(srv, rc):
    if rc != DIC_OK:
        raise DicError(rc, dic_server_last_error(srv))


def dic_server_add_reference(srv, image: DicImage, roi_ptr: int, params: DicParams) -> int:
    rid = C.c_int32()
    _scheck(srv, load_library().dic_server_add_reference(srv, C.byref(image), C.c_void_p(roi_ptr or 0),
                                                         C.byref(params), C.byref(rid)))
    return rid.value


def dic_server_remove_reference(srv, ref_id: int):
    _scheck(srv, load_library().dic_server_remove_reference(srv, int(ref_id)))


def dic_server_submit(srv, ref_id: int, image: DicImage, seeds: Sequence[DicSeed], result: DicResult) -> int:
    arr = (DicSeed * len(seeds))(*seeds)
    t = C.c_int64()
    _scheck(srv, load_library().dic_server_submit(srv, int(ref_id), C.byref(image), arr, len(seeds),
                                                  C.byref(result), C.byref(t)))
    return t.value


def dic_server_step(srv, steps: int = 1):
    _scheck(srv, load_library().dic_server_step(srv, int(steps)))


def dic_server_poll(srv, ticket: int):
    done, status, st = C.c_int32(), C.c_int32(), DicStats()
    _scheck(srv, load_library().dic_server_poll(srv, int(ticket), C.byref(done), C.byref(status), C.byref(st)))
    return bool(done.value), status.value, {k: getattr(st, k) for k, _ in DicStats._fields_}


def dic_server_forget(srv, ticket: int):
    _scheck(srv, load_library().dic_server_forget(srv, int(ticket)))


def dic_server_get_stats(srv) -> dict:
    s = DicServerStats()
    _scheck(srv, load_library().dic_server_get_stats(srv, C.byref(s)))
    return {k: getattr(s, k) for k, _ in DicServerStats._fields_}


def dic_server_destroy(srv):
    load_library().dic_server_destroy(srv)


# ---- torch convenience -----------------------------------------------------
def _image(t) -> DicImage:
    import torch
    if not t.is_cuda:
        raise ValueError("images must be device tensors")
    if t.dim() != 2:
        raise ValueError("images must be 2-D [H][W]")
    if t.stride(1) != 1:
        raise ValueError("image rows must be contiguous")
    if t.dtype == torch.uint8:
        pix, es = PIX_U8, 1
    elif t.dtype in (torch.int16, torch.uint16):
        pix, es = PIX_U16, 2
    elif t.dtype == torch.float32:
        pix, es = PIX_F32, 4
    else:
        raise ValueError("unsupported image dtype %s" % t.dtype)
    return DicImage(t.shape[1], t.shape[0], t.stride(0) * es, pix, t.data_ptr())


def to_device_image(a, device="cuda"):
    """numpy image -> device tensor (uint16 data travels as int16 bits)."""
    import numpy as np
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(device)


class Engine:
    """A library context bound to one device and the current torch stream."""

    def __init__(self, device: int = 0):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = dic_create(device, self.stream.cuda_stream)
        self.shape = None
        self._keep = []

    def close(self):
        if self.ctx is not None:
            dic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_reference(self, ref, roi=None, *, subset_size, step, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
                      seed_radius=8, guess="extrapolate", coef_fp16=False, reduce_fp64=True, nan_unconverged=False,
                      threads_per_subset=0, tile_side=0, cost="znssd", lm_lambda=0.0):
        prm = _params(subset_size, step, shape, tol, max_iter, zncc_min, seed_radius, guess, coef_fp16, reduce_fp64,
                      nan_unconverged, threads_per_subset, tile_side, cost, lm_lambda)
        roi_ptr = 0
        if roi is not None:
            import torch
            if roi.dtype != torch.uint8 or not roi.is_cuda or not roi.is_contiguous() or tuple(roi.shape) != tuple(
                    ref.shape):
                raise ValueError("roi must be a contiguous uint8 device tensor shaped like the image")
            roi_ptr = roi.data_ptr()
        self.ref = ref
        dic_set_reference(self.ctx, _image(ref), roi_ptr, prm)
        self.shape = shape
        self.grid = dic_grid_shape(self.ctx)
        return self.grid

    def _alloc(self):
        import torch
        nx, ny = self.grid[0], self.grid[1]
        d = self.device
        out = dict(p=torch.empty((self.shape, ny, nx), dtype=torch.float32, device=d),
                   zncc=torch.empty((ny, nx), dtype=torch.float32, device=d),
                   iters=torch.empty((ny, nx), dtype=torch.int16, device=d),
                   status=torch.empty((ny, nx), dtype=torch.int8, device=d),
                   wave=torch.empty((ny, nx), dtype=torch.int32, device=d))
        res = DicResult(out["p"].data_ptr(), out["zncc"].data_ptr(), out["iters"].data_ptr(),
                        out["status"].data_ptr(), out["wave"].data_ptr())
        return out, res

    @staticmethod
    def _seeds(seeds: Iterable) -> List[DicSeed]:
        return [DicSeed(float(s[0]), float(s[1]), float(s[2]) if len(s) > 2 else 0.0,
                        float(s[3]) if len(s) > 3 else 0.0) for s in seeds]

    def correlate(self, deformed, seeds):
        out, res = self._alloc()
        dic_correlate(self.ctx, _image(deformed), self._seeds(seeds), res)
        return out

    def correlate_noalloc(self, deformed, seeds, out=None):
        """dic_correlate_noalloc into caller-owned result tensors (allocated here
        when `out` is None, as a caller would before entering its loop)."""
        if out is None:
            out, res = self._alloc()
        else:
            res = DicResult(out["p"].data_ptr(), out["zncc"].data_ptr(), out["iters"].data_ptr(),
                            out["status"].data_ptr(), out["wave"].data_ptr())
        dic_correlate_noalloc(self.ctx, _image(deformed), self._seeds(seeds), res)
        return out

    def correlate_batch(self, frames, seeds):
        """frames: list of device images; seeds: one list shared by all frames, or one list per frame."""
        seeds = list(seeds)
        per_frame = len(seeds) == len(frames) and all(isinstance(s, (list, tuple)) and len(s) > 0 and
                                                        isinstance(s[0], (list, tuple)) for s in seeds)
        lists = seeds if per_frame else [seeds] * len(frames)
        ns = len(lists[0])
        if any(len(s) != ns for s in lists):
            raise ValueError("every frame needs the same number of seeds")
        flat = [sd for s in lists for sd in self._seeds(s)]
        outs, ress = zip(*[self._alloc() for _ in frames])
        dic_correlate_batch(self.ctx, [_image(f) for f in frames], flat, ns, list(ress))
        return list(outs)

    def multiwindow(self, deformed, *, max_disp, subpixel=False, mad_threshold=2.0):
        """dic_multiwindow: per-node rigid estimates u, v (float32) and valid (int8), plus the level sizes."""
        import torch
        nx, ny = self.grid[0], self.grid[1]
        u = torch.empty((ny, nx), dtype=torch.float32, device=self.device)
        v = torch.empty_like(u)
        valid = torch.empty((ny, nx), dtype=torch.int8, device=self.device)
        lv = dic_multiwindow(self.ctx, _image(deformed), DicMwParams(int(max_disp), int(bool(subpixel)),
                                                                     float(mad_threshold)),
                             u.data_ptr(), v.data_ptr(), valid.data_ptr())
        return {"u": u, "v": v, "valid": valid, "levels": lv}

    def correlate_mw(self, deformed, seeds, *, max_disp, mad_threshold=2.0):
        """dic_correlate_mw: reliability-guided correlation seeded by the multi-window estimate."""
        out, res = self._alloc()
        dic_correlate_mw(self.ctx, _image(deformed), self._seeds(seeds),
                         DicMwParams(int(max_disp), 0, float(mad_threshold)), res)
        return out

    def correlate_sequence(self, frames, seeds, roi=None, *, update=True, min_converged=0.95, min_zncc=0.9):
        """dic_correlate_sequence: every frame on the original nodes, and the reference of each."""
        outs, ress = zip(*[self._alloc() for _ in frames])
        refs = dic_correlate_sequence(self.ctx, [_image(f) for f in frames], _roi_ptr(roi, self.ref),
                                      self._seeds(seeds), DicSeqParams(int(bool(update)), float(min_converged),
                                                                       float(min_zncc)), list(ress))
        return list(outs), refs

    def reference_arrays(self):
        """dic_reference_arrays: the current reference's stored coefficients (1/36 of
        the classical ones), interpolant and gradient, as device tensors [H][W]."""
        import torch
        H, W = self.ref.shape
        out = {k: torch.empty((H, W), dtype=torch.float32, device=self.device) for k in ("coef", "f", "fx", "fy")}
        dic_reference_arrays(self.ctx, *[out[k].data_ptr() for k in ("coef", "f", "fx", "fy")])
        return out

    def correlate_chunked(self, ref, deformed, roi=None, *, seeds, band_rows, halo, boundary_seeds=8, **params):
        """dic_correlate_chunked on HOST numpy images (uint8, uint16 or float32
        [H][W]) and an optional host uint8 ROI: the whole grid's result as host
        numpy arrays, with one band of the pair on the device at a time.  The
        context's reference afterwards is the last band's window."""
        import numpy as np
        ref = np.ascontiguousarray(ref)
        deformed = np.ascontiguousarray(deformed)
        if ref.shape != deformed.shape or ref.dtype != deformed.dtype or ref.ndim != 2:
            raise ValueError("reference and deformed must be 2-D host arrays of one shape and dtype")
        pix = {np.dtype(np.uint8): PIX_U8, np.dtype(np.uint16): PIX_U16, np.dtype(np.float32): PIX_F32}.get(ref.dtype)
        if pix is None:
            raise ValueError("pixels must be uint8, uint16 or float32")
        H, W = ref.shape
        if roi is not None:
            roi = np.ascontiguousarray(roi, dtype=np.uint8)
            if roi.shape != ref.shape:
                raise ValueError("roi must be shaped like the images")
        shape = params.get("shape", 6)
        nx, ny = _grid(params["subset_size"], params["step"], W, H)
        out = dict(p=np.empty((shape, ny, nx), np.float32), zncc=np.empty((ny, nx), np.float32),
                   iters=np.empty((ny, nx), np.int16), status=np.empty((ny, nx), np.int8),
                   wave=np.empty((ny, nx), np.int32))
        res = DicResult(*[out[k].ctypes.data for k in ("p", "zncc", "iters", "status", "wave")])
        ri = DicImage(W, H, ref.strides[0], pix, ref.ctypes.data)
        di = DicImage(W, H, deformed.strides[0], pix, deformed.ctypes.data)
        dic_correlate_chunked(self.ctx, ri, di, roi.ctypes.data if roi is not None else 0, _params(**params),
                              self._seeds(seeds), DicChunkParams(int(band_rows), int(halo), int(boundary_seeds)), res)
        self.ref = None
        self.shape = shape
        self.grid = dic_grid_shape(self.ctx)
        return out

    def strain(self, u, v, status=None, *, step, window=5, basis="bilinear", measure="green_lagrange"):
        """dic_strain on device displacement planes u, v [ny][nx] (e.g. a result's p[0], p[1])."""
        import torch
        for t in (u, v):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 2):
                raise ValueError("u and v must be contiguous float32 device tensors [ny][nx]")
        if status is not None and not (status.is_cuda and status.dtype == torch.int8 and status.is_contiguous()):
            raise ValueError("status must be a contiguous int8 device tensor")
        ny, nx = u.shape
        F = torch.empty((4, ny, nx), dtype=torch.float32, device=u.device)
        eps = torch.empty((3, ny, nx), dtype=torch.float32, device=u.device)
        prm = DicStrainParams(int(window), STRAIN_BASIS[basis], STRAIN_MEASURE[measure])
        dic_strain(self.ctx, u.data_ptr(), v.data_ptr(), status.data_ptr() if status is not None else 0, nx, ny,
                   step, prm, F.data_ptr(), eps.data_ptr())
        return {"F": F, "eps": eps}

    def stats(self) -> dict:
        return dic_get_stats(self.ctx)


def _params(subset_size, step, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7, seed_radius=8, guess="extrapolate",
            coef_fp16=False, reduce_fp64=True, nan_unconverged=False, threads_per_subset=0,
            tile_side=0, cost="znssd", lm_lambda=0.0) -> DicParams:
    return DicParams(subset_size, step, shape, max_iter, tol, zncc_min, seed_radius, 1 if guess == "copy" else 0,
                     int(bool(coef_fp16)), int(bool(reduce_fp64)), int(bool(nan_unconverged)), threads_per_subset,
                     tile_side, COST[cost], float(lm_lambda))


def _roi_ptr(roi, ref) -> int:
    if roi is None:
        return 0
    import torch
    if roi.dtype != torch.uint8 or not roi.is_cuda or not roi.is_contiguous() or tuple(roi.shape) != tuple(ref.shape):
        raise ValueError("roi must be a contiguous uint8 device tensor shaped like the image")
    return roi.data_ptr()


def dic_reference_arrays(ctx, coef_ptr: int, f_ptr: int, fx_ptr: int, fy_ptr: int):
    _check(ctx, load_library().dic_reference_arrays(ctx, *[C.c_void_p(x or 0) for x in (coef_ptr, f_ptr, fx_ptr,
                                                                                        fy_ptr)]))


def dic_node_grid(width: int, height: int, subset_size: int, step: int):
    nx, ny = C.c_int32(), C.c_int32()
    rc = load_library().dic_node_grid(int(width), int(height), int(subset_size), int(step), C.byref(nx),
                                      C.byref(ny))
    if rc != DIC_OK:
        raise DicError(rc, "no node grid for a %dx%d image, subset %d, step %d" % (width, height, subset_size, step))
    return nx.value, ny.value


def _grid(subset_size, step, W, H):
    """Node grid of a reference, from the library."""
    return dic_node_grid(W, H, subset_size, step)


class Server:
    """Continuous-batching server on one device and the current torch stream.

    add_reference() makes a reference resident; submit() queues a request and
    returns (ticket, output tensors); step() admits and advances requests;
    poll() tells whether a ticket is done.  Deformed images and outputs are
    kept alive here until their request is done.
    """

    def __init__(self, device: int = 0, max_active: int = 16, hbm_budget_bytes: float = 64e9):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.srv = dic_server_create(device, self.stream.cuda_stream, max_active, hbm_budget_bytes)
        self._refs = {}
        self._live = {}

    def close(self):
        if self.srv is not None:
            dic_server_destroy(self.srv)
            self.srv = None
            self._live.clear()
            self._refs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_reference(self, ref, roi=None, **params) -> int:
        prm = _params(**params)
        rid = dic_server_add_reference(self.srv, _image(ref), _roi_ptr(roi, ref), prm)
        nx, ny = _grid(prm.subset_size, prm.step, ref.shape[1], ref.shape[0])
        self._refs[rid] = (ref, roi, prm.shape, nx, ny)
        return rid

    def remove_reference(self, ref_id: int):
        dic_server_remove_reference(self.srv, ref_id)
        self._refs.pop(ref_id, None)

    def submit(self, ref_id: int, deformed, seeds):
        import torch
        if ref_id not in self._refs:   # the library reports the unknown id
            dic_server_submit(self.srv, ref_id, _image(deformed), Engine._seeds(seeds), DicResult())
            raise DicError(DIC_E_INVAL, "unknown reference %d" % ref_id)
        _, _, shape, nx, ny = self._refs[ref_id]
        d = self.device
        out = dict(p=torch.empty((shape, ny, nx), dtype=torch.float32, device=d),
                   zncc=torch.empty((ny, nx), dtype=torch.float32, device=d),
                   iters=torch.empty((ny, nx), dtype=torch.int16, device=d),
                   status=torch.empty((ny, nx), dtype=torch.int8, device=d),
                   wave=torch.empty((ny, nx), dtype=torch.int32, device=d))
        res = DicResult(out["p"].data_ptr(), out["zncc"].data_ptr(), out["iters"].data_ptr(),
                        out["status"].data_ptr(), out["wave"].data_ptr())
        t = dic_server_submit(self.srv, ref_id, _image(deformed), Engine._seeds(seeds), res)
        self._live[t] = (deformed, out)
        return t, out

    def step(self, steps: int = 1):
        dic_server_step(self.srv, steps)

    def poll(self, ticket: int):
        """(done, status code, counters); a done ticket's tensors are released here."""
        done, status, st = dic_server_poll(self.srv, ticket)
        if done:
            self._live.pop(ticket, None)
        return done, status, st

    def forget(self, ticket: int):
        """Drop a finished request's record in the library (the ticket becomes unknown)."""
        dic_server_forget(self.srv, ticket)

    def stats(self) -> dict:
        return dic_server_get_stats(self.srv)
