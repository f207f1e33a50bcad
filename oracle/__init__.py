"""ctypes front end of the FP64 oracle (dic_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package's smoke check
and by the benchmark's CPU-baseline leg, never by the library's own path.
Images are handed over as float64 arrays of raw pixel values; every output is
float64 / int32 numpy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dic_oracle.c")
_SRC_MW = os.path.join(_HERE, "mw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST = dict(CONVERGED=0, NOT_REACHED=1, NOT_IN_ROI=2, MAX_ITER=3, LOW_ZNCC=4, OUT_OF_BOUNDS=5,
          FLAT_REF=6, FLAT_DEF=7, SINGULAR=8, NAN=9)
ORDER = dict(wave=0, sequential=1)
GUESS = dict(extrapolate=0, copy=1)
COST = dict(znssd=0, nssd=1, ssd=2)

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP over wave members)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in (_SRC, _SRC_MW))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC,
                               _SRC_MW, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.orc_prefilter_2d.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_prefilter_line.argtypes = [dp, C.c_long, C.c_long]
        L.orc_eval_many.argtypes = [dp, C.c_int, C.c_int, dp, dp, C.c_long, dp, dp, dp]
        L.orc_compose.argtypes = [dp, dp, C.c_int, dp]
        L.orc_compose.restype = C.c_int
        L.orc_transfer_guess.argtypes = [dp, C.c_int, C.c_double, C.c_double, C.c_int, dp]
        L.orc_icgn_single.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                      C.c_double, C.c_double, dp, dp, dp, ip, ip, C.c_int, C.c_double]
        L.orc_seed_single.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_double, C.c_double, ip, ip, dp]
        L.orc_seed_single.restype = C.c_int
        L.orc_correlate.argtypes = [dp, dp, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, dp, C.c_int, C.c_int,
                                    dp, dp, ip, ip, ip, dp, C.c_int, C.c_double]
        L.orc_correlate.restype = C.c_long
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.orc_fft2.argtypes = [dp, dp, C.c_int, C.c_int]
        L.orc_phase_corr.argtypes = [dp, dp, C.c_int, dp]
        L.orc_map_peak.argtypes = [dp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.orc_gauss3.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_gauss3.restype = C.c_double
        L.orc_mw_levels.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip, C.POINTER(C.c_int)]
        L.orc_mw_levels.restype = C.c_int
        L.orc_mad_filter.argtypes = [ip, ip, C.c_void_p, C.c_int, C.c_int, C.c_double, u8p]
        L.orc_mad_filter.restype = C.c_long
        L.orc_multiwindow.argtypes = [dp, dp, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_double, dp, dp, ip, dp, ip]
        L.orc_multiwindow.restype = C.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def prefilter(img) -> np.ndarray:
    """Cubic B-spline coefficients (mirror boundary) of a 2-D image."""
    img = _f64(img)
    H, W = img.shape
    out = np.empty_like(img)
    lib().orc_prefilter_2d(img, W, H, out)
    return out


def prefilter_line(s) -> np.ndarray:
    s = _f64(s).copy()
    lib().orc_prefilter_line(s, s.size, 1)
    return s


def evaluate(coef, x, y):
    """Interpolant value and (d/dx, d/dy) at points (x, y)."""
    coef = _f64(coef)
    H, W = coef.shape
    x = _f64(np.atleast_1d(x))
    y = _f64(np.atleast_1d(y))
    v = np.empty_like(x)
    gx = np.empty_like(x)
    gy = np.empty_like(x)
    lib().orc_eval_many(coef, W, H, x, y, x.size, v, gx, gy)
    return v, gx, gy


def compose(p, dp, npar):
    """p o dp^{-1} for the rigid (2), affine (6) or quadratic (12) shape."""
    a = np.zeros(12)
    b = np.zeros(12)
    a[:npar] = np.asarray(p, np.float64)[:npar]
    b[:npar] = np.asarray(dp, np.float64)[:npar]
    out = np.zeros(12)
    ok = lib().orc_compose(a, b, npar, out)
    if not ok:
        raise ZeroDivisionError("increment warp not invertible")
    return out[:npar]


def transfer_guess(pm, npar, ddx, ddy, mode="extrapolate"):
    a = np.zeros(12)
    a[:npar] = np.asarray(pm, np.float64)[:npar]
    out = np.zeros(12)
    lib().orc_transfer_guess(a, npar, float(ddx), float(ddy), GUESS[mode], out)
    return out[:npar]


def icgn(ref, deformed, xc, yc, p_init, N, npar=6, tol=1e-4, max_iter=50, zncc_min=0.7, cost="znssd",
         lm_lambda=0.0):
    """IC-GN (or, with lm_lambda > 0, Levenberg-Marquardt) of one subset centred at
    (xc, yc) from p_init on the chosen cost.  Returns (p, zncc, iters, status)."""
    ref = _f64(ref)
    de = _f64(deformed)
    H, W = ref.shape
    pi = np.zeros(12)
    pi[:len(p_init)] = p_init
    p = np.zeros(12)
    z = np.zeros(1)
    it = np.zeros(1, np.int32)
    st = np.zeros(1, np.int32)
    lib().orc_icgn_single(ref, de, W, H, N, npar, tol, max_iter, zncc_min, float(xc), float(yc), pi, p, z, it, st,
                          COST[cost], float(lm_lambda))
    return p[:npar], float(z[0]), int(it[0]), int(st[0])


def seed_search(ref, deformed, xc, yc, N, R, u0=0.0, v0=0.0):
    ref_a = np.asarray(ref)
    int_pix = int(np.issubdtype(ref_a.dtype, np.integer))
    ref = _f64(ref)
    de = _f64(deformed)
    H, W = ref.shape
    du = np.zeros(1, np.int32)
    dv = np.zeros(1, np.int32)
    z = np.zeros(1)
    ok = lib().orc_seed_single(ref, de, W, H, int_pix, N, R, int(xc), int(yc), float(u0), float(v0), du, dv, z)
    return bool(ok), int(du[0]), int(dv[0]), float(z[0])


def correlate(ref, deformed, roi=None, *, subset_size, step, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
              seed_radius=8, seeds, order="wave", guess="extrapolate", threads=1, cost="znssd", lm_lambda=0.0):
    """Reliability-guided correlation of one pair.

    seeds: iterable of (x, y, u0, v0).  Returns a dict of [ny][nx] arrays
    (p is [12][ny][nx], only the first `shape` planes meaningful) plus
    'seed_nodes' rows (node, du, dv, zncc) and 'seconds'.
    """
    ref_a = np.asarray(ref)
    int_pix = int(np.issubdtype(ref_a.dtype, np.integer))
    ref = _f64(ref)
    de = _f64(deformed)
    H, W = ref.shape
    N = subset_size
    nx = (W - N) // step + 1 if W >= N else 0
    ny = (H - N) // step + 1 if H >= N else 0
    nn = nx * ny
    p = np.zeros((12, ny, nx))
    z = np.zeros((ny, nx))
    it = np.zeros((ny, nx), np.int32)
    st = np.zeros((ny, nx), np.int32)
    wv = np.zeros((ny, nx), np.int32)
    sd = np.asarray(list(seeds), np.float64).reshape(-1, 4)
    so = np.zeros((max(1, len(sd)), 4))
    roi_arr = None
    roi_ptr = None
    if roi is not None:
        roi_arr = np.ascontiguousarray(roi, dtype=np.uint8)
        roi_ptr = roi_arr.ctypes.data
    t0 = time.perf_counter()
    ns = lib().orc_correlate(ref, de, W, H, roi_ptr, int_pix, N, step, shape, tol, max_iter, zncc_min, seed_radius,
                             GUESS[guess], ORDER[order], _f64(sd.ravel()) if len(sd) else np.zeros(4), len(sd),
                             int(threads), p.reshape(-1), z.reshape(-1), it.reshape(-1), st.reshape(-1),
                             wv.reshape(-1), so.reshape(-1), COST[cost], float(lm_lambda))
    dt = time.perf_counter() - t0
    if ns < 0:
        raise ValueError("no seed could be placed on an active node")
    return dict(p=p, zncc=z, iters=it, status=st, wave=wv, seed_nodes=so[:ns], nx=nx, ny=ny, seconds=dt,
                u=p[0], v=p[1], subset_size=N, step=step)


# ---- multi-window FFT initial guess (mw_oracle.c) ----------------------------
def fft2(a, inverse=False):
    """2-D radix-2 FFT of a square complex array (no 1/n scale on the inverse)."""
    a = np.asarray(a, np.complex128)
    W = a.shape[0]
    re = np.ascontiguousarray(a.real)
    im = np.ascontiguousarray(a.imag)
    lib().orc_fft2(re, im, W, 1 if inverse else -1)
    return re + 1j * im


def phase_corr(f, g):
    """Eq. (1) correlation map of two square real windows (scaled by 1/W^2)."""
    f = _f64(f)
    r = np.empty_like(f)
    lib().orc_phase_corr(f, _f64(g), f.shape[0], r)
    return r


def map_peak(r):
    """Signed peak index (qx, qy) in [-W/2, W/2) and its lead over the next value."""
    r = _f64(r)
    qx, qy, m = C.c_int(), C.c_int(), C.c_double()
    lib().orc_map_peak(r, r.shape[0], C.byref(qx), C.byref(qy), C.byref(m))
    return qx.value, qy.value, m.value


def gauss3(a, b, c):
    return float(lib().orc_gauss3(float(a), float(b), float(c)))


def mw_levels(max_disp, N, W, H):
    """(regular window sizes, node-level size) of the multi-window schedule."""
    sizes = np.zeros(32, np.int32)
    wf = C.c_int()
    n = lib().orc_mw_levels(int(max_disp), int(N), int(W), int(H), sizes, C.byref(wf))
    return [int(x) for x in sizes[:n]], wf.value


def mad_filter(u, v, ok=None, thr=2.0):
    """One MAD outlier pass over integer grid fields; returns (u, v, replaced)."""
    u = np.ascontiguousarray(u, np.int32).copy()
    v = np.ascontiguousarray(v, np.int32).copy()
    ny, nx = u.shape
    rep = np.zeros((ny, nx), np.uint8)
    okp = None
    if ok is not None:
        oka = np.ascontiguousarray(ok, np.uint8)
        okp = oka.ctypes.data
    lib().orc_mad_filter(u.reshape(-1), v.reshape(-1), okp, nx, ny, float(thr), rep.reshape(-1))
    return u, v, rep.astype(bool)


def multiwindow(ref, deformed, roi=None, *, subset_size, step, max_disp, subpixel=False, mad_threshold=2.0):
    """Multi-window FFT estimate at every node: dict of u, v, valid, margin [ny][nx] and the level sizes."""
    ref = _f64(ref)
    de = _f64(deformed)
    H, W = ref.shape
    N = subset_size
    nx = (W - N) // step + 1 if W >= N else 0
    ny = (H - N) // step + 1 if H >= N else 0
    u = np.zeros((ny, nx))
    v = np.zeros((ny, nx))
    val = np.zeros((ny, nx), np.int32)
    mg = np.zeros((ny, nx))
    lv = np.zeros(33, np.int32)
    roi_arr = None
    roi_ptr = None
    if roi is not None:
        roi_arr = np.ascontiguousarray(roi, dtype=np.uint8)
        roi_ptr = roi_arr.ctypes.data
    n = lib().orc_multiwindow(ref, de, W, H, roi_ptr, N, step, int(max_disp), int(bool(subpixel)),
                              float(mad_threshold), u.reshape(-1), v.reshape(-1), val.reshape(-1), mg.reshape(-1), lv)
    if n < 0:
        raise ValueError("the image cannot hold a node-level window")
    return dict(u=u, v=v, valid=val.astype(bool), margin=mg, levels=[int(x) for x in lv[:n]])
