"""Seeded synthetic speckle image pairs with known displacement fields.

This module is the input generator shared by the oracle tests, the GPU
parity tests and the benchmark.  It holds none of the correlation method's
arithmetic (no interpolation, no cost function, no solver): it only renders
Gaussian-blob speckle, moves the blobs by an analytic field, adds noise and
derives the region of interest and the ground truth at grid nodes.

Blob model: I(x, y) = sum_k A_k exp(-((x-X_k)^2 + (y-Y_k)^2) / (2 s_k^2)),
point-sampled at integer pixel centres (pixel (row i, col j) sits at x=j,
y=i) and truncated at radius 5 s_k.  The deformed image renders the same
blobs, unchanged in shape, at (X_k + u(X_k, Y_k), Y_k + v(X_k, Y_k)).  Noise
is independent N(0, sigma_n) per image; integer images are rounded to the
nearest integer and clipped to [0, 2^bits - 1].

Random draws: numpy Generator(PCG64(seed)); blob draw order X, Y, sigma, A;
each image's noise uses its own generator.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
import threading
from typing import Callable, Optional

import numpy as np

Field = Callable[[np.ndarray, np.ndarray], tuple]


# --------------------------------------------------------------------------
# blob rendering
# --------------------------------------------------------------------------
def _render_blobs(W: int, H: int, X, Y, S, A, chunk_px: int = 1 << 23) -> np.ndarray:
    """Sum of truncated Gaussian blobs sampled at integer pixel centres (float64)."""
    img = np.zeros(W * H, dtype=np.float64)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    S = np.asarray(S, np.float64)
    A = np.asarray(A, np.float64)
    if X.size == 0:
        return img.reshape(H, W)
    R = int(math.ceil(5.0 * float(S.max())))
    off = np.arange(-R, R + 1, dtype=np.int64)
    K = off.size
    per = max(1, chunk_px // (K * K))
    for b0 in range(0, X.size, per):
        x = X[b0:b0 + per]
        y = Y[b0:b0 + per]
        s = S[b0:b0 + per]
        a = A[b0:b0 + per]
        cx = np.floor(x).astype(np.int64)
        cy = np.floor(y).astype(np.int64)
        px = cx[:, None] + off[None, :]                  # [b, K]
        py = cy[:, None] + off[None, :]
        dx2 = (px - x[:, None]) ** 2                       # [b, K]
        dy2 = (py - y[:, None]) ** 2
        inv = 1.0 / (2.0 * s * s)
        r2 = dy2[:, :, None] + dx2[:, None, :]             # [b, K(y), K(x)]
        val = a[:, None, None] * np.exp(-r2 * inv[:, None, None])
        keep = r2 <= (25.0 * s * s)[:, None, None]
        keep &= ((px >= 0) & (px < W))[:, None, :]
        keep &= ((py >= 0) & (py < H))[:, :, None]
        lin = py[:, :, None] * W + px[:, None, :]
        img += np.bincount(lin[keep], weights=val[keep], minlength=W * H)
    return img.reshape(H, W)


_LARGE = 1 << 24          # pixels above which the C renderer and chunked finishing are used
_HERE = os.path.dirname(os.path.abspath(__file__))


_speckle = None
_speckle_lock = threading.Lock()


def _speckle_lib():
    """Compile (if needed) and load the OpenMP blob renderer used for large images.
    Callers may render from several threads: the first one builds and loads the
    library under a lock, the others reuse it."""
    global _speckle
    with _speckle_lock:
        if _speckle is not None:
            return _speckle
        src = os.path.join(_HERE, "speckle_render.c")
        lib = os.path.join(_HERE, "libspeckle.so")
        if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            tmp = lib + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
            os.replace(tmp, lib)
        L = ctypes.CDLL(lib)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.speckle_render.argtypes = [np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS"), ctypes.c_long,
                                     ctypes.c_long, dp, dp, dp, dp,
                                     np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"), ctypes.c_long,
                                     ctypes.c_double, ctypes.c_long]
        _speckle = L
        return L


def _render_blobs_large(W: int, H: int, X, Y, S, A) -> np.ndarray:
    """Same blob model as _render_blobs, float32 output, band-parallel in C."""
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    S = np.ascontiguousarray(S, np.float64)
    A = np.ascontiguousarray(A, np.float64)
    order = np.argsort(Y, kind="stable").astype(np.int64)
    img = np.empty((H, W), np.float32)
    _speckle_lib().speckle_render(img, W, H, X, Y, S, A, order, X.size, float(S.max()) if X.size else 0.0, 256)
    return img


def _finish(img: np.ndarray, noise_sigma: float, noise_seed: Optional[int], bits: Optional[int]):
    if img.size > _LARGE:
        return _finish_chunked(img, noise_sigma, noise_seed, bits)
    out = img.copy()
    if noise_sigma > 0 and noise_seed is not None:
        rng = np.random.Generator(np.random.PCG64(noise_seed))
        out += rng.normal(0.0, noise_sigma, size=out.shape)
    if bits is None:
        return out.astype(np.float32)
    out = np.clip(np.rint(out), 0, (1 << bits) - 1)
    return out.astype(np.uint8 if bits <= 8 else np.uint16)


def _finish_chunked(img: np.ndarray, noise_sigma, noise_seed, bits, rows=2048):
    """Row-chunked noise, rounding and clipping (the noise values are the same
    sequence a single draw would give)."""
    H, W = img.shape
    dt = np.float32 if bits is None else (np.uint8 if bits <= 8 else np.uint16)
    out = np.empty((H, W), dt)
    rng = np.random.Generator(np.random.PCG64(noise_seed)) if noise_sigma > 0 and noise_seed is not None else None
    for y0 in range(0, H, rows):
        blk = img[y0:y0 + rows].astype(np.float64)
        if rng is not None:
            blk += rng.normal(0.0, noise_sigma, size=blk.shape)
        if bits is None:
            out[y0:y0 + rows] = blk
        else:
            out[y0:y0 + rows] = np.clip(np.rint(blk), 0, (1 << bits) - 1)
    return out


# --------------------------------------------------------------------------
# displacement fields (absolute pixel coordinates)
# --------------------------------------------------------------------------
def field_affine(u0, v0, dudx=0.0, dudy=0.0, dvdx=0.0, dvdy=0.0, xc=0.0, yc=0.0) -> Field:
    def f(x, y):
        x = np.asarray(x, np.float64) - xc
        y = np.asarray(y, np.float64) - yc
        return u0 + dudx * x + dudy * y, v0 + dvdx * x + dvdy * y
    f.grad = lambda x, y: (np.full_like(np.asarray(x, np.float64), dudx), np.full_like(np.asarray(x, np.float64), dudy),
                           np.full_like(np.asarray(x, np.float64), dvdx), np.full_like(np.asarray(x, np.float64), dvdy))
    return f


def field_c1() -> Field:
    """u = 1.37 + 0.002 x, v = -0.81 + 0.001 y."""
    return field_affine(1.37, -0.81, dudx=0.002, dvdy=0.001)


def field_sine(H: int, amp=0.5, lam0=10.0, lam1=300.0) -> Field:
    """u = amp sin(2 pi x / lam(y)), lam(y) = lam0 + (lam1-lam0) y/(H-1), v = 0."""
    def lam(y):
        return lam0 + (lam1 - lam0) * np.asarray(y, np.float64) / (H - 1)

    def f(x, y):
        x = np.asarray(x, np.float64)
        return amp * np.sin(2 * np.pi * x / lam(y)), np.zeros_like(x)

    def grad(x, y):
        x = np.asarray(x, np.float64)
        L = lam(y)
        ph = 2 * np.pi * x / L
        dudx = amp * np.cos(ph) * 2 * np.pi / L
        dudy = amp * np.cos(ph) * (-2 * np.pi * x / L ** 2) * (lam1 - lam0) / (H - 1)
        z = np.zeros_like(x)
        return dudx, dudy, z, z
    f.grad = grad
    return f


def field_quadratic_c3(W: int, H: int) -> Field:
    """Centred x~ = x - W/2, y~ = y - H/2:
    u = 1e-5 x~^2 + 0.3 + 0.02 x~,  v = -2e-5 x~ y~ + 0.2 + 0.02 y~."""
    xc, yc = W / 2.0, H / 2.0

    def f(x, y):
        xt = np.asarray(x, np.float64) - xc
        yt = np.asarray(y, np.float64) - yc
        return 1e-5 * xt * xt + 0.3 + 0.02 * xt, -2e-5 * xt * yt + 0.2 + 0.02 * yt

    def grad(x, y):
        xt = np.asarray(x, np.float64) - xc
        yt = np.asarray(y, np.float64) - yc
        return 2e-5 * xt + 0.02, np.zeros_like(xt), -2e-5 * yt, -2e-5 * xt + 0.02
    f.grad = grad
    return f


def field_large(W: int, H: int) -> Field:
    """A displacement far beyond any subset: translation (0.1526 W, -0.0915 H)
    (312.6, -187.3 px at 2048^2) plus 1 % / -0.5 % normal strain about the centre."""
    return field_affine(0.1526 * W, -0.0915 * H, dudx=0.01, dvdy=-0.005, xc=W / 2.0, yc=H / 2.0)


def field_bump_c4(W: int, H: int, t=(3.41, -7.92), amp=0.8, width=4000.0) -> Field:
    """(u, v) = (t_x + amp exp(-r^2 / (2 width^2)), t_y), r from the image centre."""
    xc, yc = W / 2.0, H / 2.0

    def f(x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        r2 = (x - xc) ** 2 + (y - yc) ** 2
        return t[0] + amp * np.exp(-r2 / (2 * width * width)), np.full_like(x, t[1])

    def grad(x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        r2 = (x - xc) ** 2 + (y - yc) ** 2
        e = amp * np.exp(-r2 / (2 * width * width))
        z = np.zeros_like(x)
        return -e * (x - xc) / width ** 2, -e * (y - yc) / width ** 2, z, z
    f.grad = grad
    return f


# --------------------------------------------------------------------------
# pairs, ROI, grid, ground truth
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Pair:
    ref: np.ndarray
    deformed: np.ndarray
    roi: np.ndarray           # uint8 [H][W], 1 = inside
    field: Field
    bits: Optional[int]


def draw_blobs(W, H, nblobs, sigma, amp, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(0.0, W, nblobs)
    Y = rng.uniform(0.0, H, nblobs)
    S = rng.uniform(sigma[0], sigma[1], nblobs)
    A = rng.uniform(amp[0], amp[1], nblobs)
    return X, Y, S, A


def roi_from_field(W: int, H: int, field: Field, margin: int = 4, rows: int = 1024) -> np.ndarray:
    """Pixels >= margin inside the image whose displaced position is also >= margin inside."""
    out = np.empty((H, W), np.uint8)
    lo = margin
    xx = np.arange(W, dtype=np.float64)[None, :]
    for y0 in range(0, H, rows):
        yy = np.arange(y0, min(H, y0 + rows), dtype=np.float64)[:, None]
        X = np.broadcast_to(xx, (yy.shape[0], W))
        Y = np.broadcast_to(yy, (yy.shape[0], W))
        u, v = field(X, Y)
        ok = (X >= lo) & (X <= W - 1 - lo) & (Y >= lo) & (Y <= H - 1 - lo)
        ok &= (X + u >= lo) & (X + u <= W - 1 - lo) & (Y + v >= lo) & (Y + v <= H - 1 - lo)
        out[y0:y0 + yy.shape[0]] = ok
    return out


def make_pair(W, H, nblobs, sigma, amp, field: Field, noise_sigma, bits, seed_blobs,
              seed_noise_ref, seed_noise_def, roi_margin=4) -> Pair:
    X, Y, S, A = draw_blobs(W, H, nblobs, sigma, amp, seed_blobs)
    render = _render_blobs_large if W * H > _LARGE else _render_blobs
    ref = render(W, H, X, Y, S, A)
    u, v = field(X, Y)
    de = render(W, H, X + u, Y + v, S, A)
    return Pair(_finish(ref, noise_sigma, seed_noise_ref, bits),
                _finish(de, noise_sigma, seed_noise_def, bits),
                roi_from_field(W, H, field, roi_margin), field, bits)


def noise_frames(w, nframes):
    """Reference plus `nframes` deformed frames of workload `w` that differ only
    in their noise (noise seeds seed_noise_def + i; frame 0 is w.pair()'s
    deformed image), and the ROI.  The blobs are rendered once."""
    X, Y, S, A = draw_blobs(w.W, w.H, w.nblobs, w.sigma, w.amp, w.seed_blobs)
    render = _render_blobs_large if w.W * w.H > _LARGE else _render_blobs
    f = w.field()
    u, v = f(X, Y)
    ref = _finish(render(w.W, w.H, X, Y, S, A), w.noise, w.seed_noise_ref, w.bits)
    clean = render(w.W, w.H, X + u, Y + v, S, A)
    frames = [_finish(clean, w.noise, w.seed_noise_def + i, w.bits) for i in range(nframes)]
    return ref, frames, roi_from_field(w.W, w.H, f)


def displacement_grid(nx, ny, step, kind="smooth", noise=0.0, invalid=0.0, seed=0):
    """Seeded displacement fields u, v [ny][nx] (float32) on a node grid of the
    given step, and a status array (int8, 0 = valid, 3 = not converged) with a
    fraction `invalid` of invalid nodes: inputs for the strain step.
    kinds: "smooth" (sinusoids and a quadratic, strain ~1e-2), "rotation"
    (rotation by 0.3 rad with 4 % / -2 % stretch about the grid centre), "shear"
    (simple shear 0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = np.meshgrid(np.arange(nx) * float(step), np.arange(ny) * float(step))
    Xc, Yc = X - X.mean(), Y - Y.mean()
    if kind == "smooth":
        u = 0.8 + 0.01 * Xc - 0.004 * Yc + 2e-5 * Xc * Xc + 0.3 * np.sin(2 * np.pi * Y / 400.0)
        v = -0.3 + 0.006 * Xc + 0.015 * Yc - 3e-5 * Xc * Yc + 0.2 * np.cos(2 * np.pi * X / 300.0)
    elif kind == "rotation":
        c, s = np.cos(0.3), np.sin(0.3)
        a, d = 1.04, 0.98
        u = (c * a - 1.0) * Xc - s * d * Yc
        v = s * a * Xc + (c * d - 1.0) * Yc
    elif kind == "shear":
        u, v = 0.1 * Yc, 0.0 * Xc
    else:
        raise ValueError(kind)
    if noise > 0:
        u = u + rng.normal(0.0, noise, u.shape)
        v = v + rng.normal(0.0, noise, v.shape)
    status = np.where(rng.uniform(size=u.shape) < invalid, 3, 0).astype(np.int8)
    return u.astype(np.float32), v.astype(np.float32), status


def grid_shape(W, H, N, step):
    """Nodes at x_c = h + i*step, i < nx = floor((W-N)/step)+1 (y likewise), h=(N-1)/2."""
    nx = (W - N) // step + 1 if W >= N else 0
    ny = (H - N) // step + 1 if H >= N else 0
    return nx, ny


def node_centres(W, H, N, step):
    nx, ny = grid_shape(W, H, N, step)
    h = (N - 1) // 2
    xs = h + step * np.arange(nx)
    ys = h + step * np.arange(ny)
    return xs, ys


def truth_at_nodes(field: Field, W, H, N, step):
    """Ground-truth (u, v, du/dx, du/dy, dv/dx, dv/dy) at every node centre, [ny][nx] arrays."""
    xs, ys = node_centres(W, H, N, step)
    X, Y = np.meshgrid(xs.astype(np.float64), ys.astype(np.float64))
    u, v = field(X, Y)
    g = field.grad(X, Y) if hasattr(field, "grad") else (None,) * 4
    return u, v, g


# --------------------------------------------------------------------------
# the workloads (sizes, speckle statistics and fields as specified per config)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    W: int
    H: int
    bits: int
    nblobs: int
    sigma: tuple
    amp: tuple
    noise: float
    N: int
    step: int
    shape: int
    tol: float
    max_iter: int
    zncc_min: float
    seed_radius: int
    seeds: list               # [(x, y, u0, v0)]
    seed_blobs: int
    seed_noise_ref: int
    seed_noise_def: int
    field_name: str
    max_disp: int = 0         # multi-window FFT: estimate of the largest displacement (0: not used)

    def field(self) -> Field:
        if self.field_name == "c1":
            return field_c1()
        if self.field_name == "sine":
            return field_sine(self.H)
        if self.field_name == "quad":
            return field_quadratic_c3(self.W, self.H)
        if self.field_name == "bump":
            return field_bump_c4(self.W, self.H)
        if self.field_name == "large":
            return field_large(self.W, self.H)
        raise ValueError(self.field_name)

    def pair(self) -> Pair:
        return make_pair(self.W, self.H, self.nblobs, self.sigma, self.amp, self.field(), self.noise,
                         self.bits, self.seed_blobs, self.seed_noise_ref, self.seed_noise_def)

    def params(self) -> dict:
        return dict(subset_size=self.N, step=self.step, shape=self.shape, tol=self.tol,
                    max_iter=self.max_iter, zncc_min=self.zncc_min, seed_radius=self.seed_radius)


def workload(name: str, size: Optional[int] = None, **over) -> Workload:
    """Named workloads.  `size` shrinks the image (blob count scaled to keep the density)."""
    if name == "c1":        # 512^2 u8 speckle, affine field, subset 21 step 5
        W = size or 512
        d = dict(name="c1", W=W, H=W, bits=8, nblobs=int(round(3000 * W * W / 512 ** 2)), sigma=(2.0, 4.0),
                 amp=(60.0, 200.0), noise=2.0, N=21, step=5, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
                 seed_radius=8, seeds=[(W / 2, W / 2, 0.0, 0.0)], seed_blobs=1001, seed_noise_ref=1002,
                 seed_noise_def=1003, field_name="c1")
    elif name == "c2":      # 2048^2 12-bit speckle, sinusoidal u, subset 31 step 2
        W = size or 2048
        d = dict(name="c2", W=W, H=W, bits=12, nblobs=int(round(48000 * W * W / 2048 ** 2)), sigma=(2.0, 4.0),
                 amp=(960.0, 3200.0), noise=4.0, N=31, step=2, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
                 seed_radius=4, seeds=[(W / 2, W / 2, 0.0, 0.0)], seed_blobs=2001, seed_noise_ref=2002,
                 seed_noise_def=2003, field_name="sine")
    elif name == "c3":      # 4096^2 u8 speckle, quadratic field + 2 % strain, subsets 21/41 step 4
        W = size or 4096
        d = dict(name="c3", W=W, H=W, bits=8, nblobs=int(round(192000 * W * W / 4096 ** 2)), sigma=(2.0, 4.0),
                 amp=(60.0, 200.0), noise=2.0, N=21, step=4, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
                 seed_radius=4, seeds=[(W / 2, W / 2, 0.3, 0.2)], seed_blobs=3001, seed_noise_ref=3002,
                 seed_noise_def=3003, field_name="quad")
    elif name == "c4":      # 32768^2 u8 speckle, rigid shift + Gaussian bump, subset 41 step 20, 16 seeds
        W = size or 32768
        seeds = [((i + 0.5) * W / 4, (j + 0.5) * W / 4, 3.41, -7.92) for j in range(4) for i in range(4)]
        d = dict(name="c4", W=W, H=W, bits=8, nblobs=int(round(0.02 * W * W)), sigma=(1.5, 3.0),
                 amp=(60.0, 200.0), noise=2.0, N=41, step=20, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
                 seed_radius=12, seeds=seeds, seed_blobs=4001, seed_noise_ref=4002, seed_noise_def=4003,
                 field_name="bump")
    elif name == "large":   # 2048^2 u8 speckle, translation of ~0.15 image widths: multi-window FFT seeding
        W = size or 2048
        # dense SEM-like speckle (0.03 blobs/px^2, sigma 1.5-3 px): a 32-px window holds enough
        # texture for its phase-correlation peak
        d = dict(name="large", W=W, H=W, bits=8, nblobs=int(round(0.03 * W * W)), sigma=(1.5, 3.0),
                 amp=(60.0, 200.0), noise=2.0, N=31, step=8, shape=6, tol=1e-4, max_iter=50, zncc_min=0.7,
                 seed_radius=8, seeds=[(W / 2, W / 2, 0.0, 0.0)], seed_blobs=6001, seed_noise_ref=6002,
                 seed_noise_def=6003, field_name="large", max_disp=int(round(0.3125 * W)))
    else:
        raise ValueError(name)
    d.update(over)
    return Workload(**d)


# --------------------------------------------------------------------------
# serving mix: resident 4096^2 references, requests on centred windows
# --------------------------------------------------------------------------
SERVE_REF_SIZE = 4096
SERVE_SIZES = (256, 512, 1024, 2048, 4096)
SERVE_SUBSETS = (15, 21, 31, 51)
SERVE_STEPS = (1, 2, 5)
SERVE_DENSITY = 3000 / 512 ** 2          # blobs per px^2, as the 512^2 u8 workload


@dataclasses.dataclass
class ServeRequest:
    index: int
    arrival: float            # seconds from the start of the run
    ref: int                  # 0..7
    S: int                    # window side
    N: int
    step: int
    t: tuple                  # (tx, ty) at the window centre
    grad: tuple               # (du/dx, du/dy, dv/dx, dv/dy) about the window centre

    def field(self) -> Field:
        c = self.S / 2.0
        return field_affine(self.t[0], self.t[1], *self.grad, xc=c, yc=c)


def serve_trace(duration: float = 60.0, rate: float = 20.0, seed: int = 5000, nrefs: int = 8):
    """Poisson arrivals at `rate` per second over `duration` seconds; each request
    draws a reference, a window size, a subset size and a step uniformly, a
    translation uniform in the disc of radius 5 px and gradient entries uniform
    in [-0.01, 0.01]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        ref = int(rng.integers(nrefs))
        S = int(SERVE_SIZES[rng.integers(len(SERVE_SIZES))])
        N = int(SERVE_SUBSETS[rng.integers(len(SERVE_SUBSETS))])
        st = int(SERVE_STEPS[rng.integers(len(SERVE_STEPS))])
        r = 5.0 * math.sqrt(rng.uniform())
        a = rng.uniform(0.0, 2.0 * math.pi)
        g = tuple(float(x) for x in rng.uniform(-0.01, 0.01, 4))
        out.append(ServeRequest(len(out), t, ref, S, N, st, (r * math.cos(a), r * math.sin(a)), g))
    return out


def serve_reference_blobs(ref: int):
    W = SERVE_REF_SIZE
    return draw_blobs(W, W, int(round(SERVE_DENSITY * W * W)), (2.0, 4.0), (60.0, 200.0), 5001 + ref)


def serve_reference(ref: int, blobs=None) -> np.ndarray:
    """The 4096^2 u8 reference image `ref` (blob seed 5001+ref, noise seed 5011+ref)."""
    W = SERVE_REF_SIZE
    X, Y, S, A = blobs if blobs is not None else serve_reference_blobs(ref)
    return _finish(_render_blobs_large(W, W, X, Y, S, A), 2.0, 5011 + ref, 8)


def serve_window(S: int):
    """Origin of the centred S x S window in the reference."""
    return (SERVE_REF_SIZE - S) // 2


def serve_margin(S: int) -> int:
    """ROI margin of a window: 4 px of interpolation support plus the largest
    displacement the request fields reach (5 px + 0.02 * S / 2)."""
    return 10 + int(math.ceil(0.01 * S))


def serve_roi(S: int) -> np.ndarray:
    m = serve_margin(S)
    roi = np.zeros((S, S), np.uint8)
    roi[m:S - m, m:S - m] = 1
    return roi


def serve_frame(req: ServeRequest, blobs) -> np.ndarray:
    """Deformed S x S window of request `req` (noise seed 5100 + index): the
    reference blobs near the window, moved by the request's field evaluated at
    their reference position, in window coordinates."""
    X, Y, S_, A = blobs
    o = serve_window(req.S)
    pad = 64.0
    sel = (X >= o - pad) & (X < o + req.S + pad) & (Y >= o - pad) & (Y < o + req.S + pad)
    x, y = X[sel] - o, Y[sel] - o
    u, v = req.field()(x, y)
    img = _render_blobs_large(req.S, req.S, x + u, y + v, S_[sel], A[sel])
    return _finish(img, 2.0, 5100 + req.index, 8)
