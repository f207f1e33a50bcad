// Internal interface between the host engine (dic_engine.hip) and the
// gfx950 kernels (dic_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace dicmi {

// Coefficient arrays carry this many mirrored samples on every side, so that
// the 4x4 taps of any in-image point (x0-1 .. x0+2) never need index folding.
constexpr int kPad = 4;
// Fourth word of a raw buffer descriptor on this GPU family (32-bit data format,
// no swizzle); with stride 0 the descriptor is a plain byte-addressed view.
constexpr int kBufferWord3 = 0x00020000;
// The wave kernels stage a coefficient window with 32-bit byte offsets from its
// origin, so the window side times the coefficient row pitch, in bytes, must stay
// below 2^31.
// Row pitch of the LDS coefficient window: the smallest value >= the window side
// congruent to the subset size N modulo 32.  Thread i of a subset reads column
// i mod N of subset row i div N, so with this pitch the threads of a wavefront
// over an untransformed subset fall on consecutive LDS banks (a quarter fewer
// bank conflicts than with the window side as pitch; modulo 64 measured the
// same).  Windows whose padded size would pass 32 KiB keep the unpadded pitch.
inline int lds_pitch(int N, int ts)
{
    const int lp = ts + (((N - ts) % 32) + 32) % 32;
    return lp * ts <= 8192 ? lp : ts;
}
// The wave kernel addresses a subset's coefficient window (ts rows of cpitch
// floats) and its reference rows (N rows of ppitch interleaved 12-byte pixels)
// with 32-bit buffer offsets from the subset's corner.
inline bool buffer_offsets_fit(int64_t cpitch, int ts, int64_t ppitch, int N)
{
    return 4 * cpitch * ts <= 0x7fffffffLL && 12 * ppitch * N <= 0x7fffffffLL;
}
// Frames one batched launch may carry (the frame table travels in the kernel
// arguments, which hold at most 4 KiB).
constexpr int kMaxFrames = 32;

enum NodeStatus : int8_t {
    kConverged = 0,
    kNotReached = 1,
    kNotInRoi = 2,
    kMaxIter = 3,
    kLowZncc = 4,
    kOutOfBounds = 5,
    kFlatRef = 6,
    kFlatDef = 7,
    kSingular = 8,
    kNan = 9
};

// Per-node reference cache, doubles, structure of arrays [slot][node]:
//   slot 0       f_m     subset mean of the reference intensities
//   slot 1       df2     sum (f_i - f_m)^2 (formed exactly like the iteration's dg2)
//   slot 2       Sfb     sum fbar_i
//   slots 3..    SJ[np]  sum J_i          (steepest-descent images, Eq. (5) order)
//   next np      SJf[np] sum J_i fbar_i, centred like the iteration's sums
//   next np(np+1)/2      inverse of the Gauss-Newton Hessian, upper triangle row-major
inline int cache_slots(int np) { return 3 + 2 * np + np * (np + 1) / 2; }

struct RefView {
    const float *coef;   // reference spline coefficients at (0,0) of a padded array
    int64_t cpitch;      // elements per coefficient row
    const float *pa;     // per pixel the reference interpolant and its x and y derivatives,
                         // interleaved: [H][ppitch][3]
    int64_t ppitch;      // pixels per row of pa
    const double *cache; // [cache_slots][nodes]
    const int8_t *flag;  // per node: -1 inactive, 0 usable, else a NodeStatus
    const void *raw;     // resident copy of the raw reference pixels [H][W]
    int pixel;           // dic_pixel of raw
    int W, H, N, step, nx, ny;
    int64_t nodes;
    // iteration parameters of the context that owns this reference
    int max_iter;
    double tol2;         // tol^2 (the norm is compared squared)
    float zncc_min;
    int guess_copy;      // 1: copy the neighbour's p, 0: extrapolate
    int half;            // deformed coefficients stored as FP16
    int ts;              // side of the LDS coefficient window
    int lp;              // LDS row pitch of that window (lds_pitch(N, ts))
    double inv_n;        // 1 / (N * N), correctly rounded
    int cost;            // 0 ZNSSD (Eq. (4)), 1 NSSD (Eq. (3)), 2 SSD (Eq. (2)); the variant kernel only
    double lm_lambda;    // initial Levenberg-Marquardt damping (0: Gauss-Newton); the variant kernel only
};

// Device-resident state of one frame of a (batched) correlation.
struct FrameState {
    const void *dcoef;    // deformed coefficients at (0,0) of a padded array (float or __half)
    int64_t dpitch;       // elements per row
    const void *draw;     // raw deformed pixels
    int64_t draw_pitch;   // bytes per row
    int dpixel;
    float *p;             // [np][nodes]
    float *zncc;
    int16_t *iters;
    int8_t *status;
    int32_t *wave;
    uint64_t *pkey;       // parent key of every node (ordered ZNCC << 2 | direction priority)
    int32_t *list0, *list1; // frontier ping-pong lists
    int32_t *counts;      // counts[k] = size of wave k
    double *seed_p;       // [nseeds][2]
    int32_t *seed_nodes;  // [nseeds]
    int32_t nseeds;
    unsigned long long *stat; // [0] computed, [1] converged, [2] iterations
    const RefView *ref;   // DEVICE copy of the reference view this frame correlates against
    int k_base;           // launch step at which this frame's wave 0 runs (wave = step - k_base)
    int kmax;             // last valid index of counts (nodes + 1)
};

// What a wave kernel reads of a frame (FrameState without the raw image and the
// seed list, which only the seed search reads): 120 bytes, so that 32 frames fit
// the 4 KiB of kernel arguments.
struct WaveFrame {
    const void *dcoef;
    int64_t dpitch;
    float *p;
    float *zncc;
    int16_t *iters;
    int8_t *status;
    int32_t *wave;
    uint64_t *pkey;
    int32_t *list0, *list1;
    int32_t *counts;
    double *seed_p;
    unsigned long long *stat;
    const RefView *ref;
    int k_base;
    int kmax;
    WaveFrame() = default;
    WaveFrame(const FrameState &F)
        : dcoef(F.dcoef), dpitch(F.dpitch), p(F.p), zncc(F.zncc), iters(F.iters), status(F.status), wave(F.wave),
          pkey(F.pkey), list0(F.list0), list1(F.list1), counts(F.counts), seed_p(F.seed_p), stat(F.stat),
          ref(F.ref), k_base(F.k_base), kmax(F.kmax)
    {
    }
};

// The frames of one launch, passed by value as a kernel argument: uniform
// indexing gives scalar loads, and the pointers are known to be global.
struct FrameTable {
    WaveFrame f[kMaxFrames];
    int n;
};
static_assert(sizeof(FrameTable) + sizeof(int) <= 4096, "the frame table must fit the kernel arguments");

// ---- launchers (dic_kernels.hip) -------------------------------------
void launch_prefilter(const void *src, int64_t src_pitch_bytes, int pixel, int W, int H, float *tmp,
                      int64_t tmp_pitch, void *dst_at_origin, int64_t dst_pitch, bool half, hipStream_t s);
void launch_ref_pixels(const RefView &R, float *pa, hipStream_t s);
// copies component a (0 interpolant, 1 x derivative, 2 y derivative) of the interleaved
// reference array to out [H][W]
void launch_ref_component(const RefView &R, int a, float *out, hipStream_t s);
void launch_active(const uint8_t *roi, const RefView &R, int8_t *flag, hipStream_t s);
bool launch_ref_nodes(const RefView &R, int np, int tps, double *cache, int8_t *flag, hipStream_t s);
void launch_init_frame(const RefView &R, const FrameState &F, int np, hipStream_t s);
void launch_seed_search(const RefView &R, const FrameState *F_dev, int nframes, int nseeds, int radius,
                        const int32_t *seed_center_dev, double *zbuf, hipStream_t s);
void launch_seed_pick(const RefView &R, const FrameState *F_dev, int nframes, int nseeds, int radius,
                      const int32_t *seed_center_dev, const double *zbuf, hipStream_t s);
// max_ts: the largest window side of the launch's frames; lds_floats: the largest
// window footprint in LDS (side times lds_pitch) among them
bool launch_wave(const FrameTable &F, int step, int np, int N, int tps, bool f64, int max_ts, int lds_floats,
                 int grid, hipStream_t s);
void launch_gather_next(const FrameState *F_dev, int n, int step, int32_t *out, hipStream_t s);
void launch_frame_stats(const RefView &R, const FrameState &F, hipStream_t s);
void launch_count_wave(const FrameState *F_dev, int nframes, int k, int32_t *out, hipStream_t s);
void launch_zero32(void *p, int64_t words, hipStream_t s);
int pixels_per_thread(int N, int T);
void launch_finalize(const RefView &R, const FrameState &F, int np, bool nan_unconverged, hipStream_t s);
int wave_grid_hint(int np, int tps, int device, int chains);
bool supported_tps(int N, int tps);
// the variants' wave kernel (rigid shape, NSSD / SSD, Levenberg-Marquardt; dic_variants.hip)
bool launch_wave_var(const FrameTable &F, int step, int np, int grid, hipStream_t s);
int tile_side(int N);

} // namespace dicmi
