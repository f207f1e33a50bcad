/*
 * dic.h -- C ABI of the MI355X (gfx950) reliability-guided 2D digital image
 * correlation library.
 *
 * The library computes, for every node of a regular grid of square subsets
 * inside a region of interest, the shape-function parameters that map the
 * reference subset onto the deformed image (Hirst et al., arXiv 2601.12941,
 * Sec. 2.2): cubic B-spline gray-level interpolation, the zero-normalised
 * sum of squared differences of Eq. (4) as the cost, the affine or quadratic
 * shape function of Eq. (5) (parameters p0..p11 in that equation's order),
 * per-subset inverse-compositional Gauss-Newton minimisation, and
 * reliability-guided propagation of initial guesses from a seed to
 * 4-neighbours (Sec. 2.4), processed as breadth-first frontier waves.
 *
 * Conventions
 *   - Pixel (row i, column j) sits at x = j, y = i.  Nodes sit at
 *     x_c = h + i*step (i < nx = floor((W-N)/step)+1), y likewise, with
 *     h = (N-1)/2; result arrays are row-major [ny][nx].
 *   - Every image, mask and result pointer is DEVICE memory on the context's
 *     device, owned by the caller.  Seeds are a HOST array.
 *   - All work is ordered on the context's HIP stream; every call that
 *     launches work returns after it has completed.
 *   - Errors: negative dic_status, with a message in dic_last_error().  After
 *     DIC_E_INVAL, DIC_E_NOSEED or DIC_E_UNSUPPORTED the context stays usable;
 *     after DIC_E_DEVICE it must be destroyed.  Output contents are undefined
 *     after any error.
 *   - One context must not be used from two host threads at once.
 */
#ifndef DIC_H
#define DIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dic_ctx dic_ctx; /* opaque: owns the reference precompute and all scratch */

typedef enum {
    DIC_OK = 0,
    DIC_E_INVAL = -1,       /* bad argument, size or call order inside one call */
    DIC_E_NOMEM = -2,       /* device allocation failed */
    DIC_E_DEVICE = -3,      /* HIP runtime or kernel error */
    DIC_E_STATE = -4,       /* dic_correlate before dic_set_reference */
    DIC_E_NOSEED = -5,      /* no seed lies on an active node */
    DIC_E_UNSUPPORTED = -6  /* valid but not built (e.g. a variant in the serving loop) */
} dic_status;

typedef enum { DIC_PIX_U8 = 0, DIC_PIX_U16 = 1, DIC_PIX_F32 = 2 } dic_pixel;

/* Shape functions of Eq. (5); the value is the parameter count. */
typedef enum { DIC_SHAPE_RIGID = 2, DIC_SHAPE_AFFINE = 6, DIC_SHAPE_QUADRATIC = 12 } dic_shape;

/* Per-node status codes (dic_result.status). */
enum {
    DIC_NODE_CONVERGED = 0,     /* increment norm below tol and ZNCC >= zncc_min */
    DIC_NODE_NOT_REACHED = 1,   /* active but never given a guess by propagation */
    DIC_NODE_NOT_IN_ROI = 2,    /* some subset pixel outside the ROI mask */
    DIC_NODE_MAX_ITER = 3,      /* max_iter iterations without convergence */
    DIC_NODE_LOW_ZNCC = 4,      /* converged with ZNCC < zncc_min */
    DIC_NODE_OUT_OF_BOUNDS = 5, /* a warped pixel left [0, W-1] x [0, H-1] */
    DIC_NODE_FLAT_REF = 6,      /* reference subset RMS deviation < 1e-6 of its mean level */
    DIC_NODE_FLAT_DEF = 7,      /* same for the warped deformed subset */
    DIC_NODE_SINGULAR = 8,      /* Gauss-Newton Hessian not positive definite */
    DIC_NODE_NAN = 9            /* NaN in the data or the iteration */
};

/* A 2-D image in device memory. */
typedef struct {
    int32_t width, height;
    int64_t pitch_bytes;  /* distance between rows, >= width * pixel size */
    int32_t pixel;        /* dic_pixel */
    const void *data;     /* DEVICE pointer to row 0 */
} dic_image;

/* Correlation parameters (Listing 1's subset size / step, Sec. 2.2's
 * convergence threshold and iteration cap, Eq. (5)'s shape function). */
typedef struct {
    int32_t subset_size;        /* N: odd, 5 <= N <= 63 */
    int32_t step;               /* grid step in pixels, >= 1 */
    int32_t shape;              /* dic_shape: rigid, affine or quadratic (Eq. (5)) */
    int32_t max_iter;           /* >= 1 */
    double tol;                 /* convergence threshold on |dp| in pixels (see dic_correlate) */
    double zncc_min;            /* a converged subset with lower ZNCC is LOW_ZNCC and does not propagate */
    int32_t seed_radius;        /* integer search radius R of the seed initialisation, 0..64 */
    int32_t guess_mode;         /* 0: extrapolate the neighbour's shape function, 1: copy it */
    int32_t coef_fp16;          /* 1: deformed-image spline coefficients stored as FP16 */
    int32_t reduce_fp64;        /* 1: cross-lane sums and the normal-equation solve in FP64; 0: FP32 */
    int32_t nan_unconverged;    /* 1: write NaN into p of every node that is not CONVERGED */
    int32_t threads_per_subset; /* 0 = automatic; else 64, 128 or 256 threads (one workgroup) per subset,
                                   or 16 / 32: four / two subsets share one 64-lane wavefront
                                   (affine shape, N <= 16) */
    int32_t tile_side;          /* side of the LDS window of deformed coefficients, in samples:
                                   0 = automatic (N + 9: the taps' reach and 3 samples of drift
                                   room on each side), else
                                   N + 5 .. 96; a warped subset that does not fit reads global memory */
    int32_t cost;               /* dic_cost: the criterion each subset minimises (Sec. 2.2) */
    double lm_lambda;           /* 0: Gauss-Newton increments; > 0: Levenberg-Marquardt with this initial
                                   damping: (H + lambda diag H) dp = -b; an evaluation whose undamped
                                   increment is not longer (convergence norm) than at the last accepted one is
                                   accepted and divides lambda by 10, else lambda * 10 and the step is retaken
                                   from the last accepted p; an accepted evaluation with an undamped increment
                                   below tol takes it and converges; the reported ZNCC is the last accepted */
} dic_params;

/* Costs of Sec. 2.2.  Every cost reports the ZNCC (1 - ZNSSD/2) as its
 * correlation coefficient, which also ranks the propagation and is compared
 * with zncc_min; the seed search is an integer ZNCC search for every cost.
 * The rigid shape, NSSD, SSD and lm_lambda > 0 run on a general kernel (one
 * 256-thread workgroup per subset, FP64 sums; threads_per_subset must be 0 or
 * 256, tile_side and reduce_fp64 are ignored); ZNSSD with the affine or
 * quadratic shape and lm_lambda = 0 runs on the tuned kernels. */
typedef enum {
    DIC_COST_ZNSSD = 0, /* Eq. (4): zero-normalised SSD, residual fbar - (|fbar|/|gbar|) gbar */
    DIC_COST_NSSD = 1,  /* Eq. (3): normalised SSD, residual f - (|f|/|g|) g */
    DIC_COST_SSD = 2    /* Eq. (2): residual f - g */
} dic_cost;

/* A seed: a point near which propagation starts (snapped to the nearest
 * active node) and a guess (u0, v0) for the centre of its integer search. */
typedef struct {
    double x, y, u0, v0;
} dic_seed;

/* Caller-allocated DEVICE result arrays, each [ny][nx] row-major (p is
 * [shape][ny][nx]: plane k holds parameter p_k of Eq. (5)). */
typedef struct {
    float *p;
    float *zncc;      /* zero-normalised cross-correlation 1 - ZNSSD/2 at the last evaluated p */
    int16_t *iters;   /* IC-GN iterations performed (0 if never computed) */
    int8_t *status;   /* DIC_NODE_* */
    int32_t *wave;    /* frontier wave that computed the node (0 = seed), -1 if never computed */
} dic_result;

typedef struct {
    int64_t nodes;          /* nx * ny */
    int64_t active;         /* nodes whose subset lies inside the ROI */
    int64_t computed;       /* nodes on which IC-GN ran (all frames of the last call) */
    int64_t converged;      /* CONVERGED nodes (all frames of the last call) */
    int64_t iterations;     /* total IC-GN iterations (all frames of the last call) */
    int32_t waves;          /* frontier waves launched by the last call */
    int32_t frames;         /* frames in the last call */
    int32_t threads_per_subset;
    int32_t seed_du, seed_dv; /* integer seed shift of the first seed of the last frame */
    double ms_total;        /* device time of the last call (HIP events) */
    double ms_icgn;         /* device time from the first to the last IC-GN wave kernel */
    double ms_prefilter;    /* device time of the deformed-image prefilter */
    double ms_wave_kernels; /* device time of the chunks of back-to-back wave launches, host gaps excluded */
    int32_t wave_launches;  /* IC-GN wave steps of the last call: one wave kernel launch per step and
                               launch chain, counting the up to two steps launched ahead of the
                               host's last wave-size read, which find no subset */
    int32_t launch_chains;  /* streams the wave launches of the last call ran on: a batched call of
                               16, 32, 48 or 64 frames, or of more than 32, runs its two halves as two
                               chains, each frame's waves in order on its chain's stream; otherwise 1 */
} dic_stats;

/* Create a context on HIP device `device`, ordering its work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
dic_status dic_create(dic_ctx **out, int device, void *hip_stream);

/*
 * Set (or replace) the reference image, ROI and parameters.  Computes and
 * keeps resident: the reference spline coefficients (Sec. 2.2), the
 * reference intensities and gradients at every pixel, and per node the
 * subset mean and norm, the Gauss-Newton Hessian's inverse and the sums the
 * iteration reuses.  roi_mask_dev: DEVICE uint8 [height][width] (pitch =
 * width), nonzero = inside; NULL = whole image.  A node is active iff all N^2
 * of its pixels are inside.  DIC_E_INVAL, before any state changes, when the
 * image is too wide for the 32-bit offsets a subset is addressed with:
 * 12 * P * N and 4 * Q * T must stay below 2^31, with P = width rounded up to
 * 64, Q = width + 8 rounded up to 64, N the subset size and T the window side
 * (about 5.7 M pixels of width at N = 31).
 */
dic_status dic_set_reference(dic_ctx *c, const dic_image *ref, const uint8_t *roi_mask_dev, const dic_params *prm);

/* Grid of the current reference: nx, ny, the first node centre (x0, y0) and
 * the step.  Any pointer may be NULL. */
dic_status dic_grid_shape(const dic_ctx *c, int32_t *nx, int32_t *ny, int32_t *x0, int32_t *y0, int32_t *step);

/* Copies of the current reference's precompute, for inspection (Sec. 2.2's
 * cubic B-spline interpolation of the reference): each non-NULL output is a
 * caller-allocated DEVICE array [height][width] (pitch = width) of FP32.
 *   coef_out: the prefilter's coefficients as stored, 1/36 of the classical
 *             B-spline coefficients (the interpolation weights are 6 times the
 *             B-spline's on each axis, so the interpolant is unchanged);
 *   f_out, fx_out, fy_out: the interpolant and its x and y derivatives at every
 *             integer pixel (the reference values and gradients the iteration
 *             uses).
 * DIC_E_STATE before dic_set_reference. */
dic_status dic_reference_arrays(dic_ctx *c, float *coef_out, float *f_out, float *fx_out, float *fy_out);

/* Node grid of a width x height image for a subset size and step, without a
 * context (nodes at h + i*step, i < floor((width - N) / step) + 1).  HOST
 * outputs; either may be NULL.  DIC_E_INVAL when the subset does not fit or
 * subset_size or step is below 1. */
dic_status dic_node_grid(int32_t width, int32_t height, int32_t subset_size, int32_t step, int32_t *nx, int32_t *ny);

/*
 * Correlate one deformed image (same size as the reference) from `nseeds`
 * host seeds; results go to `out` (device arrays, [ny][nx]).
 * Per node: inverse-compositional Gauss-Newton on ZNSSD (Eq. (4)) until the
 * increment norm sqrt(dp0^2 + dp1^2 + h^2 sum_{2..5} dpj^2 + h^4 sum_{6..11}
 * dpj^2) < tol, or max_iter.  Seeds: integer ZNCC search over
 * round(u0, v0) + [-R, R]^2, then IC-GN.  Propagation: wave k+1 holds every
 * active, unvisited node with a CONVERGED 4-neighbour in wave k, started from
 * the guess of the neighbour with the largest ZNCC (exact ties: left, right,
 * up, down).  Returns DIC_E_NOSEED if no seed reaches an active node.
 */
dic_status dic_correlate(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds, dic_result *out);

/*
 * Correlate `nframes` deformed images against the same reference in one
 * batched pass: wave k of every frame goes into one launch, or, for 16, 32, 48
 * or 64 frames and for more than 32, into one launch per launch chain (the two
 * halves of the frames on two streams; see dic_stats.launch_chains).
 * seeds: nframes * nseeds host seeds (frame-major); outs: nframes results.
 * 1 <= nframes <= 64 (DIC_E_INVAL otherwise).  Each frame's results equal
 * those of dic_correlate on that frame alone.
 */
dic_status dic_correlate_batch(dic_ctx *c, const dic_image *defs, int32_t nframes, const dic_seed *seeds,
                               int32_t nseeds, dic_result *outs);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * correlation as dic_correlate, bitwise, with no hipMalloc, hipFree or other
 * allocating call.  Per-frame scratch lives in one library-owned device array
 * of dic_noalloc_scratch_bytes() bytes (64 MiB) per device, held until the
 * process ends; the context's own buffers come from dic_create and
 * dic_set_reference, the result arrays from the caller.  At most 64 seeds.
 * A reference whose scratch does not fit (deformed coefficients, parent keys,
 * frontier lists and wave sizes: about 36 bytes per pixel-grid node plus 4 (2
 * with FP16) bytes per padded pixel; a 2048 x 2048 image at step 2 needs
 * 38 MB) is refused with DIC_E_INVAL before any work is queued.
 * Every call on one device shares that device's array and leaves its last
 * contents there (each call clears what it needs): calls that overlap on one
 * device, from any context or stream, race and must be serialised by the
 * caller.
 */
dic_status dic_correlate_noalloc(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds,
                                 dic_result *out);

/* Bytes of the per-device scratch array dic_correlate_noalloc uses. */
int64_t dic_noalloc_scratch_bytes(void);

/* Counters and timings of the last call. */
dic_status dic_get_stats(const dic_ctx *c, dic_stats *out);

/* Release the context and everything it owns. */
dic_status dic_destroy(dic_ctx *c);

/* Message of the last error on this context ("" if none); valid until the next call. */
const char *dic_last_error(const dic_ctx *c);

/* ------------------------------------------------------------------------
 * Multi-window FFT initial guess (Sec. 2.2, Eq. (1); Sec. 4's MAD outlier
 * removal).
 *
 * Rigid displacements from the normalised (phase) cross-correlation of square
 * windows: powers of two from the smallest above max_disp (at most 4096, and
 * no larger than the image) down to the smallest power of two holding the
 * subset (Wf), then one Wf window per node of the reference's grid.  Windows
 * of a level overlap by half; each is compared with the deformed window
 * shifted by its integer guess (the exact bilinear interpolation of the
 * previous level's integer field at its centre, zero on the first level; a
 * shifted window leaving the image keeps its guess); both are tapered by a
 * separable Hann weight before the transform.  After every level a 3x3
 * normalised-median test replaces a window whose u or v differs from its
 * neighbours' median by more than mad_threshold * (MAD + 1 px) with the
 * neighbours' medians.  A level resolves shifts up to half its window, so
 * max_disp should be about twice the largest expected displacement.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t max_disp;      /* estimate of the largest displacement in pixels, >= 1 */
    int32_t subpixel;      /* 1: 3-point Gaussian fit around each node's peak (the MULTIWINDOW mode) */
    double mad_threshold;  /* normalised-median threshold (2 is usual); 0 disables the test */
} dic_mw_params;

/*
 * The multi-window estimate at every node of the current reference's grid
 * against `def` (DEVICE image, same size).  Outputs (caller-allocated DEVICE
 * [ny][nx]): u_out, v_out (integers unless subpixel), valid_out (int8: 1 for
 * active nodes, 0 elsewhere).  levels_out (HOST, 32 entries, may be NULL):
 * the window sizes used, the node level last; *nlevels (may be NULL) their
 * count.  Workspace is kept by the context (two 128 MiB batch buffers and a
 * few bytes per window).  Returns after completion.
 */
dic_status dic_multiwindow(dic_ctx *c, const dic_image *def, const dic_mw_params *prm, float *u_out, float *v_out,
                           int8_t *valid_out, int32_t *levels_out, int32_t *nlevels);

/* Reliability-guided correlation seeded by the multi-window estimate (the
 * paper's default MULTIWINDOW_RG): each seed's (u0, v0) becomes the estimate
 * at the node it snaps to, then dic_correlate runs with those seeds. */
dic_status dic_correlate_mw(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds,
                            const dic_mw_params *prm, dic_result *out);

/* ------------------------------------------------------------------------
 * Sequences with reference updating (Sec. 6: the reference moves through the
 * sequence of deformed images to follow large strains).
 *
 * Frames are correlated in order against the current reference, which starts
 * as the context's.  When the fraction of active nodes that converge, or their
 * mean ZNCC, falls below its threshold (and the previous frame is not already
 * the reference), the previous frame becomes the reference (dic_set_reference
 * on it with the same ROI mask and parameters: the context keeps it after the
 * call) and the frame is correlated again.  Every result is on the original
 * reference's nodes: node X sits at x = X + u_r(X) in the current reference
 * (u_r the reference's accumulated result), the incremental result is
 * interpolated bilinearly at x (terms of non-zero weight only),
 * u = u_r + u_inc(x), the gradients compose as G = G_inc + G_r + G_inc G_r,
 * ZNCC interpolates, iterations and wave index come from the nearest node;
 * status NOT_REACHED where the reference's node did not converge or x leaves
 * the grid, else the first non-converged status of the weighted nodes.
 * Seeds: the given positions; the guess is (u0, v0) for frame 0, zero for the
 * first frame after an update, else the previous frame's incremental result at
 * the seed's node.  Rigid and affine shapes when updating.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t update;        /* 1: update the reference on a quality drop; 0: every frame against the original */
    double min_converged;  /* fraction of active nodes that must converge (e.g. 0.95) */
    double min_zncc;       /* mean ZNCC over converged nodes required (e.g. 0.9) */
} dic_seq_params;

/* frames: nframes DEVICE images (kept valid during the call); roi_mask_dev as
 * for dic_set_reference (used for updated references); outs: nframes
 * caller-allocated results; ref_of_frame (HOST, may be NULL): the frame each
 * result was correlated against (-1: the original reference). */
dic_status dic_correlate_sequence(dic_ctx *c, const dic_image *frames, int32_t nframes, const uint8_t *roi_mask_dev,
                                  const dic_seed *seeds, int32_t nseeds, const dic_seq_params *sp, dic_result *outs,
                                  int32_t *ref_of_frame);

/* ------------------------------------------------------------------------
 * Out-of-core correlation (Sec. 6: images split into chunks that are loaded
 * one at a time, for pairs larger than the device's memory).
 *
 * Both images and every output stay in HOST memory; only one band of the pair
 * is on the device at a time.  The node grid (the one dic_set_reference would
 * build for the whole image) is cut into bands of band_rows node rows.  A
 * band's window holds its subsets' pixel rows plus `halo` rows above and
 * below (the top rounded down to a multiple of the step), with the ROI
 * limited to the band's subsets; the window becomes the context's reference
 * (the context keeps the last band's afterwards) and the deformed window is
 * correlated against it.  Bands are done outward from the band of the first
 * seed: first downward, then upward.  A band's seeds are the given seeds whose
 * nearest node row lies in it and, except for the first band, up to
 * boundary_seeds evenly spaced nodes of its node row next to the finished
 * neighbour whose node across the boundary converged, guessed with that
 * node's displacement.  A second sweep, from the outermost bands back toward
 * the first, correlates again every band that has no converged node, seeded
 * across its other boundary.  Active nodes of a band with no usable seed stay
 * NOT_REACHED.  Propagation restarts in every band, so wave indices count from
 * each band's seeds and a node's starting guess can differ from a single pass
 * over the whole grid: converged values agree with it within the convergence
 * threshold where the halo covers the vertical motion (otherwise warped
 * pixels leave the window and the node is OUT_OF_BOUNDS); the spline
 * prefilter sees the window's edges, whose influence decays by 0.268 per
 * pixel.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t band_rows;      /* node rows per band, >= 1 */
    int32_t halo;           /* extra pixel rows above and below a band, >= 0 (cover |v| plus the spline's reach) */
    int32_t boundary_seeds; /* seeds taken across each band boundary, 1..64 */
} dic_chunk_params;

/* ref_host, def_host: HOST images (pitch_bytes in host memory); roi_host: HOST
 * mask [height][width] or NULL; seeds as for dic_correlate in full-image
 * pixels; out_host: HOST arrays laid out as dic_result for the whole grid.
 * Allocates device windows for the tallest band for the duration of the call.
 * DIC_E_INVAL for bad sizes or parameters; errors of dic_set_reference and
 * dic_correlate pass through (the outputs then hold the bands done so far). */
dic_status dic_correlate_chunked(dic_ctx *c, const dic_image *ref_host, const dic_image *def_host,
                                 const uint8_t *roi_host, const dic_params *prm, const dic_seed *seeds,
                                 int32_t nseeds, const dic_chunk_params *cp, dic_result *out_host);

/* ------------------------------------------------------------------------
 * Strain post-processing (Sec. 2.3, Eq. (6)-(9)).
 *
 * For every node whose window of window x window nodes (centred on it) lies
 * inside the grid and holds only valid displacements (status CONVERGED when a
 * status array is given, finite u and v), u_x and u_y are fitted by linear
 * least squares in the chosen polynomial basis of the local node offsets in
 * pixels (Eq. (8)-(9)); F = I + grad u is taken from the fit's derivatives at
 * the window centre (Eq. (6)), and the chosen strain measure from F.  Every
 * other node gets NaN in every output.  Bases: bilinear [1, x, y, xy] and
 * biquadratic [1, x, y, xy, x^2, y^2, x^2 y, x y^2, x^2 y^2] (the value of the
 * enum is the number of basis terms, the "window elements").
 * ------------------------------------------------------------------------ */
typedef enum { DIC_STRAIN_BILINEAR = 4, DIC_STRAIN_BIQUADRATIC = 9 } dic_strain_basis;

typedef enum {
    DIC_STRAIN_GREEN_LAGRANGE = 0, /* (F^T F - I) / 2 */
    DIC_STRAIN_HENCKY = 1,         /* ln sqrt(F^T F) */
    DIC_STRAIN_EULER_ALMANSI = 2,  /* (I - (F F^T)^-1) / 2 */
    DIC_STRAIN_BIOT_RIGHT = 3,     /* sqrt(F^T F) - I */
    DIC_STRAIN_BIOT_LEFT = 4       /* sqrt(F F^T) - I */
} dic_strain_measure;

typedef struct {
    int32_t window;   /* nodes per side of the smoothing window: odd, 3..15 */
    int32_t basis;    /* dic_strain_basis */
    int32_t measure;  /* dic_strain_measure */
} dic_strain_params;

/*
 * u, v: DEVICE float [ny][nx] displacements on a grid of `step` pixels (the
 * u = p0 and v = p1 planes of a dic_result); status: DEVICE int8 [ny][nx] or
 * NULL.  Outputs (caller-allocated DEVICE float): F_out [4][ny][nx] holding
 * F_xx, F_xy, F_yx, F_yy and eps_out [3][ny][nx] holding eps_xx, eps_xy,
 * eps_yy.  Ordered on the context's stream (no reference needed); returns
 * after completion.  DIC_E_INVAL for a bad window, basis, measure or size.
 */
dic_status dic_strain(dic_ctx *c, const float *u, const float *v, const int8_t *status, int32_t nx, int32_t ny,
                      int32_t step, const dic_strain_params *prm, float *F_out, float *eps_out);

/* Virtual strain gauge of Eq. (7) in pixels: (window - 1) * step + subset_size. */
int32_t dic_vsg(int32_t window, int32_t step, int32_t subset_size);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of correlation requests.
 *
 * A server keeps reference precomputes resident (dic_server_add_reference,
 * one per reference image, region and parameter set) and runs requests (one
 * deformed frame against one resident reference each).  Submitted requests
 * wait in FIFO order; at every dic_server_step call the server admits waiting
 * requests while an active slot is free and their scratch fits the HBM budget,
 * then advances every active request by one frontier wave per launch step:
 * all active requests with the same shape and threads per subset share one
 * launch per step, each at its own wave.  Requests whose propagation has ended
 * are retired (results final, scratch returned to the pool) at the end of the
 * call.  A request's results are the ones dic_correlate gives for it alone.
 * Results arrays are caller-owned DEVICE memory, as for dic_correlate, and
 * must stay allocated until the request is done.
 * ------------------------------------------------------------------------ */
typedef struct dic_server dic_server;

typedef struct {
    int32_t max_active;       /* requests on the device at once, 1..64 */
    double hbm_budget_bytes;  /* device bytes for resident references plus active requests' scratch */
} dic_server_params;

typedef struct {
    int64_t submitted, admitted, completed;
    int32_t active, waiting;
    int64_t steps;            /* launch steps so far */
    double used_bytes;        /* references + active requests */
    double pool_bytes;        /* request scratch kept for reuse */
} dic_server_stats;

dic_status dic_server_create(dic_server **out, int device, void *hip_stream, const dic_server_params *prm);

/* Make a reference resident (same arguments as dic_set_reference); *ref_id
 * names it in later submissions.  Fails with DIC_E_NOMEM, before allocating,
 * when its precompute does not fit the budget next to the resident references
 * and active requests (idle pooled scratch is released first). */
dic_status dic_server_add_reference(dic_server *s, const dic_image *ref, const uint8_t *roi_mask_dev,
                                    const dic_params *prm, int32_t *ref_id);

/* Release a resident reference and its pooled request scratch.  Fails with
 * DIC_E_STATE while a waiting or active request uses it; its id is not
 * reused.  Tickets of finished requests stay pollable. */
dic_status dic_server_remove_reference(dic_server *s, int32_t ref_id);

/* Queue a request: deformed image (DEVICE, same size as the reference),
 * host seeds, caller-allocated DEVICE results.  *ticket identifies it.  The
 * image and result arrays must stay valid until the request is done. */
dic_status dic_server_submit(dic_server *s, int32_t ref_id, const dic_image *def, const dic_seed *seeds,
                             int32_t nseeds, dic_result *out, int64_t *ticket);

/* Admit what fits, run `steps` launch steps (1..256), retire finished
 * requests.  Returns after the device work of the call has completed. */
dic_status dic_server_step(dic_server *s, int32_t steps);

/* *done = 1 once the request's results are final; *status is then DIC_OK or
 * the request's error (DIC_E_NOSEED; DIC_E_NOMEM if its scratch does not fit
 * the budget even beside its own reference alone).  A request that does not
 * fit now waits at the head of the queue.  st
 * (may be NULL) receives the request's counters. */
dic_status dic_server_poll(dic_server *s, int64_t ticket, int32_t *done, int32_t *status, dic_stats *st);

/* Drop the record of a finished request (its ticket becomes unknown); a
 * long-running server calls it once a result has been consumed.  DIC_E_STATE
 * if the request is not done yet. */
dic_status dic_server_forget(dic_server *s, int64_t ticket);

dic_status dic_server_get_stats(const dic_server *s, dic_server_stats *out);
dic_status dic_server_destroy(dic_server *s);
const char *dic_server_last_error(const dic_server *s);

#ifdef __cplusplus
}
#endif

#endif /* DIC_H */
