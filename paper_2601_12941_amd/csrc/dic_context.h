// Internal: the library context and the helpers shared by the engine
// (dic_engine.hip) and the serving loop (dic_server.hip).  Not public ABI.
#pragma once

#include "../../include/dic.h"
#include "dic_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace dicmi {

// Launch chains of a batched call: groups of frames whose waves run on streams of
// their own (the frames are independent; only a frame's own waves are ordered).
// Two halves when the frame count splits into two groups of a multiple of 8 (each
// group keeps the frame-to-XCD affinity of the wave kernel) or when one launch
// cannot carry all frames; chain g holds frames [g n / chains, (g + 1) n / chains).
constexpr int kMaxChains = 4;
constexpr int kMaxBatch = 2 * kMaxFrames;   // frames one batched call may carry
inline int launch_chains(int nframes) { return (nframes % 16 == 0 || nframes > kMaxFrames) ? 2 : 1; }

struct FrameBuf {
    void *dcoef_base = nullptr;  // padded deformed coefficients
    uint64_t *pkey = nullptr;
    int32_t *list0 = nullptr, *list1 = nullptr, *counts = nullptr;
    double *seed_p = nullptr;
    int32_t *seed_nodes = nullptr;
    int seed_capacity = 0;       // seeds seed_p / seed_nodes hold
    unsigned long long *stat = nullptr;
};

// Nodes along one image extent: centres h + i*step while the subset fits.
inline int grid_count(int extent, int subset_size, int step) { return (extent - subset_size) / step + 1; }

inline size_t pixel_size(int pixel) { return pixel == DIC_PIX_U8 ? 1 : (pixel == DIC_PIX_U16 ? 2 : 4); }

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Multi-window window schedule (dic_fft.hip): regular sizes, node-level size.
int mw_levels(int max_disp, int N, int W, int H, int *sizes, int *wf);

// Device address of the allocation-free entry point's scratch array on
// `device` (dic_noalloc.hip); nullptr if the lookup fails.
void *noalloc_scratch(int device);
constexpr size_t kNoallocStageBytes = 4096;

// Shared steps of the correlate entry points (dic_engine.hip).
dic_status check_correlate_args(dic_ctx *c, const dic_image *defs, int32_t nframes, const dic_seed *seeds,
                                int32_t nseeds, const dic_result *outs);
// Seeds of every frame snapped to active nodes and de-duplicated, with the
// centres of their integer searches; host arrays of nframes*nseeds and
// 2*nframes*nseeds entries, nuniq[nframes].
dic_status snap_frame_seeds(dic_ctx *c, const dic_seed *seeds, int nframes, int nseeds, int32_t *seed_nodes,
                            int32_t *centre, int *nuniq);
// Host record of one frame over device buffers the caller provides.
void fill_frame(const dic_ctx *c, FrameState &F, const dic_image &def, const dic_result &out, void *dcoef_base,
                uint64_t *pkey, int32_t *list0, int32_t *list1, int32_t *counts, double *seed_p,
                int32_t *seed_nodes, int nseeds, unsigned long long *stat);
// Prefilter, seed search, every wave, finalisation and counters of nframes
// frames whose records hf[] point at allocated buffers; allocates nothing
// (chunk_timing: per-chunk events, created on first use).
dic_status run_frames(dic_ctx *c, const dic_image *defs, int nframes, int nseeds, const FrameState *hf,
                      FrameState *d_frames, const int32_t *h_seed_nodes, const int32_t *h_centre, int32_t *d_centre,
                      double *d_zbuf, bool chunk_timing);

} // namespace dicmi

using namespace dicmi;

struct dic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    bool has_ref = false;
    dic_params prm{};
    int W = 0, H = 0, nx = 0, ny = 0, np = 6, tps = 64;
    bool variant = false;          // rigid shape, NSSD / SSD or LM damping: the general wave kernel
    int64_t nodes = 0, active = 0;
    int ref_pixel = 0;

    float *ref_coef_base = nullptr;
    int64_t cpitch = 0;            // coefficient row pitch (elements)
    float *pa = nullptr;   // interleaved interpolant and gradient [H][ppitch][3]
    int64_t ppitch = 0;
    double *cache = nullptr;
    int8_t *flag = nullptr;
    void *ref_raw = nullptr;
    float *tmp = nullptr;          // prefilter row-pass scratch
    int64_t tpitch = 0;
    std::vector<int8_t> flag_host;

    std::vector<FrameBuf> frames;
    FrameState *d_frames = nullptr;
    std::vector<FrameState> h_frames;
    int32_t *d_centre = nullptr;
    double *d_zbuf = nullptr;
    int zbuf_capacity = 0, centre_capacity = 0;
    int32_t *d_wave_total = nullptr;   // wave sizes, [kMaxChains][nodes + 130]: one row per launch chain
    hipStream_t chain_stream[kMaxChains] = {};   // launch chains 1.. of batched calls (default priority)
    hipEvent_t chain_ev[kMaxChains] = {};        // fork (0) and join (1..) events of the chains
    hipEvent_t count_ev[kMaxChains] = {};        // each chain's next-wave size has reached the host
    RefView *d_view = nullptr;   // device copy of view(), read by the wave kernel
    int32_t *h_pinned = nullptr;
    unsigned long long *h_stats = nullptr;  // pinned: 4 counters per frame, then the last frame's seed shift
    void *noalloc_base = nullptr;           // this device's scratch array (dic_correlate_noalloc)
    int32_t *h_noalloc = nullptr;           // pinned staging of dic_correlate_noalloc (seeds, frame record)
    double *d_strain_w = nullptr;           // least-squares derivative weights of dic_strain
    void *mw_a = nullptr, *mw_b = nullptr;  // dic_multiwindow: batch buffers (complex FP32)
    size_t mw_cap_f2 = 0;
    void *mw_int = nullptr;                 // dic_multiwindow: per-window integer fields, flags, estimates
    int64_t mw_cap_w = 0;
    float *mw_node_u = nullptr;             // dic_correlate_mw: the node estimates
    int64_t mw_node_cap = 0;
    void *seq_buf = nullptr;                // dic_correlate_sequence: two incremental results
    size_t seq_cap = 0;
    double *seq_part = nullptr;             // dic_correlate_sequence: quality partial sums
    hipEvent_t ev[4] = {};
    std::vector<hipEvent_t> chunk_ev;
    dic_stats stats{};

    size_t coef_elems() const { return static_cast<size_t>(cpitch) * (H + 2 * kPad); }
    int window_side() const { return prm.tile_side ? prm.tile_side : tile_side(prm.subset_size); }

    RefView view() const
    {
        RefView R;
        R.coef = ref_coef_base + kPad * cpitch + kPad;
        R.cpitch = cpitch;
        R.pa = pa;
        R.ppitch = ppitch;
        R.cache = cache;
        R.flag = flag;
        R.raw = ref_raw;
        R.pixel = ref_pixel;
        R.W = W;
        R.H = H;
        R.N = prm.subset_size;
        R.step = prm.step;
        R.nx = nx;
        R.ny = ny;
        R.nodes = nodes;
        R.max_iter = prm.max_iter;
        R.tol2 = prm.tol * prm.tol;
        R.zncc_min = static_cast<float>(prm.zncc_min);
        R.guess_copy = prm.guess_mode;
        R.half = prm.coef_fp16 != 0;
        R.ts = window_side();
        R.lp = lds_pitch(prm.subset_size, R.ts);
        R.inv_n = 1.0 / (static_cast<double>(prm.subset_size) * prm.subset_size);
        R.cost = prm.cost;
        R.lm_lambda = prm.lm_lambda;
        return R;
    }
};

#define FAIL(code, ...)                                                                                               \
    do {                                                                                                              \
        char buf_[512];                                                                                               \
        snprintf(buf_, sizeof(buf_), __VA_ARGS__);                                                                    \
        c->err = buf_;                                                                                                \
        return code;                                                                                                  \
    } while (0)

#define HIPCHK(expr)                                                                                                  \
    do {                                                                                                              \
        hipError_t e_ = (expr);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            if (e_ == hipErrorOutOfMemory) FAIL(DIC_E_NOMEM, "%s: %s", #expr, hipGetErrorString(e_));               \
            FAIL(DIC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));                                              \
        }                                                                                                             \
    } while (0)

namespace dicmi {

template <typename T> inline void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

inline void free_reference(dic_ctx *c)
{
    dfree(c->ref_coef_base);
    dfree(c->pa);
    dfree(c->cache);
    dfree(c->flag);
    dfree(c->ref_raw);
    dfree(c->tmp);
    dfree(c->d_wave_total);
    dfree(c->d_view);
    for (auto &f : c->frames) {
        dfree(f.dcoef_base);
        dfree(f.pkey);
        dfree(f.list0);
        dfree(f.list1);
        dfree(f.counts);
        dfree(f.seed_p);
        dfree(f.seed_nodes);
        dfree(f.stat);
    }
    c->frames.clear();
    c->has_ref = false;
}

inline dic_status check_image(dic_ctx *c, const dic_image *im, const char *what)
{
    if (!im) FAIL(DIC_E_INVAL, "%s image is NULL", what);
    if (!im->data) FAIL(DIC_E_INVAL, "%s image data is NULL", what);
    if (im->pixel < DIC_PIX_U8 || im->pixel > DIC_PIX_F32) FAIL(DIC_E_INVAL, "%s pixel type %d", what, im->pixel);
    if (im->width < 1 || im->height < 1) FAIL(DIC_E_INVAL, "%s size %dx%d", what, im->width, im->height);
    if (im->pitch_bytes < static_cast<int64_t>(im->width * pixel_size(im->pixel)))
        FAIL(DIC_E_INVAL, "%s pitch %lld below row size", what, static_cast<long long>(im->pitch_bytes));
    return DIC_OK;
}

// Ensure per-frame scratch for `n` frames.
inline dic_status ensure_frames(dic_ctx *c, int n)
{
    const int np = c->np;
    const bool half = c->prm.coef_fp16 != 0;
    while (static_cast<int>(c->frames.size()) < n) {
        FrameBuf f;
        HIPCHK(hipMalloc(&f.dcoef_base, c->coef_elems() * (half ? sizeof(__half) : sizeof(float))));
        HIPCHK(hipMalloc(&f.pkey, sizeof(uint64_t) * c->nodes));
        HIPCHK(hipMalloc(&f.list0, sizeof(int32_t) * c->nodes));
        HIPCHK(hipMalloc(&f.list1, sizeof(int32_t) * c->nodes));
        HIPCHK(hipMalloc(&f.counts, sizeof(int32_t) * (c->nodes + 2)));
        HIPCHK(hipMalloc(&f.stat, sizeof(unsigned long long) * 4));
        f.seed_p = nullptr;
        f.seed_nodes = nullptr;
        c->frames.push_back(f);
    }
    (void)np;
    if (!c->d_frames) HIPCHK(hipMalloc(&c->d_frames, sizeof(FrameState) * kMaxBatch));
    return DIC_OK;
}

// Nearest active node to (x, y), ties to smaller y then smaller x; -1 if none.
// Searches square rings of grid nodes around the node nearest to (x, y) and
// stops once a ring cannot hold a node closer than the best found.
inline int64_t snap_seed(const dic_ctx *c, double x, double y)
{
    const int h = (c->prm.subset_size - 1) / 2, s = c->prm.step;
    const int nx = c->nx, ny = c->ny;
    if (nx < 1 || ny < 1) return -1;
    auto clampi = [](double v, int hi) { return v < 0.0 ? 0 : (v > hi ? hi : static_cast<int>(std::lround(v))); };
    const int i0 = clampi((x - h) / s, nx - 1), j0 = clampi((y - h) / s, ny - 1);
    int64_t best = -1;
    double bd = 0.0;
    int bj = 0, bi = 0;
    auto consider = [&](int i, int j) {
        const int64_t node = static_cast<int64_t>(j) * nx + i;
        if (c->flag_host[node] < 0) return;
        const double dx = h + static_cast<double>(i) * s - x, dy = h + static_cast<double>(j) * s - y;
        const double d = dx * dx + dy * dy;
        if (best < 0 || d < bd || (d == bd && (j < bj || (j == bj && i < bi)))) {
            best = node;
            bd = d;
            bj = j;
            bi = i;
        }
    };
    // every node of ring r has |i - i0| = r or |j - j0| = r, so it lies at least
    // min(gap_x(r), gap_y(r)) from (x, y)
    auto gap = [&](int r, int k0, int n, double v) {
        double g = -1.0;
        for (int k : {k0 - r, k0 + r}) {
            if (k < 0 || k >= n) continue;
            const double dd = std::fabs(h + static_cast<double>(k) * s - v);
            g = g < 0.0 ? dd : std::min(g, dd);
        }
        return g;
    };
    const int rmax = std::max(nx, ny);
    for (int r = 0; r <= rmax; ++r) {
        if (best >= 0) {
            const double gx = gap(r, i0, nx, x), gy = gap(r, j0, ny, y);
            double lb = gx < 0.0 ? gy : (gy < 0.0 ? gx : std::min(gx, gy));
            if (lb >= 0.0 && lb * lb > bd) break;
        }
        const int ja = std::max(0, j0 - r), jb = std::min(ny - 1, j0 + r);
        const int ia = std::max(0, i0 - r), ib = std::min(nx - 1, i0 + r);
        for (int j = ja; j <= jb; ++j) {
            if (j == j0 - r || j == j0 + r) {
                for (int i = ia; i <= ib; ++i) consider(i, j);
            } else {
                if (i0 - r >= 0) consider(i0 - r, j);
                if (r > 0 && i0 + r < nx) consider(i0 + r, j);
            }
        }
    }
    return best;
}

} // namespace dicmi
