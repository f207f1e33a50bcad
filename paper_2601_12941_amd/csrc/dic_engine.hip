// Host engine and C ABI of the reliability-guided DIC library (include/dic.h).
//
// The context owns every device buffer of the path: the resident reference
// precompute (coefficients, per-pixel intensity and gradient, per-node
// Hessian inverse and sums), and per-frame scratch (deformed coefficients,
// frontier lists, parent keys).  Caller-owned result arrays double as the
// propagation state: a node's p, read by its children in the next wave, is
// the p it reports.
//
// Wave loop: waves are launched back to back on the context's stream; the
// host reads the size of the next wave only once per chunk of waves (the
// chunk doubles up to 64), so host synchronisation is amortised; waves
// launched past the end of propagation find an empty frontier and exit.
#include "dic_context.h"

using namespace dicmi;

extern "C" {

dic_status dic_create(dic_ctx **out, int device, void *hip_stream)
{
    if (!out) return DIC_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return DIC_E_DEVICE;
    if (device < 0 || device >= ndev) return DIC_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return DIC_E_DEVICE;
    dic_ctx *c = new dic_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    auto drop = [](dic_ctx *d) {
        for (auto &e : d->ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : d->count_ev)
            if (e) (void)hipEventDestroy(e);
        delete d;
    };
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            drop(c);
            return DIC_E_DEVICE;
        }
    for (auto &e : c->count_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            drop(c);
            return DIC_E_DEVICE;
        }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_pinned), 64 * sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->h_stats), sizeof(unsigned long long) * (4 * kMaxBatch + 2)) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->h_noalloc), kNoallocStageBytes) != hipSuccess) {
        if (c->h_pinned) (void)hipHostFree(c->h_pinned);
        if (c->h_stats) (void)hipHostFree(c->h_stats);
        drop(c);
        return DIC_E_DEVICE;
    }
    // the allocation-free entry point's scratch array on this device (looked up
    // once per device; dic_correlate_noalloc reports a failed lookup)
    c->noalloc_base = noalloc_scratch(device);
    *out = c;
    return DIC_OK;
}

const char *dic_last_error(const dic_ctx *c) { return c ? c->err.c_str() : "null context"; }

dic_status dic_destroy(dic_ctx *c)
{
    if (!c) return DIC_E_INVAL;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_reference(c);
    dfree(c->d_frames);
    dfree(c->d_centre);
    dfree(c->d_zbuf);
    dfree(c->d_strain_w);
    dfree(c->mw_a);
    dfree(c->mw_b);
    dfree(c->mw_int);
    dfree(c->mw_node_u);
    dfree(c->seq_buf);
    dfree(c->seq_part);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->h_stats) (void)hipHostFree(c->h_stats);
    if (c->h_noalloc) (void)hipHostFree(c->h_noalloc);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->chunk_ev) (void)hipEventDestroy(e);
    for (auto &e : c->count_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->chain_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &q : c->chain_stream)
        if (q) {
            (void)hipStreamSynchronize(q);
            (void)hipStreamDestroy(q);
        }
    delete c;
    return DIC_OK;
}

dic_status dic_grid_shape(const dic_ctx *c, int32_t *nx, int32_t *ny, int32_t *x0, int32_t *y0, int32_t *step)
{
    if (!c) return DIC_E_INVAL;
    if (!c->has_ref) return DIC_E_STATE;
    const int h = (c->prm.subset_size - 1) / 2;
    if (nx) *nx = c->nx;
    if (ny) *ny = c->ny;
    if (x0) *x0 = h;
    if (y0) *y0 = h;
    if (step) *step = c->prm.step;
    return DIC_OK;
}

dic_status dic_reference_arrays(dic_ctx *c, float *coef_out, float *f_out, float *fx_out, float *fy_out)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!c->has_ref) FAIL(DIC_E_STATE, "dic_reference_arrays before dic_set_reference");
    HIPCHK(hipSetDevice(c->device));
    const size_t row = sizeof(float) * c->W;
    if (coef_out)
        HIPCHK(hipMemcpy2DAsync(coef_out, row, c->ref_coef_base + kPad * c->cpitch + kPad, sizeof(float) * c->cpitch,
                                row, c->H, hipMemcpyDeviceToDevice, c->stream));
    float *dst[3] = {f_out, fx_out, fy_out};
    const RefView R = c->view();
    for (int a = 0; a < 3; ++a)
        if (dst[a]) {
            launch_ref_component(R, a, dst[a], c->stream);
            HIPCHK(hipGetLastError());
        }
    HIPCHK(hipStreamSynchronize(c->stream));
    return DIC_OK;
}

dic_status dic_node_grid(int32_t width, int32_t height, int32_t subset_size, int32_t step, int32_t *nx, int32_t *ny)
{
    if (subset_size < 1 || step < 1 || width < subset_size || height < subset_size) return DIC_E_INVAL;
    if (nx) *nx = grid_count(width, subset_size, step);
    if (ny) *ny = grid_count(height, subset_size, step);
    return DIC_OK;
}

dic_status dic_get_stats(const dic_ctx *c, dic_stats *out)
{
    if (!c || !out) return DIC_E_INVAL;
    *out = c->stats;
    return DIC_OK;
}

dic_status dic_set_reference(dic_ctx *c, const dic_image *ref, const uint8_t *roi_mask_dev, const dic_params *prm)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!prm) FAIL(DIC_E_INVAL, "params is NULL");
    dic_status st = check_image(c, ref, "reference");
    if (st != DIC_OK) return st;
    const dic_params p = *prm;
    if (p.subset_size < 5 || p.subset_size > 63 || (p.subset_size & 1) == 0)
        FAIL(DIC_E_INVAL, "subset_size %d (odd, 5..63)", p.subset_size);
    if (p.step < 1) FAIL(DIC_E_INVAL, "step %d", p.step);
    if (p.shape != DIC_SHAPE_RIGID && p.shape != DIC_SHAPE_AFFINE && p.shape != DIC_SHAPE_QUADRATIC)
        FAIL(DIC_E_INVAL, "shape %d", p.shape);
    if (p.cost < DIC_COST_ZNSSD || p.cost > DIC_COST_SSD) FAIL(DIC_E_INVAL, "cost %d", p.cost);
    if (!(p.lm_lambda >= 0.0) || !std::isfinite(p.lm_lambda)) FAIL(DIC_E_INVAL, "lm_lambda %g", p.lm_lambda);
    const bool variant = p.shape == DIC_SHAPE_RIGID || p.cost != DIC_COST_ZNSSD || p.lm_lambda > 0.0;
    if (p.max_iter < 1 || p.max_iter > 32767) FAIL(DIC_E_INVAL, "max_iter %d", p.max_iter);
    if (!(p.tol > 0.0) || !std::isfinite(p.tol)) FAIL(DIC_E_INVAL, "tol %g", p.tol);
    if (!std::isfinite(p.zncc_min)) FAIL(DIC_E_INVAL, "zncc_min %g", p.zncc_min);
    if (p.seed_radius < 0 || p.seed_radius > 64) FAIL(DIC_E_INVAL, "seed_radius %d", p.seed_radius);
    if (p.guess_mode != 0 && p.guess_mode != 1) FAIL(DIC_E_INVAL, "guess_mode %d", p.guess_mode);
    if (ref->width < p.subset_size || ref->height < p.subset_size)
        FAIL(DIC_E_INVAL, "image %dx%d smaller than subset %d", ref->width, ref->height, p.subset_size);
    int tps = p.threads_per_subset;
    if (tps == 0) tps = variant ? 256 : (p.subset_size <= 23 ? 64 : (p.subset_size <= 37 ? 128 : 256));
    if (variant && tps != 256)
        FAIL(DIC_E_INVAL, "threads_per_subset %d: the rigid shape, NSSD, SSD and LM run 256 threads per subset", tps);
    if (!variant && !supported_tps(p.subset_size, tps))
        FAIL(DIC_E_INVAL, "threads_per_subset %d unsupported for subset %d", tps, p.subset_size);
    if (p.tile_side != 0 && (p.tile_side < p.subset_size + 5 || p.tile_side > 96))
        FAIL(DIC_E_INVAL, "tile_side %d (0, or %d..96)", p.tile_side, p.subset_size + 5);
    if (tps < 64 && p.shape != DIC_SHAPE_AFFINE)
        FAIL(DIC_E_UNSUPPORTED, "packed subsets (%d threads per subset) are built for the affine shape", tps);
    if (!variant && p.shape == DIC_SHAPE_QUADRATIC && tps == 64 && p.subset_size > 21)
        FAIL(DIC_E_UNSUPPORTED, "quadratic shape with 64 threads is built for subsets up to 21");
    {
        const int64_t cp = round_up(ref->width + 2 * kPad, 64), pp = round_up(ref->width, 64);
        const int ts = p.tile_side ? p.tile_side : tile_side(p.subset_size);
        if (!buffer_offsets_fit(cp, ts, pp, p.subset_size))
            FAIL(DIC_E_INVAL, "image width %d with a %d-sample window: subset offsets exceed 32 bits", ref->width, ts);
    }

    HIPCHK(hipSetDevice(c->device));
    HIPCHK(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    free_reference(c);
    c->prm = p;
    c->prm.threads_per_subset = tps;
    c->tps = tps;
    c->np = p.shape;
    c->variant = variant;
    c->W = ref->width;
    c->H = ref->height;
    c->nx = grid_count(c->W, p.subset_size, p.step);
    c->ny = grid_count(c->H, p.subset_size, p.step);
    c->nodes = static_cast<int64_t>(c->nx) * c->ny;
    c->ref_pixel = ref->pixel;
    c->cpitch = round_up(c->W + 2 * kPad, 64);
    c->ppitch = round_up(c->W, 64);
    c->tpitch = round_up(c->W, 64);
    hipStream_t s = c->stream;

    HIPCHK(hipMalloc(&c->ref_coef_base, c->coef_elems() * sizeof(float)));
    HIPCHK(hipMalloc(&c->tmp, sizeof(float) * c->tpitch * c->H));
    HIPCHK(hipMalloc(&c->pa, sizeof(float) * 3 * c->ppitch * c->H));
    // the general kernel of the variants reduces the reference side per subset: no per-node cache
    if (!variant) HIPCHK(hipMalloc(&c->cache, sizeof(double) * cache_slots(c->np) * c->nodes));
    HIPCHK(hipMalloc(&c->flag, c->nodes));
    const size_t rowb = c->W * pixel_size(ref->pixel);
    HIPCHK(hipMalloc(&c->ref_raw, rowb * c->H));
    HIPCHK(hipMalloc(&c->d_wave_total, sizeof(int32_t) * kMaxChains * (c->nodes + 130)));
    HIPCHK(hipMemcpy2DAsync(c->ref_raw, rowb, ref->data, ref->pitch_bytes, rowb, c->H, hipMemcpyDeviceToDevice, s));
    if (!variant) HIPCHK(hipMemsetAsync(c->cache, 0, sizeof(double) * cache_slots(c->np) * c->nodes, s));

    RefView R = c->view();
    HIPCHK(hipMalloc(&c->d_view, sizeof(RefView)));
    HIPCHK(hipMemcpyAsync(c->d_view, &R, sizeof(RefView), hipMemcpyHostToDevice, s));
    launch_prefilter(ref->data, ref->pitch_bytes, ref->pixel, c->W, c->H, c->tmp, c->tpitch, const_cast<float *>(R.coef),
                     c->cpitch, false, s);
    launch_ref_pixels(R, c->pa, s);
    launch_active(roi_mask_dev, R, c->flag, s);
    if (!variant && !launch_ref_nodes(R, c->np, tps, c->cache, c->flag, s)) {
        HIPCHK(hipStreamSynchronize(s));
        free_reference(c);
        FAIL(DIC_E_UNSUPPORTED, "no reference-precompute kernel for shape %d, %d threads, subset %d", c->np, tps,
             p.subset_size);
    }
    HIPCHK(hipGetLastError());
    c->flag_host.resize(c->nodes);
    HIPCHK(hipMemcpyAsync(c->flag_host.data(), c->flag, c->nodes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    c->active = 0;
    for (int64_t i = 0; i < c->nodes; ++i) c->active += c->flag_host[i] >= 0;
    c->has_ref = true;
    c->stats = dic_stats{};
    c->stats.nodes = c->nodes;
    c->stats.active = c->active;
    c->stats.threads_per_subset = tps;
    return DIC_OK;
}

} // extern "C"

namespace dicmi {

dic_status check_correlate_args(dic_ctx *c, const dic_image *defs, int32_t nframes, const dic_seed *seeds,
                                int32_t nseeds, const dic_result *outs)
{
    if (!c->has_ref) FAIL(DIC_E_STATE, "dic_correlate before dic_set_reference");
    if (nframes < 1 || nframes > kMaxBatch) FAIL(DIC_E_INVAL, "nframes %d (1..%d)", nframes, kMaxBatch);
    if (!defs || !outs) FAIL(DIC_E_INVAL, "NULL images or results");
    if (nseeds < 1 || !seeds) FAIL(DIC_E_INVAL, "no seeds");
    for (int f = 0; f < nframes; ++f) {
        dic_status st = check_image(c, defs + f, "deformed");
        if (st != DIC_OK) return st;
        if (defs[f].width != c->W || defs[f].height != c->H)
            FAIL(DIC_E_INVAL, "deformed image %d is %dx%d, reference is %dx%d", f, defs[f].width, defs[f].height, c->W,
                 c->H);
        if (!outs[f].p || !outs[f].zncc || !outs[f].iters || !outs[f].status || !outs[f].wave)
            FAIL(DIC_E_INVAL, "result %d has a NULL array", f);
    }
    for (int q = 0; q < nframes * nseeds; ++q)
        if (!std::isfinite(seeds[q].x) || !std::isfinite(seeds[q].y) || !std::isfinite(seeds[q].u0) ||
            !std::isfinite(seeds[q].v0))
            FAIL(DIC_E_INVAL, "seed %d is not finite", q);
    return DIC_OK;
}

dic_status snap_frame_seeds(dic_ctx *c, const dic_seed *seeds, int nframes, int nseeds, int32_t *seed_nodes,
                            int32_t *centre, int *nuniq)
{
    for (int f = 0; f < nframes; ++f) {
        nuniq[f] = 0;
        for (int q = 0; q < nseeds; ++q) {
            const dic_seed &sd = seeds[f * nseeds + q];
            const int64_t node = snap_seed(c, sd.x, sd.y);
            if (node < 0) continue;
            bool dup = false;
            for (int r = 0; r < nuniq[f]; ++r) dup = dup || seed_nodes[f * nseeds + r] == node;
            if (dup) continue;
            const int u = nuniq[f]++;
            seed_nodes[f * nseeds + u] = static_cast<int32_t>(node);
            centre[2 * (f * nseeds + u)] = static_cast<int32_t>(std::lround(sd.u0));
            centre[2 * (f * nseeds + u) + 1] = static_cast<int32_t>(std::lround(sd.v0));
        }
        if (nuniq[f] == 0) FAIL(DIC_E_NOSEED, "frame %d: no seed lies on an active node", f);
    }
    return DIC_OK;
}

void fill_frame(const dic_ctx *c, FrameState &F, const dic_image &def, const dic_result &out, void *dcoef_base,
                uint64_t *pkey, int32_t *list0, int32_t *list1, int32_t *counts, double *seed_p,
                int32_t *seed_nodes, int nseeds, unsigned long long *stat)
{
    const size_t esz = c->prm.coef_fp16 ? sizeof(__half) : sizeof(float);
    F.dcoef = static_cast<char *>(dcoef_base) + (kPad * c->cpitch + kPad) * esz;
    F.dpitch = c->cpitch;
    F.draw = def.data;
    F.draw_pitch = def.pitch_bytes;
    F.dpixel = def.pixel;
    F.p = out.p;
    F.zncc = out.zncc;
    F.iters = out.iters;
    F.status = out.status;
    F.wave = out.wave;
    F.pkey = pkey;
    F.list0 = list0;
    F.list1 = list1;
    F.counts = counts;
    F.seed_p = seed_p;
    F.seed_nodes = seed_nodes;
    F.nseeds = nseeds;
    F.stat = stat;
    F.ref = c->d_view;
    F.k_base = 0;
    F.kmax = static_cast<int>(c->nodes + 1);
}

dic_status run_frames(dic_ctx *c, const dic_image *defs, int nframes, int nseeds, const FrameState *hf,
                      FrameState *d_frames, const int32_t *h_seed_nodes, const int32_t *h_centre, int32_t *d_centre,
                      double *d_zbuf, bool chunk_timing)
{
    hipStream_t s = c->stream;
    const bool half = c->prm.coef_fp16 != 0;
    RefView R = c->view();
    HIPCHK(hipEventRecord(c->ev[0], s));
    for (int f = 0; f < nframes; ++f) {
        const FrameState &F = hf[f];
        launch_prefilter(defs[f].data, defs[f].pitch_bytes, defs[f].pixel, c->W, c->H, c->tmp, c->tpitch,
                         const_cast<void *>(F.dcoef), c->cpitch, half, s);
        launch_init_frame(R, F, c->np, s);
        launch_zero32(F.stat, 8, s);
        HIPCHK(hipMemcpyAsync(F.seed_nodes, h_seed_nodes + f * nseeds, sizeof(int32_t) * nseeds,
                              hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipEventRecord(c->ev[1], s));
    HIPCHK(hipMemcpyAsync(d_centre, h_centre, sizeof(int32_t) * 2 * nframes * nseeds, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_frames, hf, sizeof(FrameState) * nframes, hipMemcpyHostToDevice, s));
    launch_zero32(c->d_wave_total, launch_chains(nframes) * (c->nodes + 130), s);
    launch_seed_search(R, d_frames, nframes, nseeds, c->prm.seed_radius, d_centre, d_zbuf, s);
    launch_seed_pick(R, d_frames, nframes, nseeds, c->prm.seed_radius, d_centre, d_zbuf, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev[2], s));

    // Launch chains: the frames are independent, so a batch is split into groups
    // whose waves run on streams of their own.  Wave k + 1 of a group waits only
    // for wave k of that group, and the last workgroups of one group's launch share
    // the GPU with the other groups' launches instead of leaving it idle.
    const int nchain = launch_chains(nframes);
    const int grid = wave_grid_hint(c->np, c->variant ? 256 : c->tps, c->device, nchain);
    int off[kMaxChains + 1];
    for (int g = 0; g <= nchain; ++g) off[g] = g * nframes / nchain;
    for (int g = 1; g < nchain; ++g)
        if (!c->chain_stream[g]) HIPCHK(hipStreamCreateWithFlags(&c->chain_stream[g], hipStreamNonBlocking));
    for (int g = 0; g < nchain && nchain > 1; ++g)
        if (!c->chain_ev[g]) HIPCHK(hipEventCreateWithFlags(&c->chain_ev[g], hipEventDisableTiming));
    hipStream_t cs[kMaxChains];
    for (int g = 0; g < kMaxChains; ++g) cs[g] = g == 0 ? s : c->chain_stream[g];
    FrameTable table[kMaxChains];
    std::memset(table, 0, sizeof(table));
    for (int g = 0; g < nchain; ++g) {
        for (int f = off[g]; f < off[g + 1]; ++f) table[g].f[f - off[g]] = hf[f];
        table[g].n = off[g + 1] - off[g];
    }
    if (nchain > 1) {
        // the other chains start after the frames' set-up and seeds on the first stream
        HIPCHK(hipEventRecord(c->chain_ev[0], s));
        for (int g = 1; g < nchain; ++g) HIPCHK(hipStreamWaitEvent(cs[g], c->chain_ev[0], 0));
    }
    const int64_t tstride = c->nodes + 130;   // wave sizes of chain g at d_wave_total + g * tstride
    const bool f64 = c->prm.reduce_fp64 != 0;
    int k = 0, chunk = 4, nchunk = 0;
    bool live[kMaxChains];
    for (int g = 0; g < kMaxChains; ++g) live[g] = g < nchain;
    auto join = [&]() -> dic_status {
        // the first stream waits for the other chains' work so far
        for (int g = 1; g < nchain; ++g) {
            HIPCHK(hipEventRecord(c->chain_ev[g], cs[g]));
            HIPCHK(hipStreamWaitEvent(s, c->chain_ev[g], 0));
        }
        return DIC_OK;
    };
    // Waves go in chunks of 4, 8, ... 64; after a chunk the host reads the size of
    // every chain's next wave to decide whether to go on.  The first kAhead waves of
    // the next chunk are launched before that read, so the GPU runs them while the
    // host waits; a chain whose next wave is empty gets at most kAhead launches that
    // find no subset and return at once.
    constexpr int kAhead = 2;
    bool launched = true;
    auto launch_range = [&](int g, int k0, int k1) {
        for (int kk = k0; kk < k1 && launched; ++kk)
            launched = c->variant ? launch_wave_var(table[g], kk, c->np, grid, cs[g])
                                  : launch_wave(table[g], kk, c->np, c->prm.subset_size, c->tps, f64, R.ts,
                                                R.ts * R.lp, grid, cs[g]);
    };
    auto chunk_open = [&]() -> dic_status {
        if (chunk_timing) {
            if (static_cast<int>(c->chunk_ev.size()) < 2 * (nchunk + 1)) {
                hipEvent_t a, b;
                HIPCHK(hipEventCreate(&a));
                HIPCHK(hipEventCreate(&b));
                c->chunk_ev.push_back(a);
                c->chunk_ev.push_back(b);
            }
            HIPCHK(hipEventRecord(c->chunk_ev[2 * nchunk], s));
        }
        return DIC_OK;
    };
    // size of wave kk of every live chain, summed over its frames, on its way to the
    // host; then the chunk's end
    auto chunk_close = [&](int kk, bool count) -> dic_status {
        if (!launched) {
            // no kernel for these parameters: let the chains' work so far finish on
            // the call's stream before reporting it
            const dic_status js = join();
            if (js != DIC_OK) return js;
            FAIL(DIC_E_UNSUPPORTED, "no kernel for shape %d, %d threads, subset %d", c->np, c->tps,
                 c->prm.subset_size);
        }
        HIPCHK(hipGetLastError());
        for (int g = 0; g < nchain && count; ++g) {
            if (!live[g]) continue;
            launch_count_wave(d_frames + off[g], off[g + 1] - off[g], kk, c->d_wave_total + g * tstride, cs[g]);
            HIPCHK(hipMemcpyAsync(c->h_pinned + g, c->d_wave_total + g * tstride + kk, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, cs[g]));
            HIPCHK(hipEventRecord(c->count_ev[g], cs[g]));
        }
        if (chunk_timing) {
            const dic_status js = join();
            if (js != DIC_OK) return js;
            HIPCHK(hipEventRecord(c->chunk_ev[2 * nchunk + 1], s));
        }
        ++nchunk;
        return DIC_OK;
    };
    dic_status st = chunk_open();
    if (st != DIC_OK) return st;
    k = static_cast<int>(std::min<int64_t>(chunk, c->nodes + 1));
    for (int g = 0; g < nchain; ++g) launch_range(g, 0, k);
    st = chunk_close(k, true);
    if (st != DIC_OK) return st;
    for (;;) {
        const int ahead = static_cast<int>(std::min<int64_t>(k + kAhead, c->nodes + 1));
        st = chunk_open();
        if (st != DIC_OK) return st;
        for (int g = 0; g < nchain; ++g)
            if (live[g]) launch_range(g, k, ahead);
        bool any = false;
        for (int g = 0; g < nchain; ++g) {
            if (!live[g]) continue;
            HIPCHK(hipEventSynchronize(c->count_ev[g]));
            live[g] = c->h_pinned[g] != 0 && k <= c->nodes;
            any = any || live[g];
        }
        if (!any) {
            // every chain is done: the look-ahead launches found nothing
            k = std::max(k, ahead);
            st = chunk_close(k, false);
            if (st != DIC_OK) return st;
            break;
        }
        chunk = std::min(chunk * 2, 64);
        const int kend = static_cast<int>(std::min<int64_t>(k + chunk, c->nodes + 1));
        for (int g = 0; g < nchain; ++g)
            if (live[g]) launch_range(g, ahead, kend);
        k = std::max(kend, ahead);
        st = chunk_close(k, true);
        if (st != DIC_OK) return st;
    }
    {
        const dic_status js = join();
        if (js != DIC_OK) return js;
    }
    HIPCHK(hipEventRecord(c->ev[3], s));
    for (int f = 0; f < nframes; ++f) {
        launch_frame_stats(R, hf[f], s);
        launch_finalize(R, hf[f], c->np, c->prm.nan_unconverged != 0, s);
    }
    HIPCHK(hipGetLastError());

    // counters: per frame computed / converged / iterations / waves (largest wave
    // index + 1); the call's wave count is the longest frame's
    unsigned long long *hs = c->h_stats;
    for (int f = 0; f < nframes; ++f)
        HIPCHK(hipMemcpyAsync(hs + 4 * f, hf[f].stat, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost, s));
    double *sp = reinterpret_cast<double *>(hs + 4 * kMaxBatch);
    HIPCHK(hipMemcpyAsync(sp, hf[nframes - 1].seed_p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dic_stats S{};
    S.nodes = c->nodes;
    S.active = c->active;
    S.threads_per_subset = c->tps;
    S.frames = nframes;
    for (int f = 0; f < nframes; ++f) {
        S.computed += static_cast<int64_t>(hs[4 * f + 0]);
        S.converged += static_cast<int64_t>(hs[4 * f + 1]);
        S.iterations += static_cast<int64_t>(hs[4 * f + 2]);
        S.waves = std::max(S.waves, static_cast<int32_t>(hs[4 * f + 3]));
    }
    S.seed_du = static_cast<int32_t>(sp[0]);
    S.seed_dv = static_cast<int32_t>(sp[1]);
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
    S.ms_total = ms;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    S.ms_icgn = ms;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    S.ms_prefilter = ms;
    S.wave_launches = k;
    S.launch_chains = nchain;
    if (chunk_timing) {
        for (int q = 0; q < nchunk; ++q) {
            HIPCHK(hipEventElapsedTime(&ms, c->chunk_ev[2 * q], c->chunk_ev[2 * q + 1]));
            S.ms_wave_kernels += ms;
        }
    } else {
        S.ms_wave_kernels = S.ms_icgn;
    }
    c->stats = S;
    return DIC_OK;
}

} // namespace dicmi

extern "C" {

dic_status dic_correlate_batch(dic_ctx *c, const dic_image *defs, int32_t nframes, const dic_seed *seeds,
                               int32_t nseeds, dic_result *outs)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    dic_status st = check_correlate_args(c, defs, nframes, seeds, nseeds, outs);
    if (st != DIC_OK) return st;
    HIPCHK(hipSetDevice(c->device));
    st = ensure_frames(c, nframes);
    if (st != DIC_OK) return st;

    // seeds: snap to active nodes, de-duplicate per frame, integer search centre
    std::vector<int32_t> seed_nodes(static_cast<size_t>(nframes) * nseeds), centre(2 * nframes * nseeds);
    std::vector<int> nuniq(nframes, 0);
    st = snap_frame_seeds(c, seeds, nframes, nseeds, seed_nodes.data(), centre.data(), nuniq.data());
    if (st != DIC_OK) return st;
    const int side = 2 * c->prm.seed_radius + 1;
    const int need_z = nframes * nseeds * side * side;
    if (need_z > c->zbuf_capacity) {
        dfree(c->d_zbuf);
        HIPCHK(hipMalloc(&c->d_zbuf, sizeof(double) * need_z));
        c->zbuf_capacity = need_z;
    }
    if (2 * nframes * nseeds > c->centre_capacity) {
        dfree(c->d_centre);
        HIPCHK(hipMalloc(&c->d_centre, sizeof(int32_t) * 2 * nframes * nseeds));
        c->centre_capacity = 2 * nframes * nseeds;
    }
    c->h_frames.resize(nframes);
    for (int f = 0; f < nframes; ++f) {
        // seed buffers only grow: repeated calls with the same seed count allocate nothing
        FrameBuf &fb = c->frames[f];
        if (nseeds > fb.seed_capacity) {
            dfree(fb.seed_p);
            dfree(fb.seed_nodes);
            HIPCHK(hipMalloc(&fb.seed_p, sizeof(double) * 2 * nseeds));
            HIPCHK(hipMalloc(&fb.seed_nodes, sizeof(int32_t) * nseeds));
            fb.seed_capacity = nseeds;
        }
        fill_frame(c, c->h_frames[f], defs[f], outs[f], fb.dcoef_base, fb.pkey, fb.list0, fb.list1, fb.counts,
                   fb.seed_p, fb.seed_nodes, nuniq[f], fb.stat);
    }
    return run_frames(c, defs, nframes, nseeds, c->h_frames.data(), c->d_frames, seed_nodes.data(), centre.data(),
                      c->d_centre, c->d_zbuf, true);
}

dic_status dic_correlate(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds, dic_result *out)
{
    return dic_correlate_batch(c, def, 1, seeds, nseeds, out);
}

} // extern "C"
