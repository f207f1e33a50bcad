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
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return DIC_E_DEVICE;
        }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_pinned), 64 * sizeof(int32_t)) != hipSuccess) {
        delete c;
        return DIC_E_DEVICE;
    }
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
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->chunk_ev) (void)hipEventDestroy(e);
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
    if (p.shape == DIC_SHAPE_RIGID) FAIL(DIC_E_UNSUPPORTED, "rigid shape function is not built");
    if (p.shape != DIC_SHAPE_AFFINE && p.shape != DIC_SHAPE_QUADRATIC) FAIL(DIC_E_INVAL, "shape %d", p.shape);
    if (p.max_iter < 1 || p.max_iter > 32767) FAIL(DIC_E_INVAL, "max_iter %d", p.max_iter);
    if (!(p.tol > 0.0) || !std::isfinite(p.tol)) FAIL(DIC_E_INVAL, "tol %g", p.tol);
    if (!std::isfinite(p.zncc_min)) FAIL(DIC_E_INVAL, "zncc_min %g", p.zncc_min);
    if (p.seed_radius < 0 || p.seed_radius > 64) FAIL(DIC_E_INVAL, "seed_radius %d", p.seed_radius);
    if (p.guess_mode != 0 && p.guess_mode != 1) FAIL(DIC_E_INVAL, "guess_mode %d", p.guess_mode);
    if (ref->width < p.subset_size || ref->height < p.subset_size)
        FAIL(DIC_E_INVAL, "image %dx%d smaller than subset %d", ref->width, ref->height, p.subset_size);
    int tps = p.threads_per_subset;
    if (tps == 0) tps = p.subset_size <= 23 ? 64 : (p.subset_size <= 37 ? 128 : 256);
    if (!supported_tps(p.subset_size, tps))
        FAIL(DIC_E_INVAL, "threads_per_subset %d unsupported for subset %d", tps, p.subset_size);
    if (p.tile_side != 0 && (p.tile_side < p.subset_size + 5 || p.tile_side > 96))
        FAIL(DIC_E_INVAL, "tile_side %d (0, or %d..96)", p.tile_side, p.subset_size + 5);
    if (tps < 64 && p.shape != DIC_SHAPE_AFFINE)
        FAIL(DIC_E_UNSUPPORTED, "packed subsets (%d threads per subset) are built for the affine shape", tps);
    if (p.shape == DIC_SHAPE_QUADRATIC && tps == 64 && p.subset_size > 21)
        FAIL(DIC_E_UNSUPPORTED, "quadratic shape with 64 threads is built for subsets up to 21");

    HIPCHK(hipSetDevice(c->device));
    HIPCHK(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    free_reference(c);
    c->prm = p;
    c->prm.threads_per_subset = tps;
    c->tps = tps;
    c->np = p.shape;
    c->W = ref->width;
    c->H = ref->height;
    c->nx = (c->W - p.subset_size) / p.step + 1;
    c->ny = (c->H - p.subset_size) / p.step + 1;
    c->nodes = static_cast<int64_t>(c->nx) * c->ny;
    c->ref_pixel = ref->pixel;
    c->cpitch = round_up(c->W + 2 * kPad, 64);
    c->ppitch = round_up(c->W, 64);
    c->tpitch = round_up(c->W, 64);
    hipStream_t s = c->stream;

    HIPCHK(hipMalloc(&c->ref_coef_base, c->coef_elems() * sizeof(float)));
    HIPCHK(hipMalloc(&c->tmp, sizeof(float) * c->tpitch * c->H));
    HIPCHK(hipMalloc(&c->pf, sizeof(float) * c->ppitch * c->H));
    HIPCHK(hipMalloc(&c->pfx, sizeof(float) * c->ppitch * c->H));
    HIPCHK(hipMalloc(&c->pfy, sizeof(float) * c->ppitch * c->H));
    HIPCHK(hipMalloc(&c->cache, sizeof(double) * cache_slots(c->np) * c->nodes));
    HIPCHK(hipMalloc(&c->flag, c->nodes));
    const size_t rowb = c->W * pixel_size(ref->pixel);
    HIPCHK(hipMalloc(&c->ref_raw, rowb * c->H));
    HIPCHK(hipMalloc(&c->d_wave_total, sizeof(int32_t) * (c->nodes + 130)));
    HIPCHK(hipMemcpy2DAsync(c->ref_raw, rowb, ref->data, ref->pitch_bytes, rowb, c->H, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(c->cache, 0, sizeof(double) * cache_slots(c->np) * c->nodes, s));

    RefView R = c->view();
    HIPCHK(hipMalloc(&c->d_view, sizeof(RefView)));
    HIPCHK(hipMemcpyAsync(c->d_view, &R, sizeof(RefView), hipMemcpyHostToDevice, s));
    launch_prefilter(ref->data, ref->pitch_bytes, ref->pixel, c->W, c->H, c->tmp, c->tpitch, const_cast<float *>(R.coef),
                     c->cpitch, false, s);
    launch_ref_pixels(R, c->pf, c->pfx, c->pfy, s);
    launch_active(roi_mask_dev, R, c->flag, s);
    launch_ref_nodes(R, c->np, tps, c->cache, c->flag, s);
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

dic_status dic_correlate_batch(dic_ctx *c, const dic_image *defs, int32_t nframes, const dic_seed *seeds,
                               int32_t nseeds, dic_result *outs)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!c->has_ref) FAIL(DIC_E_STATE, "dic_correlate before dic_set_reference");
    if (nframes < 1 || nframes > kMaxFrames) FAIL(DIC_E_INVAL, "nframes %d (1..%d)", nframes, kMaxFrames);
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

    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    dic_status st = ensure_frames(c, nframes);
    if (st != DIC_OK) return st;

    // seeds: snap to active nodes, de-duplicate per frame, integer search centre
    std::vector<int32_t> seed_nodes(static_cast<size_t>(nframes) * nseeds), centre(2 * nframes * nseeds);
    std::vector<int> nuniq(nframes, 0);
    for (int f = 0; f < nframes; ++f) {
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
    for (int f = 0; f < nframes; ++f) {
        FrameBuf &fb = c->frames[f];
        dfree(fb.seed_p);
        dfree(fb.seed_nodes);
        HIPCHK(hipMalloc(&fb.seed_p, sizeof(double) * 2 * nseeds));
        HIPCHK(hipMalloc(&fb.seed_nodes, sizeof(int32_t) * nseeds));
    }

    const bool half = c->prm.coef_fp16 != 0;
    RefView R = c->view();
    HIPCHK(hipEventRecord(c->ev[0], s));
    c->h_frames.resize(nframes);
    for (int f = 0; f < nframes; ++f) {
        FrameBuf &fb = c->frames[f];
        FrameState &F = c->h_frames[f];
        const size_t esz = half ? sizeof(__half) : sizeof(float);
        F.dcoef = static_cast<char *>(fb.dcoef_base) + (kPad * c->cpitch + kPad) * esz;
        F.dpitch = c->cpitch;
        F.draw = defs[f].data;
        F.draw_pitch = defs[f].pitch_bytes;
        F.dpixel = defs[f].pixel;
        F.p = outs[f].p;
        F.zncc = outs[f].zncc;
        F.iters = outs[f].iters;
        F.status = outs[f].status;
        F.wave = outs[f].wave;
        F.pkey = fb.pkey;
        F.list0 = fb.list0;
        F.list1 = fb.list1;
        F.counts = fb.counts;
        F.seed_p = fb.seed_p;
        F.seed_nodes = fb.seed_nodes;
        F.nseeds = nuniq[f];
        F.stat = fb.stat;
        F.ref = c->d_view;
        F.k_base = 0;
        F.kmax = static_cast<int>(c->nodes + 1);
        launch_prefilter(defs[f].data, defs[f].pitch_bytes, defs[f].pixel, c->W, c->H, c->tmp, c->tpitch,
                         const_cast<void *>(F.dcoef), c->cpitch, half, s);
        launch_init_frame(R, F, c->np, s);
        HIPCHK(hipMemsetAsync(fb.stat, 0, sizeof(unsigned long long) * 4, s));
        HIPCHK(hipMemcpyAsync(fb.seed_nodes, seed_nodes.data() + f * nseeds, sizeof(int32_t) * nseeds,
                              hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipEventRecord(c->ev[1], s));
    HIPCHK(hipMemcpyAsync(c->d_centre, centre.data(), sizeof(int32_t) * 2 * nframes * nseeds, hipMemcpyHostToDevice,
                          s));
    HIPCHK(hipMemcpyAsync(c->d_frames, c->h_frames.data(), sizeof(FrameState) * nframes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(c->d_wave_total, 0, sizeof(int32_t) * (c->nodes + 130), s));
    launch_seed_search(R, c->d_frames, nframes, nseeds, c->prm.seed_radius, c->d_centre, c->d_zbuf, s);
    launch_seed_pick(R, c->d_frames, nframes, nseeds, c->prm.seed_radius, c->d_centre, c->d_zbuf, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev[2], s));

    const int grid = wave_grid_hint(c->np, c->tps, c->device);
    FrameTable table;
    std::memset(&table, 0, sizeof(table));
    for (int f = 0; f < nframes; ++f) table.f[f] = c->h_frames[f];
    table.n = nframes;
    const bool f64 = c->prm.reduce_fp64 != 0;
    int k = 0, chunk = 4, waves = 0, nchunk = 0;
    for (;;) {
        if (static_cast<int>(c->chunk_ev.size()) < 2 * (nchunk + 1)) {
            hipEvent_t a, b;
            HIPCHK(hipEventCreate(&a));
            HIPCHK(hipEventCreate(&b));
            c->chunk_ev.push_back(a);
            c->chunk_ev.push_back(b);
        }
        HIPCHK(hipEventRecord(c->chunk_ev[2 * nchunk], s));
        for (int j = 0; j < chunk && k <= c->nodes; ++j, ++k)
            if (!launch_wave(table, k, c->np, c->prm.subset_size, c->tps, f64, R.ts, grid, s))
                FAIL(DIC_E_UNSUPPORTED, "no kernel for shape %d, %d threads, subset %d", c->np, c->tps,
                     c->prm.subset_size);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(c->chunk_ev[2 * nchunk + 1], s));
        ++nchunk;
        // size of the next wave, summed over the frames
        launch_count_wave(c->d_frames, nframes, k, c->d_wave_total, s);
        HIPCHK(hipMemcpyAsync(c->h_pinned, c->d_wave_total + k, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (c->h_pinned[0] == 0 || k > c->nodes) break;
        chunk = std::min(chunk * 2, 64);
    }
    HIPCHK(hipEventRecord(c->ev[3], s));
    for (int f = 0; f < nframes; ++f) {
        launch_frame_stats(R, c->h_frames[f], s);
        launch_finalize(R, c->h_frames[f], c->np, c->prm.nan_unconverged != 0, s);
    }
    HIPCHK(hipGetLastError());

    // counters: number of waves = first empty wave index (frame 0's counts suffice
    // per frame; over frames, the waves of the longest frame)
    std::vector<int32_t> wt(k + 1, 0);
    for (int f = 0; f < nframes; ++f) {
        std::vector<int32_t> cf(k + 1);
        HIPCHK(hipMemcpyAsync(cf.data(), c->frames[f].counts, sizeof(int32_t) * (k + 1), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int q = 0; q <= k; ++q) wt[q] += cf[q];
    }
    std::vector<unsigned long long> stat(4 * nframes);
    for (int f = 0; f < nframes; ++f)
        HIPCHK(hipMemcpyAsync(stat.data() + 4 * f, c->frames[f].stat, sizeof(unsigned long long) * 4,
                              hipMemcpyDeviceToHost, s));
    double sp[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(sp, c->frames[nframes - 1].seed_p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    waves = 0;
    while (waves <= k && wt[waves] > 0) ++waves;
    dic_stats S{};
    S.nodes = c->nodes;
    S.active = c->active;
    S.threads_per_subset = c->tps;
    S.frames = nframes;
    S.waves = waves;
    for (int f = 0; f < nframes; ++f) {
        S.computed += static_cast<int64_t>(stat[4 * f + 0]);
        S.converged += static_cast<int64_t>(stat[4 * f + 1]);
        S.iterations += static_cast<int64_t>(stat[4 * f + 2]);
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
    for (int q = 0; q < nchunk; ++q) {
        HIPCHK(hipEventElapsedTime(&ms, c->chunk_ev[2 * q], c->chunk_ev[2 * q + 1]));
        S.ms_wave_kernels += ms;
    }
    c->stats = S;
    return DIC_OK;
}

dic_status dic_correlate(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds, dic_result *out)
{
    return dic_correlate_batch(c, def, 1, seeds, nseeds, out);
}

} // extern "C"
