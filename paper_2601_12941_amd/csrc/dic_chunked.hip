// Out-of-core correlation of a pair held in host memory (paper Sec. 6: images
// partitioned into chunks loaded one at a time, so that a pair larger than the
// device's memory can be correlated).
//
// The node grid is split into bands of `band_rows` node rows.  A band's pixel
// rows, extended by `halo` rows of the deformed image's expected vertical
// motion on both sides (the window's top aligned to the grid step, so its node
// grid is the full grid's), are copied to the device for both images with the
// ROI restricted to the band's own subsets; the window becomes the context's
// reference and the deformed window is correlated against it.  Bands run
// outward from the one holding the first seed.  A band's seeds are the given
// seeds whose nearest node row lies in it and, for every band but the first,
// up to `boundary_seeds` evenly spaced nodes of its node row next to the band
// already done, each guessed from the converged node across the boundary.  A
// second sweep back toward the first band retries every band left without a
// converged node from its other neighbour (a band behind a gap in the ROI,
// reachable only from a seed further out).  A band with no usable seed keeps
// its active nodes NOT_REACHED.  Each band's results go to the caller's host
// arrays.  Within a band the propagation is the library's;
// across bands it restarts from the boundary seeds, so a node's guess may come
// from another neighbour than in one pass over the whole grid (the converged
// values agree within the convergence threshold).
#include "dic_context.h"

#include <cmath>

using namespace dicmi;

extern "C" {

dic_status dic_correlate_chunked(dic_ctx *c, const dic_image *ref_host, const dic_image *def_host,
                                 const uint8_t *roi_host, const dic_params *prm, const dic_seed *seeds,
                                 int32_t nseeds, const dic_chunk_params *cp, dic_result *out_host)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!ref_host || !def_host || !prm || !seeds || nseeds < 1 || !cp || !out_host)
        FAIL(DIC_E_INVAL, "NULL argument");
    if (!ref_host->data || !def_host->data) FAIL(DIC_E_INVAL, "NULL image data");
    if (ref_host->width != def_host->width || ref_host->height != def_host->height)
        FAIL(DIC_E_INVAL, "deformed image is %dx%d, reference is %dx%d", def_host->width, def_host->height,
             ref_host->width, ref_host->height);
    if (ref_host->pixel != def_host->pixel || ref_host->pixel < DIC_PIX_U8 || ref_host->pixel > DIC_PIX_F32)
        FAIL(DIC_E_INVAL, "pixel types %d / %d", ref_host->pixel, def_host->pixel);
    if (cp->band_rows < 1 || cp->halo < 0 || cp->boundary_seeds < 1 || cp->boundary_seeds > 64)
        FAIL(DIC_E_INVAL, "band_rows %d, halo %d, boundary_seeds %d", cp->band_rows, cp->halo, cp->boundary_seeds);
    const int W = ref_host->width, H = ref_host->height, N = prm->subset_size, s = prm->step;
    if (N < 5 || (N & 1) == 0 || s < 1 || W < N || H < N) FAIL(DIC_E_INVAL, "subset %d, step %d", N, s);
    const int np = prm->shape, h = (N - 1) / 2;
    const int nx = grid_count(W, N, s), ny = grid_count(H, N, s);
    const int64_t nn = static_cast<int64_t>(nx) * ny;
    const size_t px = pixel_size(ref_host->pixel), rowb = static_cast<size_t>(W) * px;
    if (ref_host->pitch_bytes < static_cast<int64_t>(rowb) || def_host->pitch_bytes < static_cast<int64_t>(rowb))
        FAIL(DIC_E_INVAL, "pitch below width * pixel size");
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = c->stream;

    // every node starts outside the ROI (rows no band reaches keep it)
    for (int k = 0; k < np; ++k)
        for (int64_t i = 0; i < nn; ++i) out_host->p[k * nn + i] = 0.0f;
    for (int64_t i = 0; i < nn; ++i) {
        out_host->zncc[i] = 0.0f;
        out_host->iters[i] = 0;
        out_host->status[i] = DIC_NODE_NOT_IN_ROI;
        out_host->wave[i] = -1;
    }
    const int nbands = (ny + cp->band_rows - 1) / cp->band_rows;
    // the node row nearest to a seed, and the band of the first seed
    auto seed_row = [&](const dic_seed &sd) {
        const double r = (sd.y - h) / s;
        return r <= 0.0 ? 0 : (r >= ny - 1 ? ny - 1 : static_cast<int>(std::lround(r)));
    };
    const int b0 = seed_row(seeds[0]) / cp->band_rows;

    // device windows, sized for the tallest band (grow-only within the call)
    const int max_rows = std::min(H, (cp->band_rows - 1) * s + N + 2 * cp->halo + s);
    void *d_ref = nullptr, *d_def = nullptr;
    uint8_t *d_roi = nullptr;
    float *d_p = nullptr, *d_z = nullptr;
    int16_t *d_it = nullptr;
    int8_t *d_st = nullptr;
    int32_t *d_wv = nullptr;
    const int64_t max_nodes = static_cast<int64_t>(nx) * grid_count(max_rows, N, s);
    auto release = [&]() {
        dfree(d_ref);
        dfree(d_def);
        dfree(d_roi);
        dfree(d_p);
        dfree(d_z);
        dfree(d_it);
        dfree(d_st);
        dfree(d_wv);
    };
    auto dev_err = [&](hipError_t e) -> dic_status {
        c->err = std::string("device: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? DIC_E_NOMEM : DIC_E_DEVICE;
    };
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&d_ref, rowb * max_rows)) != hipSuccess || (e = hipMalloc(&d_def, rowb * max_rows)) ||
        (e = hipMalloc(&d_roi, static_cast<size_t>(W) * max_rows)) ||
        (e = hipMalloc(&d_p, sizeof(float) * np * max_nodes)) || (e = hipMalloc(&d_z, sizeof(float) * max_nodes)) ||
        (e = hipMalloc(&d_it, sizeof(int16_t) * max_nodes)) || (e = hipMalloc(&d_st, max_nodes)) ||
        (e = hipMalloc(&d_wv, sizeof(int32_t) * max_nodes))) {
        release();
        return dev_err(e);
    }
    std::vector<uint8_t> roi_win(static_cast<size_t>(W) * max_rows);
    std::vector<float> p_win(static_cast<size_t>(np) * max_nodes), z_win(max_nodes);
    std::vector<int16_t> it_win(max_nodes);
    std::vector<int8_t> st_win(max_nodes);
    std::vector<int32_t> wv_win(max_nodes);

    // side: 0 = given seeds only, +1 = also across the boundary above, -1 = below
    auto run_band = [&](int b, int side) -> dic_status {
        const int j0 = b * cp->band_rows, j1 = std::min(ny, j0 + cp->band_rows);
        const int y_top = j0 * s, y_bot = (j1 - 1) * s + N - 1;
        int ya = std::max(0, y_top - cp->halo);
        ya = (ya / s) * s;                                   // the window's nodes are the full grid's
        const int yb = std::min(H - 1, y_bot + cp->halo);
        const int rows = yb - ya + 1;
        // ROI of the window: the caller's, limited to the band's pixel rows
        for (int y = 0; y < rows; ++y) {
            const int gy = ya + y;
            const bool in_band = gy >= y_top && gy <= y_bot;
            for (int x = 0; x < W; ++x)
                roi_win[static_cast<size_t>(y) * W + x] =
                    in_band && (!roi_host || roi_host[static_cast<int64_t>(gy) * W + x]) ? 1 : 0;
        }
        if ((e = hipMemcpy2DAsync(d_ref, rowb, static_cast<const char *>(ref_host->data) + ref_host->pitch_bytes * ya,
                                  ref_host->pitch_bytes, rowb, rows, hipMemcpyHostToDevice, st)) ||
            (e = hipMemcpy2DAsync(d_def, rowb, static_cast<const char *>(def_host->data) + def_host->pitch_bytes * ya,
                                  def_host->pitch_bytes, rowb, rows, hipMemcpyHostToDevice, st)) ||
            (e = hipMemcpyAsync(d_roi, roi_win.data(), static_cast<size_t>(W) * rows, hipMemcpyHostToDevice, st)))
            return dev_err(e);
        dic_image ri{W, rows, static_cast<int64_t>(rowb), ref_host->pixel, d_ref};
        dic_image di{W, rows, static_cast<int64_t>(rowb), def_host->pixel, d_def};
        dic_status rc = dic_set_reference(c, &ri, d_roi, prm);
        if (rc != DIC_OK) return rc;
        const int wny = c->ny, jw0 = ya / s;                 // window node row k is full row jw0 + k
        for (int j = j0; j < j1; ++j)                        // active nodes stay NOT_REACHED without a seed
            for (int i = 0; i < nx; ++i)
                if (c->flag_host[static_cast<int64_t>(j - jw0) * nx + i] >= 0)
                    out_host->status[static_cast<int64_t>(j) * nx + i] = DIC_NODE_NOT_REACHED;
        std::vector<dic_seed> sd;
        for (int q = 0; q < nseeds; ++q) {
            const int jq = seed_row(seeds[q]);
            if (jq < j0 || jq >= j1) continue;
            dic_seed x = seeds[q];
            x.y -= ya;
            sd.push_back(x);
        }
        if (side != 0) {
            // the node row next to the finished neighbour, guessed across the boundary
            const int jr = side > 0 ? j0 : j1 - 1, jn = side > 0 ? j0 - 1 : j1;
            std::vector<int> conv;
            for (int i = 0; i < nx; ++i)
                if (out_host->status[static_cast<int64_t>(jn) * nx + i] == DIC_NODE_CONVERGED) conv.push_back(i);
            const int64_t nc = static_cast<int64_t>(conv.size());
            const int take = static_cast<int>(std::min<int64_t>(cp->boundary_seeds, nc));
            for (int q = 0; q < take; ++q) {
                const int i = conv[(q * nc) / take + nc / (2 * take)];
                const int64_t m = static_cast<int64_t>(jn) * nx + i;
                sd.push_back(dic_seed{static_cast<double>(h + i * s), static_cast<double>(h + jr * s - ya),
                                      out_host->p[m], out_host->p[nn + m]});
            }
        }
        if (sd.empty()) return DIC_OK;
        dic_result r{d_p, d_z, d_it, d_st, d_wv};
        rc = dic_correlate(c, &di, sd.data(), static_cast<int32_t>(sd.size()), &r);
        if (rc == DIC_E_NOSEED) return DIC_OK;               // no seed on an active node of the band
        if (rc != DIC_OK) return rc;
        const int64_t wn = static_cast<int64_t>(nx) * wny;
        if ((e = hipMemcpyAsync(p_win.data(), d_p, sizeof(float) * np * wn, hipMemcpyDeviceToHost, st)) ||
            (e = hipMemcpyAsync(z_win.data(), d_z, sizeof(float) * wn, hipMemcpyDeviceToHost, st)) ||
            (e = hipMemcpyAsync(it_win.data(), d_it, sizeof(int16_t) * wn, hipMemcpyDeviceToHost, st)) ||
            (e = hipMemcpyAsync(st_win.data(), d_st, wn, hipMemcpyDeviceToHost, st)) ||
            (e = hipMemcpyAsync(wv_win.data(), d_wv, sizeof(int32_t) * wn, hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st)))
            return dev_err(e);
        for (int j = j0; j < j1; ++j) {
            const int k = j - jw0;
            if (k < 0 || k >= wny) continue;
            for (int i = 0; i < nx; ++i) {
                const int64_t g = static_cast<int64_t>(j) * nx + i, w = static_cast<int64_t>(k) * nx + i;
                for (int a = 0; a < np; ++a) out_host->p[a * nn + g] = p_win[a * wn + w];
                out_host->zncc[g] = z_win[w];
                out_host->iters[g] = it_win[w];
                out_host->status[g] = st_win[w];
                out_host->wave[g] = wv_win[w];
            }
        }
        return DIC_OK;
    };
    auto any_converged = [&](int b) {
        const int64_t lo = static_cast<int64_t>(b) * cp->band_rows * nx;
        const int64_t hi = std::min<int64_t>(nn, lo + static_cast<int64_t>(cp->band_rows) * nx);
        for (int64_t g = lo; g < hi; ++g)
            if (out_host->status[g] == DIC_NODE_CONVERGED) return true;
        return false;
    };
    // first sweep outward from the first seed's band; second sweep back toward it
    // for bands left without a converged node, seeded across their other boundary
    dic_status rc = run_band(b0, 0);
    for (int b = b0 + 1; rc == DIC_OK && b < nbands; ++b) rc = run_band(b, +1);
    for (int b = b0 - 1; rc == DIC_OK && b >= 0; --b) rc = run_band(b, -1);
    for (int b = nbands - 2; rc == DIC_OK && b > b0; --b)
        if (!any_converged(b)) rc = run_band(b, -1);
    for (int b = 1; rc == DIC_OK && b < b0; ++b)
        if (!any_converged(b)) rc = run_band(b, +1);
    release();
    return rc;
}

} // extern "C"
