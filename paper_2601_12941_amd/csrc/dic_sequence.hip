// Multi-frame correlation with reference updating (paper Sec. 6: the
// reference moves through the sequence of deformed images to follow large
// strains, after Pan et al. 2012).
//
// Every frame is correlated against the current reference with dic_correlate;
// when the fraction of active nodes that converge, or their mean ZNCC, falls
// below a threshold, the previous frame becomes the reference
// (dic_set_reference on it, same ROI mask and parameters) and the frame is
// correlated again.  Results are expressed on the original reference's nodes:
// a node X sits at x = X + u_r(X) in the current reference, where u_r is the
// accumulated displacement of that reference; the incremental result is
// interpolated bilinearly at x (k_seq_accumulate), u = u_r + u_inc(x), and the
// displacement gradients compose, G = G_inc + G_r + G_inc G_r.  Seeds: the
// user's positions, guessed from the user's (u0, v0) on the first frame, from
// zero on the first frame after an update, and otherwise from the previous
// frame's incremental result at the seed's node.
#include "dic_context.h"

#include <cmath>

using namespace dicmi;

namespace {

constexpr int kQualBlocks = 256;

// Per-block partial sums of (active, converged, sum ZNCC over converged), then
// one fixed-order sum: the same total on every run.
__global__ __launch_bounds__(256) void k_seq_quality(const int8_t *status, const float *zncc, int64_t n,
                                                     double *part)
{
    __shared__ double sa[256], sc[256], sz[256];
    double a = 0.0, cv = 0.0, z = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const int8_t st = status[i];
        a += st != kNotInRoi ? 1.0 : 0.0;
        if (st == kConverged) {
            cv += 1.0;
            z += static_cast<double>(zncc[i]);
        }
    }
    sa[threadIdx.x] = a;
    sc[threadIdx.x] = cv;
    sz[threadIdx.x] = z;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sc[threadIdx.x] += sc[threadIdx.x + s];
            sz[threadIdx.x] += sz[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = sa[0];
        part[3 * blockIdx.x + 1] = sc[0];
        part[3 * blockIdx.x + 2] = sz[0];
    }
}

__global__ void k_seq_quality_final(const double *part, int nb, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, cv = 0.0, z = 0.0;
    for (int b = 0; b < nb; ++b) {
        a += part[3 * b];
        cv += part[3 * b + 1];
        z += part[3 * b + 2];
    }
    out[0] = a;
    out[1] = cv;
    out[2] = z;
}

struct SeqResult {
    float *p;
    float *zncc;
    int16_t *iters;
    int8_t *status;
    int32_t *wave;
};

// One thread per original node: the incremental result `inc` on the current
// reference's grid, interpolated at the node's position in that reference
// (`ref` = the reference's accumulated result, absent for the original).
__global__ void k_seq_accumulate(SeqResult ref, int has_ref, SeqResult inc, SeqResult out, int np, int nx, int ny,
                                 int h, int step)
{
    const int64_t nn = static_cast<int64_t>(nx) * ny;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const int i = static_cast<int>(c % nx), j = static_cast<int>(c / nx);
    // defaults: not reached
    for (int k = 0; k < np; ++k) out.p[k * nn + c] = 0.0f;
    out.zncc[c] = 0.0f;
    out.iters[c] = 0;
    out.wave[c] = -1;
    out.status[c] = kNotReached;
    double ur = 0.0, vr = 0.0, G[4] = {0.0, 0.0, 0.0, 0.0};
    if (!has_ref) {
        if (inc.status[c] == kNotInRoi) {
            out.status[c] = kNotInRoi;
            return;
        }
    } else {
        const int8_t rs = ref.status[c];
        if (rs != kConverged) {
            out.status[c] = rs == kNotInRoi ? kNotInRoi : kNotReached;
            return;
        }
        ur = ref.p[c];
        vr = ref.p[nn + c];
        if (np >= 6)
            for (int k = 0; k < 4; ++k) G[k] = ref.p[(2 + k) * nn + c];
    }
    const double x = static_cast<double>(h + i * step) + ur, y = static_cast<double>(h + j * step) + vr;
    const double fx = (x - h) / step, fy = (y - h) / step;
    if (!isfinite(fx) || !isfinite(fy)) return;   // not reached (a reference state with no number)
    const double fi0 = floor(fx), fj0 = floor(fy);
    const double ax = fx - fi0, ay = fy - fj0;
    // the cell's far column / row is needed only where it carries weight
    if (fi0 < 0.0 || fj0 < 0.0 || fi0 > nx - 1 || fj0 > ny - 1 || (ax > 0.0 && fi0 + 1 > nx - 1) ||
        (ay > 0.0 && fj0 + 1 > ny - 1))
        return;
    const int i0 = static_cast<int>(fi0), j0 = static_cast<int>(fj0);
    const int64_t q[4] = {static_cast<int64_t>(j0) * nx + i0, static_cast<int64_t>(j0) * nx + i0 + 1,
                          static_cast<int64_t>(j0 + 1) * nx + i0, static_cast<int64_t>(j0 + 1) * nx + i0 + 1};
    const double w[4] = {(1 - ax) * (1 - ay), ax * (1 - ay), (1 - ax) * ay, ax * ay};
    int st = kConverged;
    for (int k = 0; k < 4; ++k)
        if (w[k] > 0.0 && inc.status[q[k]] != kConverged) {
            st = inc.status[q[k]];
            break;
        }
    auto interp = [&](const float *a) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k)
            if (w[k] > 0.0) s += w[k] * static_cast<double>(a[q[k]]);
        return s;
    };
    out.p[c] = static_cast<float>(ur + interp(inc.p));
    out.p[nn + c] = static_cast<float>(vr + interp(inc.p + nn));
    if (np >= 6) {
        const double a00 = interp(inc.p + 2 * nn), a01 = interp(inc.p + 3 * nn);
        const double a10 = interp(inc.p + 4 * nn), a11 = interp(inc.p + 5 * nn);
        // G_inc + G_r + G_inc G_r
        out.p[2 * nn + c] = static_cast<float>(a00 + G[0] + (a00 * G[0] + a01 * G[2]));
        out.p[3 * nn + c] = static_cast<float>(a01 + G[1] + (a00 * G[1] + a01 * G[3]));
        out.p[4 * nn + c] = static_cast<float>(a10 + G[2] + (a10 * G[0] + a11 * G[2]));
        out.p[5 * nn + c] = static_cast<float>(a11 + G[3] + (a10 * G[1] + a11 * G[3]));
    }
    out.zncc[c] = static_cast<float>(interp(inc.zncc));
    const int ri = min(max(static_cast<int>(floor(fx + 0.5)), 0), nx - 1);
    const int rj = min(max(static_cast<int>(floor(fy + 0.5)), 0), ny - 1);
    out.iters[c] = inc.iters[static_cast<int64_t>(rj) * nx + ri];
    out.wave[c] = inc.wave[static_cast<int64_t>(rj) * nx + ri];
    out.status[c] = static_cast<int8_t>(st);
}

SeqResult as_seq(const dic_result &r) { return SeqResult{r.p, r.zncc, r.iters, r.status, r.wave}; }

} // namespace

extern "C" {

dic_status dic_correlate_sequence(dic_ctx *c, const dic_image *frames, int32_t nframes, const uint8_t *roi_mask_dev,
                                  const dic_seed *seeds, int32_t nseeds, const dic_seq_params *sp, dic_result *outs,
                                  int32_t *ref_of_frame)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!c->has_ref) FAIL(DIC_E_STATE, "dic_correlate_sequence before dic_set_reference");
    if (!frames || nframes < 1 || !outs || !seeds || nseeds < 1 || !sp)
        FAIL(DIC_E_INVAL, "NULL frames, results, seeds or sequence params");
    if (sp->update && c->np == DIC_SHAPE_QUADRATIC)
        FAIL(DIC_E_UNSUPPORTED, "reference updating composes rigid and affine shapes only");
    for (int t = 0; t < nframes; ++t) {
        if (frames[t].width != c->W || frames[t].height != c->H)
            FAIL(DIC_E_INVAL, "frame %d is %dx%d, reference is %dx%d", t, frames[t].width, frames[t].height, c->W,
                 c->H);
        if (!outs[t].p || !outs[t].zncc || !outs[t].iters || !outs[t].status || !outs[t].wave)
            FAIL(DIC_E_INVAL, "result %d has a NULL array", t);
    }
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int np = c->np;
    const int64_t nodes = c->nodes;
    // the incremental result of the current frame and of the previous one, and the
    // quality reduction's partial sums (grow-only)
    const size_t inc_bytes = (sizeof(float) * (np + 1) + sizeof(int16_t) + sizeof(int8_t) + sizeof(int32_t)) *
                             static_cast<size_t>(nodes);
    if (!c->seq_buf || c->seq_cap < 2 * inc_bytes) {
        dfree(c->seq_buf);
        HIPCHK(hipMalloc(&c->seq_buf, 2 * inc_bytes + 256));
        c->seq_cap = 2 * inc_bytes;
    }
    if (!c->seq_part) HIPCHK(hipMalloc(&c->seq_part, sizeof(double) * (3 * kQualBlocks + 3)));
    auto carve = [&](char *base) {
        dic_result r;
        r.p = reinterpret_cast<float *>(base);
        r.zncc = r.p + np * nodes;
        r.wave = reinterpret_cast<int32_t *>(r.zncc + nodes);
        r.iters = reinterpret_cast<int16_t *>(r.wave + nodes);
        r.status = reinterpret_cast<int8_t *>(r.iters + nodes);
        return r;
    };
    dic_result inc[2] = {carve(static_cast<char *>(c->seq_buf)),
                         carve(static_cast<char *>(c->seq_buf) + ((inc_bytes + 255) / 256) * 256)};
    const dic_params prm = c->prm;
    const int h = (prm.subset_size - 1) / 2;
    int cur = -1, prev = -1;   // prev: index into inc[] of the previous frame's result against `cur`
    std::vector<dic_seed> sd(nseeds);
    for (int t = 0; t < nframes; ++t) {
        const int slot = t & 1;
        auto run = [&](bool from_prev) -> dic_status {
            for (int q = 0; q < nseeds; ++q) {
                sd[q] = seeds[q];
                if (!(cur == -1 && t == 0)) {
                    sd[q].u0 = 0.0;
                    sd[q].v0 = 0.0;
                }
                if (from_prev && prev >= 0) {
                    const int64_t node = snap_seed(c, seeds[q].x, seeds[q].y);
                    if (node < 0) continue;
                    int8_t st = 0;
                    float uv[2];
                    HIPCHK(hipMemcpy(&st, inc[prev].status + node, 1, hipMemcpyDeviceToHost));
                    HIPCHK(hipMemcpy(&uv[0], inc[prev].p + node, sizeof(float), hipMemcpyDeviceToHost));
                    HIPCHK(hipMemcpy(&uv[1], inc[prev].p + nodes + node, sizeof(float), hipMemcpyDeviceToHost));
                    if (st == kConverged) {
                        sd[q].u0 = uv[0];
                        sd[q].v0 = uv[1];
                    }
                }
            }
            return dic_correlate(c, frames + t, sd.data(), nseeds, &inc[slot]);
        };
        auto quality = [&](double &frac, double &mz) -> dic_status {
            k_seq_quality<<<kQualBlocks, 256, 0, s>>>(inc[slot].status, inc[slot].zncc, nodes, c->seq_part);
            k_seq_quality_final<<<1, 64, 0, s>>>(c->seq_part, kQualBlocks, c->seq_part + 3 * kQualBlocks);
            double q[3];
            HIPCHK(hipMemcpyAsync(q, c->seq_part + 3 * kQualBlocks, sizeof(q), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            frac = q[1] / std::max(1.0, q[0]);
            mz = q[1] > 0.0 ? q[2] / q[1] : 0.0;
            return DIC_OK;
        };
        dic_status st = run(true);
        if (st != DIC_OK) return st;
        double frac = 0.0, mz = 0.0;
        st = quality(frac, mz);
        if (st != DIC_OK) return st;
        if (sp->update && (frac < sp->min_converged || mz < sp->min_zncc) && t >= 1 && cur != t - 1) {
            st = dic_set_reference(c, frames + (t - 1), roi_mask_dev, &prm);
            if (st != DIC_OK) return st;
            cur = t - 1;
            prev = -1;
            st = run(false);
            if (st != DIC_OK) return st;
        }
        const unsigned blocks = static_cast<unsigned>((nodes + 255) / 256);
        k_seq_accumulate<<<blocks, 256, 0, s>>>(cur >= 0 ? as_seq(outs[cur]) : SeqResult{}, cur >= 0 ? 1 : 0,
                                                as_seq(inc[slot]), as_seq(outs[t]), np, c->nx, c->ny, h, prm.step);
        HIPCHK(hipGetLastError());
        if (ref_of_frame) ref_of_frame[t] = cur;
        prev = slot;
    }
    HIPCHK(hipStreamSynchronize(s));
    return DIC_OK;
}

} // extern "C"
