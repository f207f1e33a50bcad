// Multi-window FFT initial guess (paper Sec. 2.2, Eq. (1); Sec. 4's MAD outlier
// removal at every window size): rigid displacements from the phase
// correlation of square windows, from windows larger than the expected
// displacement down to one window per node of the subset grid.
//
// Per level, every window pair goes through one pipeline on the GPU:
//   load      z = w f + i w g (the two Hann-tapered real windows packed into one
//             complex array, so one complex transform yields both spectra);
//   fft2      radix-2 Stockham transforms in LDS (FP32), rows then columns;
//   cross     F conj(G) / (|F| |G|) with F, G split from Z by its Hermitian
//             symmetry;
//   ifft2     the same passes inverse;
//   peak      argmax of the real map per window, the integer displacement
//             shift - q, and on the node level the 3-point Gaussian sub-pixel fit;
//   mad       the 3x3 normalised-median test on the level's integer field;
//   guess     the next level's integer guesses by exact bilinear interpolation.
// Windows of up to 64 samples (the node level and the finest regular levels)
// run load to peak in one kernel with the windows resident in LDS, so their
// only memory traffic is the pixels and the estimates.  Larger windows go
// through batch buffers in HBM: load, rows, transpose, rows, cross, the same
// inverse, and a two-step peak search (parts of each map, then per window).
// Readings (window schedule, grids, taper, tie rules, MAD constants) follow the
// FP64 reference implementation of the same procedure; the integer steps are
// exact, so they agree bit for bit, and only the FFT's FP32 rounding can move a
// peak when two map values nearly tie.
#include "dic_context.h"

#include <climits>
#include <cmath>

using namespace dicmi;

namespace {

constexpr int kFftThreads = 256;
constexpr int kMaxLevels = 32;
constexpr int64_t kBatchElems = int64_t(1) << 24;   // complex values per batch buffer (128 MiB)
constexpr int kMaxWindow = 4096;   // largest window: two rows of it fill 64 KiB of LDS
constexpr int kMaxFusedWindow = 64; // windows up to this side run the whole pipeline in LDS
constexpr int kMaxTableWindow = 2048; // row transforms up to this length read twiddles from an LDS table

// Geometry of one level: windows of side W centred at (ox + i S, oy + j S).
struct Level {
    int W, S, ox, oy, nx, ny;
    bool nodes;   // the node level: top-left corners clamped into the image
};

__device__ __forceinline__ float pixel_at(const void *base, int64_t pitch_bytes, int pixel, int x, int y)
{
    const char *row = static_cast<const char *>(base) + static_cast<int64_t>(y) * pitch_bytes;
    if (pixel == 0) return static_cast<float>(reinterpret_cast<const uint8_t *>(row)[x]);
    if (pixel == 1) return static_cast<float>(reinterpret_cast<const uint16_t *>(row)[x]);
    return reinterpret_cast<const float *>(row)[x];
}

__device__ __forceinline__ void window_origin(const Level &L, int w, int imgW, int imgH, int &rx, int &ry)
{
    const int i = w % L.nx, j = w / L.nx;
    rx = L.ox + i * L.S - L.W / 2;
    ry = L.oy + j * L.S - L.W / 2;
    if (L.nodes) {
        rx = min(max(rx, 0), imgW - L.W);
        ry = min(max(ry, 0), imgH - L.W);
    }
}

// z = w f + i w g for windows [w0, w0 + count) of the level; skip[w] = 1 where the
// shifted deformed window would leave the image (or the node is not active).
__global__ void k_mw_load(Level L, int w0, int count, const void *ref, int64_t rpitch, int rpix, const void *def,
                          int64_t dpitch, int dpix, int imgW, int imgH, const int32_t *gu, const int32_t *gv,
                          const int8_t *active, float2 *z, uint8_t *skip)
{
    const int64_t WW = static_cast<int64_t>(L.W) * L.W;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= WW * count) return;
    const int wl = static_cast<int>(e / WW), w = w0 + wl;
    const int q = static_cast<int>(e - static_cast<int64_t>(wl) * WW);
    const int y = q / L.W, x = q - (q / L.W) * L.W;
    int rx, ry;
    window_origin(L, w, imgW, imgH, rx, ry);
    const int gx = rx + gu[w], gy = ry + gv[w];
    const bool out = gx < 0 || gy < 0 || gx > imgW - L.W || gy > imgH - L.W || (active && active[w] < 0);
    if (q == 0) skip[w] = out ? 1 : 0;
    float2 v = make_float2(0.0f, 0.0f);
    if (!out) {
        const float sx = sinpif(static_cast<float>(x) / L.W), sy = sinpif(static_cast<float>(y) / L.W);
        const float t = (sx * sx) * (sy * sy);
        v.x = t * pixel_at(ref, rpitch, rpix, rx + x, ry + y);
        v.y = t * pixel_at(def, dpitch, dpix, gx + x, gy + y);
    }
    z[e] = v;
}

// Twiddle table of a length-W transform: tw[m] = (sin, cos) of sgn pi 2m / W for
// m < W / 2, the values sincospif gives for sgn pi k / Ns at m = k W / (2 Ns) (the
// arguments are the same dyadic fractions, so the table changes no bit).
__device__ __forceinline__ void twiddles(float2 *tw, int W, float sgn)
{
    for (int m = threadIdx.x; m < W / 2; m += blockDim.x) {
        float sn, cs;
        sincospif(sgn * static_cast<float>(2 * m) / static_cast<float>(W), &sn, &cs);
        tw[m] = make_float2(sn, cs);
    }
}

// One radix-2 Stockham transform of length W per row, in LDS (FP32): a
// workgroup takes max(1, 1024 / W) consecutive rows.  INV: exp(+i ...), unscaled.
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows(float2 *data, int W, int64_t nrows)
{
    extern __shared__ float2 lds[];
    const int R = W >= 1024 ? 1 : 1024 / W;
    const int tot = R * W, half = W / 2;
    float2 *x = lds, *y = lds + tot, *tw = lds + 2 * tot;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
    const int rows = static_cast<int>(min<int64_t>(R, nrows - row0));
    float2 *g = data + row0 * W;
    const bool table = W <= kMaxTableWindow;   // the largest windows evaluate their twiddles
    const float sgn = INV ? 1.0f : -1.0f;
    for (int e = threadIdx.x; e < rows * W; e += kFftThreads) x[e] = g[e];
    if (table) twiddles(tw, W, sgn);
    __syncthreads();
    for (int Ns = 1; Ns < W; Ns <<= 1) {
        const int tstep = half / Ns;
        for (int b = threadIdx.x; b < rows * half; b += kFftThreads) {
            const int r = b / half, j = b - (b / half) * half;
            const int base = r * W, k = j & (Ns - 1);
            const float2 a0 = x[base + j], a1 = x[base + j + half];
            float s, c;
            if (table) {
                s = tw[k * tstep].x;
                c = tw[k * tstep].y;
            } else {
                sincospif(sgn * static_cast<float>(k) / static_cast<float>(Ns), &s, &c);
            }
            const float2 t = make_float2(a1.x * c - a1.y * s, a1.x * s + a1.y * c);
            const int d = base + ((j - k) << 1) + k;
            y[d] = make_float2(a0.x + t.x, a0.y + t.y);
            y[d + Ns] = make_float2(a0.x - t.x, a0.y - t.y);
        }
        __syncthreads();
        float2 *tmp = x;
        x = y;
        y = tmp;
    }
    for (int e = threadIdx.x; e < rows * W; e += kFftThreads) g[e] = x[e];
}

// Transpose every W x W matrix of the batch (tiles of up to 32 x 32 through LDS;
// one workgroup per tile, the tiles of all matrices along one grid axis).
__global__ void k_transpose(const float2 *in, float2 *out, int W)
{
    __shared__ float2 tile[32][33];
    const int T = W < 32 ? W : 32;
    const int tw = W / T;                       // tiles per matrix side
    const int64_t tile_id = blockIdx.x;
    const int64_t mat = tile_id / (static_cast<int64_t>(tw) * tw);
    const int tin = static_cast<int>(tile_id - mat * tw * tw);
    const int64_t base = mat * W * W;
    const int bx = (tin % tw) * T, by = (tin / tw) * T;
    const int tx = threadIdx.x, ty = threadIdx.y;
    if (tx < T && ty < T) tile[ty][tx] = in[base + static_cast<int64_t>(by + ty) * W + bx + tx];
    __syncthreads();
    if (tx < T && ty < T) out[base + static_cast<int64_t>(bx + ty) * W + by + tx] = tile[tx][ty];
}

// Normalised cross-power spectrum of Eq. (1) from the packed spectrum Z = F + i G.
__global__ void k_mw_cross(const float2 *Z, float2 *Rs, int W, int64_t total)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t WW = static_cast<int64_t>(W) * W;
    const int64_t m = e / WW;
    const int q = static_cast<int>(e - m * WW);
    const int a = q / W, b = q - (q / W) * W;
    const int na = (W - a) & (W - 1), nb = (W - b) & (W - 1);
    const float2 z = Z[e], zm = Z[m * WW + static_cast<int64_t>(na) * W + nb];
    // F = (Z(k) + conj Z(-k)) / 2,  G = (Z(k) - conj Z(-k)) / (2i)
    const float2 F = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
    const float2 G = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
    const float cr = F.x * G.x + F.y * G.y, ci = F.y * G.x - F.x * G.y;   // F conj(G)
    const float mag = hypotf(F.x, F.y) * hypotf(G.x, G.y);
    Rs[e] = mag > 0.0f ? make_float2(cr / mag, ci / mag) : make_float2(0.0f, 0.0f);
}

// the total order of the peak search: larger value, then smaller |q|^2, qy, qx
__device__ __forceinline__ bool peak_better(float v, int qx, int qy, float bv, int bx, int by)
{
    if (v != bv) return v > bv;
    const int d2 = qx * qx + qy * qy, b2 = bx * bx + by * by;
    return d2 < b2 || (d2 == b2 && (qy < by || (qy == by && qx < bx)));
}

__device__ __forceinline__ float gauss3(float a, float b, float c)
{
    float e;
    if (a > 0.0f && b > 0.0f && c > 0.0f) {
        const float la = logf(a), lb = logf(b), lc = logf(c);
        const float den = 2.0f * (la - 2.0f * lb + lc);
        e = den != 0.0f ? (la - lc) / den : 0.0f;
    } else {
        const float den = 2.0f * (a - 2.0f * b + c);
        e = den != 0.0f ? (a - c) / den : 0.0f;
    }
    return fabsf(e) <= 0.5f ? e : 0.0f;
}

// Peak search of the large windows in two steps.  First every map is cut into
// B = W^2 / kPeakChunk parts and one workgroup finds the best element of each
// part (value, map index) under the total order below; then one workgroup per
// window picks the best of its B parts and writes the estimate.
constexpr int kPeakChunk = 16384;

__device__ __forceinline__ int signed_q(int i, int W) { return i < W / 2 ? i : i - W; }

// the order on map indices: larger value, then smaller |q|^2, qy, qx; an index
// holding NaN never wins (a map with no number keeps the window's guess)
__device__ __forceinline__ bool index_better(float v, int e, float bv, int be, int W)
{
    if (e < 0 || !(v == v)) return false;
    if (be < 0) return true;
    return peak_better(v, signed_q(e % W, W), signed_q(e / W, W), bv, signed_q(be % W, W), signed_q(be / W, W));
}

__device__ __forceinline__ void block_best(float &bv, int &be, int W)
{
    __shared__ float sv[kFftThreads];
    __shared__ int se[kFftThreads];
    const int t = threadIdx.x;
    sv[t] = bv;
    se[t] = be;
    __syncthreads();
    for (int st = kFftThreads / 2; st > 0; st >>= 1) {
        if (t < st && index_better(sv[t + st], se[t + st], sv[t], se[t], W)) {
            sv[t] = sv[t + st];
            se[t] = se[t + st];
        }
        __syncthreads();
    }
    bv = sv[0];
    be = se[0];
}

// part results as (value, index bits) pairs in `part` (cnt * B entries)
__global__ __launch_bounds__(kFftThreads) void k_mw_peak_part(const float2 *r, int W, int B, float2 *part)
{
    const int wl = blockIdx.x / B, pi = blockIdx.x - (blockIdx.x / B) * B;
    const int64_t WW = static_cast<int64_t>(W) * W;
    const int chunk = static_cast<int>(WW / B);
    const float2 *m = r + static_cast<int64_t>(wl) * WW;
    float bv = -INFINITY;
    int be = -1;
    for (int e = pi * chunk + threadIdx.x; e < (pi + 1) * chunk; e += kFftThreads)
        if (index_better(m[e].x, e, bv, be, W)) {
            bv = m[e].x;
            be = e;
        }
    block_best(bv, be, W);
    if (threadIdx.x == 0) part[blockIdx.x] = make_float2(bv, __int_as_float(be));
}

// integer estimate shift - q into (iu, iv); with `sub`, the Gaussian fit into (fu, fv)
__global__ __launch_bounds__(kFftThreads) void k_mw_peak(const float2 *r, const float2 *part, int B, int W, int w0,
                                                          const int32_t *gu, const int32_t *gv, const uint8_t *skip,
                                                          int32_t *iu, int32_t *iv, float *fu, float *fv, int sub)
{
    const int w = w0 + blockIdx.x;
    float bv = -INFINITY;
    int be = -1;
    if (!skip[w]) {
        for (int i = threadIdx.x; i < B; i += kFftThreads) {
            const float2 pv = part[static_cast<int64_t>(blockIdx.x) * B + i];
            if (index_better(pv.x, __float_as_int(pv.y), bv, be, W)) {
                bv = pv.x;
                be = __float_as_int(pv.y);
            }
        }
        block_best(bv, be, W);
    }
    if (threadIdx.x == 0 && be < 0) {       // skipped, or no number in the map: keep the guess
        iu[w] = gu[w];
        iv[w] = gv[w];
        if (fu) {
            fu[w] = static_cast<float>(gu[w]);
            fv[w] = static_cast<float>(gv[w]);
        }
    } else if (threadIdx.x == 0) {
        const float2 *m = r + static_cast<int64_t>(blockIdx.x) * W * W;
        const int px = be % W, py = be / W;
        const int qx = signed_q(px, W), qy = signed_q(py, W);
        iu[w] = gu[w] - qx;
        iv[w] = gv[w] - qy;
        if (fu) {
            float ex = 0.0f, ey = 0.0f;
            if (sub) {
                const float b = m[py * W + px].x;
                ex = gauss3(m[py * W + ((px + W - 1) & (W - 1))].x, b, m[py * W + ((px + 1) & (W - 1))].x);
                ey = gauss3(m[((py + W - 1) & (W - 1)) * W + px].x, b, m[((py + 1) & (W - 1)) * W + px].x);
            }
            fu[w] = static_cast<float>(gu[w] - qx) - ex;
            fv[w] = static_cast<float>(gv[w] - qy) - ey;
        }
    }
}

// One radix-2 Stockham stage over `lines` transforms of length W held in LDS:
// element e of line l sits at base(l) + e * es; lines are rows (es = 1) or
// columns (es = the row pitch) of K windows of W rows each.
template <int W>
__device__ __forceinline__ void lds_stage(const float2 *x, float2 *y, int lines, int pitch, bool cols, int Ns,
                                          const float2 *tw)
{
    constexpr int half = W / 2;
    const int es = cols ? pitch : 1, tstep = half / Ns;
    for (int b = threadIdx.x; b < lines * half; b += kFftThreads) {
        const int l = b / half, j = b - (b / half) * half;
        const int win = l / W, r = l - (l / W) * W;
        const int base = win * W * pitch + (cols ? r : r * pitch);
        const int k = j & (Ns - 1);
        const float2 a0 = x[base + j * es], a1 = x[base + (j + half) * es];
        const float sn = tw[k * tstep].x, cs = tw[k * tstep].y;
        const float2 t = make_float2(a1.x * cs - a1.y * sn, a1.x * sn + a1.y * cs);
        const int d = ((j - k) << 1) + k;
        y[base + d * es] = make_float2(a0.x + t.x, a0.y + t.y);
        y[base + (d + Ns) * es] = make_float2(a0.x - t.x, a0.y - t.y);
    }
}

// 2-D transform of K windows in LDS (rows, then columns); returns the buffer
// holding the result (x or y).
template <int W>
__device__ __forceinline__ float2 *lds_fft2(float2 *x, float2 *y, int K, int pitch, const float2 *tw)
{
    for (int pass = 0; pass < 2; ++pass)
        for (int Ns = 1; Ns < W; Ns <<= 1) {
            lds_stage<W>(x, y, K * W, pitch, pass == 1, Ns, tw);
            __syncthreads();
            float2 *t = x;
            x = y;
            y = t;
        }
    return x;
}

// The whole per-window pipeline of the small levels (W <= 64) in LDS, K =
// max(1, 1024 / W^2) windows per workgroup: load and taper, forward transform,
// normalised cross-power, inverse transform, peak and sub-pixel fit.  The
// arithmetic is that of the batched pipeline (same butterflies, twiddles,
// cross-power, tie order and fit); only the order of the two 1-D passes of the
// 2-D transforms differs (rows then columns in place, instead of rows,
// transpose, rows).  HBM traffic: the two windows' pixels and the outputs.
template <int W>
__global__ __launch_bounds__(kFftThreads) void k_mw_fused(Level L, int count, const void *ref, int64_t rpitch,
                                                           int rpix, const void *def, int64_t dpitch, int dpix,
                                                           int imgW, int imgH, const int32_t *gu, const int32_t *gv,
                                                           const int8_t *active, int32_t *iu, int32_t *iv, float *fu,
                                                           float *fv, int sub)
{
    constexpr int K = W * W >= 1024 ? 1 : 1024 / (W * W);
    constexpr int P = W + 1;                     // row pitch: column passes avoid bank conflicts
    constexpr int kSz = K * W * P;
    __shared__ float2 buf[2 * kSz];
    __shared__ float2 twf[W / 2], twi[W / 2];
    __shared__ float sv[kFftThreads];
    __shared__ int sq[kFftThreads];
    __shared__ uint8_t skipw[K];
    const int w0 = blockIdx.x * K;
    const int nk = min(K, count - w0);
    float2 *x = buf, *y = buf + kSz;
    twiddles(twf, W, -1.0f);
    twiddles(twi, W, 1.0f);
    // load: z = w f + i w g
    for (int e = threadIdx.x; e < K * W * W; e += kFftThreads) {
        const int k = e / (W * W), q = e - k * (W * W);
        const int yy = q / W, xx = q - (q / W) * W;
        float2 v = make_float2(0.0f, 0.0f);
        bool out = true;
        if (k < nk) {
            const int w = w0 + k;
            int rx, ry;
            window_origin(L, w, imgW, imgH, rx, ry);
            const int gx = rx + gu[w], gy = ry + gv[w];
            out = gx < 0 || gy < 0 || gx > imgW - W || gy > imgH - W || (active && active[w] < 0);
            if (!out) {
                const float sx = sinpif(static_cast<float>(xx) / W), sy = sinpif(static_cast<float>(yy) / W);
                const float t = (sx * sx) * (sy * sy);
                v.x = t * pixel_at(ref, rpitch, rpix, rx + xx, ry + yy);
                v.y = t * pixel_at(def, dpitch, dpix, gx + xx, gy + yy);
            }
        }
        if (q == 0) skipw[k] = out ? 1 : 0;
        x[k * W * P + yy * P + xx] = v;
    }
    __syncthreads();
    float2 *z = lds_fft2<W>(x, y, K, P, twf);
    float2 *r = z == buf ? buf + kSz : buf;
    // normalised cross-power of Eq. (1) from the packed spectrum
    for (int e = threadIdx.x; e < K * W * W; e += kFftThreads) {
        const int k = e / (W * W), q = e - k * (W * W);
        const int a = q / W, b = q - (q / W) * W;
        const int na = (W - a) & (W - 1), nb = (W - b) & (W - 1);
        const float2 zz = z[k * W * P + a * P + b], zm = z[k * W * P + na * P + nb];
        const float2 F = make_float2(0.5f * (zz.x + zm.x), 0.5f * (zz.y - zm.y));
        const float2 G = make_float2(0.5f * (zz.y + zm.y), -0.5f * (zz.x - zm.x));
        const float cr = F.x * G.x + F.y * G.y, ci = F.y * G.x - F.x * G.y;
        const float mag = hypotf(F.x, F.y) * hypotf(G.x, G.y);
        r[k * W * P + a * P + b] = mag > 0.0f ? make_float2(cr / mag, ci / mag) : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
    const float2 *m = lds_fft2<W>(r, z, K, P, twi);
    // peak per window: the K windows' elements are spread over the threads in
    // groups of kFftThreads / K consecutive threads
    constexpr int G = kFftThreads / K;
    const int k = threadIdx.x / G, tl = threadIdx.x - k * G;
    float bv = -INFINITY;
    int bx = INT_MAX / 4, by = INT_MAX / 4;
    for (int q = tl; q < W * W; q += G) {
        const int yy = q / W, xx = q - (q / W) * W;
        const int qx = xx < W / 2 ? xx : xx - W, qy = yy < W / 2 ? yy : yy - W;
        const float v = m[k * W * P + yy * P + xx].x;
        if (peak_better(v, qx, qy, bv, bx, by)) {
            bv = v;
            bx = qx;
            by = qy;
        }
    }
    sv[threadIdx.x] = bv;
    sq[threadIdx.x] = ((by + W) & (W - 1)) * W + ((bx + W) & (W - 1));
    __syncthreads();
    for (int st = G / 2; st > 0; st >>= 1) {
        if (tl < st) {
            const int o = threadIdx.x + st;
            const int oq = sq[o], cq = sq[threadIdx.x];
            const int ox = oq % W, oy = oq / W, cx = cq % W, cy = cq / W;
            if (peak_better(sv[o], ox < W / 2 ? ox : ox - W, oy < W / 2 ? oy : oy - W, sv[threadIdx.x],
                            cx < W / 2 ? cx : cx - W, cy < W / 2 ? cy : cy - W)) {
                sv[threadIdx.x] = sv[o];
                sq[threadIdx.x] = oq;
            }
        }
        __syncthreads();
    }
    if (tl == 0 && k < nk) {
        const int w = w0 + k;
        if (skipw[k] || sv[threadIdx.x] == -INFINITY) {    // skipped, or no number in the map
            iu[w] = gu[w];
            iv[w] = gv[w];
            if (fu) {
                fu[w] = static_cast<float>(gu[w]);
                fv[w] = static_cast<float>(gv[w]);
            }
        } else {
            const int px = sq[threadIdx.x] % W, py = sq[threadIdx.x] / W;
            const int qx = px < W / 2 ? px : px - W, qy = py < W / 2 ? py : py - W;
            iu[w] = gu[w] - qx;
            iv[w] = gv[w] - qy;
            if (fu) {
                float ex = 0.0f, ey = 0.0f;
                if (sub) {
                    const float2 *mk = m + k * W * P;
                    const float b = mk[py * P + px].x;
                    ex = gauss3(mk[py * P + ((px + W - 1) & (W - 1))].x, b, mk[py * P + ((px + 1) & (W - 1))].x);
                    ey = gauss3(mk[((py + W - 1) & (W - 1)) * P + px].x, b, mk[((py + 1) & (W - 1)) * P + px].x);
                }
                fu[w] = static_cast<float>(gu[w] - qx) - ex;
                fv[w] = static_cast<float>(gv[w] - qy) - ey;
            }
        }
    }
}

__device__ __forceinline__ float median_small(float *a, int n)
{
    for (int i = 1; i < n; ++i) {
        const float v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
    return (n & 1) ? a[n / 2] : 0.5f * (a[n / 2 - 1] + a[n / 2]);
}

__device__ __forceinline__ int round_half_away(float v)
{
    return v >= 0.0f ? static_cast<int>(floorf(v + 0.5f)) : -static_cast<int>(floorf(-v + 0.5f));
}

// 3x3 normalised-median test on an integer grid field (Jacobi: every point
// against the unfiltered neighbours).  Every value involved is a multiple of
// 1/4, exact in FP32.  rep[i] = 1 where the point took the neighbours' medians.
__global__ void k_mw_mad(const int32_t *u, const int32_t *v, const int8_t *active, int nx, int ny, float thr,
                         int32_t *ou, int32_t *ov, uint8_t *rep)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= static_cast<int64_t>(nx) * ny) return;
    const int i = static_cast<int>(c % nx), j = static_cast<int>(c / nx);
    int32_t ru = u[c], rv = v[c];
    uint8_t rp = 0;
    if (!active || active[c] >= 0) {
        float nu[8], nv[8];
        int m = 0;
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                const int ii = i + di, jj = j + dj;
                if ((di == 0 && dj == 0) || ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
                const int64_t q = static_cast<int64_t>(jj) * nx + ii;
                if (active && active[q] < 0) continue;
                nu[m] = static_cast<float>(u[q]);
                nv[m] = static_cast<float>(v[q]);
                ++m;
            }
        if (m >= 3) {
            const float mu = median_small(nu, m), mv = median_small(nv, m);
            float du[8], dv[8];
            for (int k = 0; k < m; ++k) {
                du[k] = fabsf(nu[k] - mu);
                dv[k] = fabsf(nv[k] - mv);
            }
            const float madu = median_small(du, m), madv = median_small(dv, m);
            if (fabsf(static_cast<float>(u[c]) - mu) > thr * (madu + 1.0f) ||
                fabsf(static_cast<float>(v[c]) - mv) > thr * (madv + 1.0f)) {
                ru = round_half_away(mu);
                rv = round_half_away(mv);
                rp = 1;
            }
        }
    }
    ou[c] = ru;
    ov[c] = rv;
    if (rep) rep[c] = rp;
}

__device__ __forceinline__ int64_t round_div(int64_t num, int64_t den)
{
    return num >= 0 ? (2 * num + den) / (2 * den) : -((-2 * num + den) / (2 * den));
}

// Integer guesses of a level's windows from the previous level's field: the
// bilinear interpolation at the window centre over the four nearest coarser
// points, exact in integers (numerators over S^2), clamped to the coarse grid,
// rounded half away from zero.  Without a previous level the guess is zero.
__global__ void k_mw_guess(Level L, Level P, int has_prev, const int32_t *pu, const int32_t *pv, int32_t *gu,
                           int32_t *gv)
{
    const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= static_cast<int64_t>(L.nx) * L.ny) return;
    if (!has_prev) {
        gu[w] = 0;
        gv[w] = 0;
        return;
    }
    const int cx = L.ox + static_cast<int>(w % L.nx) * L.S, cy = L.oy + static_cast<int>(w / L.nx) * L.S;
    const int S = P.S, o = P.W / 2;
    int i0 = (cx - o) >= 0 ? (cx - o) / S : 0, j0 = (cy - o) >= 0 ? (cy - o) / S : 0;
    i0 = min(i0, P.nx - 1);
    j0 = min(j0, P.ny - 1);
    const int i1 = i0 + 1 < P.nx ? i0 + 1 : i0, j1 = j0 + 1 < P.ny ? j0 + 1 : j0;
    int64_t a = static_cast<int64_t>(cx) - o - static_cast<int64_t>(i0) * S;
    int64_t b = static_cast<int64_t>(cy) - o - static_cast<int64_t>(j0) * S;
    a = a < 0 ? 0 : a;
    b = b < 0 ? 0 : b;
    if (a > S || i1 == i0) a = i1 == i0 ? 0 : S;
    if (b > S || j1 == j0) b = j1 == j0 ? 0 : S;
    const int64_t w00 = (S - a) * (S - b), w10 = a * (S - b), w01 = (S - a) * b, w11 = a * b;
    const int64_t den = static_cast<int64_t>(S) * S;
    const int64_t q00 = static_cast<int64_t>(j0) * P.nx + i0, q10 = static_cast<int64_t>(j0) * P.nx + i1;
    const int64_t q01 = static_cast<int64_t>(j1) * P.nx + i0, q11 = static_cast<int64_t>(j1) * P.nx + i1;
    gu[w] = static_cast<int32_t>(round_div(w00 * pu[q00] + w10 * pu[q10] + w01 * pu[q01] + w11 * pu[q11], den));
    gv[w] = static_cast<int32_t>(round_div(w00 * pv[q00] + w10 * pv[q10] + w01 * pv[q01] + w11 * pv[q11], den));
}

// Node-level output: replaced nodes take the integer medians, the others their
// estimate; inactive nodes get valid = 0.
__global__ void k_mw_output(const int32_t *mu, const int32_t *mv, const uint8_t *rep, const float *fu, const float *fv,
                            const int8_t *active, int64_t nodes, float *uo, float *vo, int8_t *valid)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= nodes) return;
    const bool act = active[c] >= 0;
    valid[c] = act ? 1 : 0;
    uo[c] = act ? (rep[c] ? static_cast<float>(mu[c]) : fu[c]) : 0.0f;
    vo[c] = act ? (rep[c] ? static_cast<float>(mv[c]) : fv[c]) : 0.0f;
}

unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

} // namespace

namespace dicmi {

// Window schedule: regular level sizes (largest first, at most 4096) and the
// node-level size (0 if the image cannot hold one).
int mw_levels(int max_disp, int N, int W, int H, int *sizes, int *wf)
{
    int f = 1;
    while (f < N) f <<= 1;
    const int side = std::min(W, H);
    *wf = f <= side ? f : 0;
    int w1 = 1;
    while (w1 <= max_disp && w1 < kMaxWindow) w1 <<= 1;
    while (w1 > side) w1 >>= 1;
    int n = 0;
    for (int w = w1; w > f && n < kMaxLevels - 1; w >>= 1) sizes[n++] = w;
    return n;
}

} // namespace dicmi

namespace {

void launch_fused(const Level &L, int count, const void *ref, int64_t rpitch, int rpix, const void *def,
                  int64_t dpitch, int dpix, int imgW, int imgH, const int32_t *gu, const int32_t *gv,
                  const int8_t *active, int32_t *iu, int32_t *iv, float *fu, float *fv, int sub, hipStream_t s)
{
    const int K = L.W * L.W >= 1024 ? 1 : 1024 / (L.W * L.W);
    const unsigned nb = static_cast<unsigned>((count + K - 1) / K);
#define DIC_MW_FUSED(WIN)                                                                                          \
    k_mw_fused<WIN><<<nb, kFftThreads, 0, s>>>(L, count, ref, rpitch, rpix, def, dpitch, dpix, imgW, imgH, gu, gv, \
                                               active, iu, iv, fu, fv, sub)
    switch (L.W) {
    case 8: DIC_MW_FUSED(8); break;
    case 16: DIC_MW_FUSED(16); break;
    case 32: DIC_MW_FUSED(32); break;
    default: DIC_MW_FUSED(64); break;
    }
#undef DIC_MW_FUSED
}

// one FFT2 of `count` W x W matrices: rows of a, transpose into b, rows of b; the
// result is in b, transposed relative to the input (the cross spectrum is
// element-wise and the inverse pass transposes back)
template <bool INV> void fft2_batch(float2 *a, float2 *b, int W, int count, hipStream_t s)
{
    const int R = W >= 1024 ? 1 : 1024 / W;
    const int64_t rows = static_cast<int64_t>(W) * count;
    const size_t lds = sizeof(float2) * (2 * static_cast<size_t>(R) * W + (W <= kMaxTableWindow ? W / 2 : 0));
    const unsigned nb = static_cast<unsigned>((rows + R - 1) / R);
    k_fft_rows<INV><<<nb, kFftThreads, lds, s>>>(a, W, rows);
    const int T = W < 32 ? W : 32;
    const int64_t tiles = static_cast<int64_t>(W / T) * (W / T) * count;
    k_transpose<<<static_cast<unsigned>(tiles), dim3(32, 32), 0, s>>>(a, b, W);
    k_fft_rows<INV><<<nb, kFftThreads, lds, s>>>(b, W, rows);
}

} // namespace

extern "C" {

dic_status dic_multiwindow(dic_ctx *c, const dic_image *def, const dic_mw_params *prm, float *u_out, float *v_out,
                           int8_t *valid_out, int32_t *levels_out, int32_t *nlevels)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!c->has_ref) FAIL(DIC_E_STATE, "dic_multiwindow before dic_set_reference");
    if (!prm) FAIL(DIC_E_INVAL, "multi-window params is NULL");
    if (!u_out || !v_out || !valid_out) FAIL(DIC_E_INVAL, "NULL output array");
    dic_status st = check_image(c, def, "deformed");
    if (st != DIC_OK) return st;
    if (def->width != c->W || def->height != c->H)
        FAIL(DIC_E_INVAL, "deformed image is %dx%d, reference is %dx%d", def->width, def->height, c->W, c->H);
    if (prm->max_disp < 1) FAIL(DIC_E_INVAL, "max_disp %d", prm->max_disp);
    if (!(prm->mad_threshold >= 0.0) || !std::isfinite(prm->mad_threshold))
        FAIL(DIC_E_INVAL, "mad_threshold %g", prm->mad_threshold);
    int sizes[kMaxLevels], wf = 0;
    const int nlev = mw_levels(prm->max_disp, c->prm.subset_size, c->W, c->H, sizes, &wf);
    if (wf == 0) FAIL(DIC_E_INVAL, "the image cannot hold a %d-pixel node window", c->prm.subset_size);
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;

    // level geometry; the largest level's window count sizes the integer arrays
    std::vector<Level> lv;
    for (int l = 0; l < nlev; ++l) {
        Level L;
        L.W = sizes[l];
        L.S = L.W / 2;
        L.ox = L.oy = L.W / 2;
        L.nx = (c->W - L.W) / L.S + 1;
        L.ny = (c->H - L.W) / L.S + 1;
        L.nodes = false;
        lv.push_back(L);
    }
    Level NL;
    NL.W = wf;
    NL.S = c->prm.step;
    NL.ox = NL.oy = (c->prm.subset_size - 1) / 2;
    NL.nx = c->nx;
    NL.ny = c->ny;
    NL.nodes = true;
    lv.push_back(NL);
    int64_t maxw = 0;
    for (const Level &L : lv) maxw = std::max<int64_t>(maxw, static_cast<int64_t>(L.nx) * L.ny);

    // workspace (grow-only): two batch buffers, integer fields of two levels, guesses,
    // skip flags, the node level's float estimates and replacement flags
    const size_t need_f2 = static_cast<size_t>(std::max<int64_t>(kBatchElems, static_cast<int64_t>(lv[0].W) * lv[0].W));
    if (!c->mw_a || c->mw_cap_f2 < need_f2) {
        dfree(c->mw_a);
        dfree(c->mw_b);
        HIPCHK(hipMalloc(&c->mw_a, sizeof(float2) * need_f2));
        HIPCHK(hipMalloc(&c->mw_b, sizeof(float2) * need_f2));
        c->mw_cap_f2 = need_f2;
    }
    if (!c->mw_int || c->mw_cap_w < maxw) {
        dfree(c->mw_int);
        HIPCHK(hipMalloc(&c->mw_int, (sizeof(int32_t) * 6 + sizeof(float) * 2 + 2) * static_cast<size_t>(maxw)));
        c->mw_cap_w = maxw;
    }
    int32_t *cu = static_cast<int32_t *>(c->mw_int), *cv = cu + maxw;    // this level's estimates
    int32_t *pu = cv + maxw, *pv = pu + maxw;                            // previous level's filtered field
    int32_t *gu = pv + maxw, *gv = gu + maxw;                            // guesses
    float *fu = reinterpret_cast<float *>(gv + maxw), *fv = fu + maxw;   // node-level estimates
    uint8_t *skip = reinterpret_cast<uint8_t *>(fv + maxw), *rep = skip + maxw;
    float2 *za = static_cast<float2 *>(c->mw_a), *zb = static_cast<float2 *>(c->mw_b);

    for (size_t l = 0; l < lv.size(); ++l) {
        const Level &L = lv[l];
        const bool node_level = L.nodes;
        const int64_t M = static_cast<int64_t>(L.nx) * L.ny;
        const Level P = l > 0 ? lv[l - 1] : L;
        k_mw_guess<<<blocks_for(M, 256), 256, 0, s>>>(L, P, l > 0 ? 1 : 0, pu, pv, gu, gv);
        const int64_t WW = static_cast<int64_t>(L.W) * L.W;
        const int per = static_cast<int>(std::max<int64_t>(1, kBatchElems / WW));
        if (L.W <= kMaxFusedWindow) {
            launch_fused(L, static_cast<int>(M), c->ref_raw, static_cast<int64_t>(c->W) * pixel_size(c->ref_pixel),
                         c->ref_pixel, def->data, def->pitch_bytes, def->pixel, c->W, c->H, gu, gv,
                         node_level ? c->flag : nullptr, cu, cv, node_level ? fu : nullptr,
                         node_level ? fv : nullptr, node_level && prm->subpixel ? 1 : 0, s);
        }
        for (int64_t w0 = 0; L.W > kMaxFusedWindow && w0 < M; w0 += per) {
            const int cnt = static_cast<int>(std::min<int64_t>(per, M - w0));
            const int64_t tot = WW * cnt;
            k_mw_load<<<blocks_for(tot, 256), 256, 0, s>>>(L, static_cast<int>(w0), cnt, c->ref_raw,
                                                            static_cast<int64_t>(c->W) * pixel_size(c->ref_pixel),
                                                            c->ref_pixel, def->data, def->pitch_bytes, def->pixel,
                                                            c->W, c->H, gu, gv, node_level ? c->flag : nullptr, za,
                                                            skip);
            fft2_batch<false>(za, zb, L.W, cnt, s);   // spectrum [kx][ky] in zb
            k_mw_cross<<<blocks_for(tot, 256), 256, 0, s>>>(zb, za, L.W, tot);
            fft2_batch<true>(za, zb, L.W, cnt, s);    // map [y][x] in zb
            // za is free again: it holds the part results of the peak search
            const int B = static_cast<int>(std::max<int64_t>(1, WW / kPeakChunk));
            k_mw_peak_part<<<static_cast<unsigned>(cnt * B), kFftThreads, 0, s>>>(zb, L.W, B, za);
            k_mw_peak<<<cnt, kFftThreads, 0, s>>>(zb, za, B, L.W, static_cast<int>(w0), gu, gv, skip, cu, cv,
                                                  node_level ? fu : nullptr, node_level ? fv : nullptr,
                                                  node_level && prm->subpixel ? 1 : 0);
        }
        const float thr = static_cast<float>(prm->mad_threshold);
        if (thr > 0.0f) {
            k_mw_mad<<<blocks_for(M, 256), 256, 0, s>>>(cu, cv, node_level ? c->flag : nullptr, L.nx, L.ny, thr, pu,
                                                        pv, rep);
        } else {
            HIPCHK(hipMemcpyAsync(pu, cu, sizeof(int32_t) * M, hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(pv, cv, sizeof(int32_t) * M, hipMemcpyDeviceToDevice, s));
            launch_zero32(rep, (M + 3) / 4, s);
        }
        if (node_level)
            k_mw_output<<<blocks_for(M, 256), 256, 0, s>>>(pu, pv, rep, fu, fv, c->flag, M, u_out, v_out, valid_out);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    if (nlevels) *nlevels = static_cast<int32_t>(lv.size());
    if (levels_out)
        for (size_t l = 0; l < lv.size(); ++l) levels_out[l] = lv[l].W;
    return DIC_OK;
}

dic_status dic_correlate_mw(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds,
                            const dic_mw_params *prm, dic_result *out)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!c->has_ref) FAIL(DIC_E_STATE, "dic_correlate_mw before dic_set_reference");
    if (nseeds < 1 || !seeds) FAIL(DIC_E_INVAL, "no seeds");
    HIPCHK(hipSetDevice(c->device));
    const int64_t nodes = c->nodes;
    if (!c->mw_node_u || c->mw_node_cap < nodes) {
        dfree(c->mw_node_u);
        HIPCHK(hipMalloc(&c->mw_node_u, (2 * sizeof(float) + 1) * static_cast<size_t>(nodes)));
        c->mw_node_cap = nodes;
    }
    float *u = c->mw_node_u, *v = u + nodes;
    int8_t *valid = reinterpret_cast<int8_t *>(v + nodes);
    dic_status st = dic_multiwindow(c, def, prm, u, v, valid, nullptr, nullptr);
    if (st != DIC_OK) return st;
    // each seed's search centre: the estimate at the node it snaps to
    std::vector<dic_seed> sd(seeds, seeds + nseeds);
    for (int q = 0; q < nseeds; ++q) {
        if (!std::isfinite(sd[q].x) || !std::isfinite(sd[q].y)) continue;   // dic_correlate reports it
        const int64_t node = snap_seed(c, sd[q].x, sd[q].y);
        if (node < 0) continue;
        float uv[2];
        HIPCHK(hipMemcpy(&uv[0], u + node, sizeof(float), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(&uv[1], v + node, sizeof(float), hipMemcpyDeviceToHost));
        sd[q].u0 = uv[0];
        sd[q].v0 = uv[1];
    }
    return dic_correlate(c, def, sd.data(), nseeds, out);
}

} // extern "C"
