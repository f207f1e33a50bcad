// gfx950 kernels of the reliability-guided 2D DIC path.
//
// Paper: Hirst et al., "Pyvale", arXiv 2601.12941.  Sec. 2.2 fixes the cubic
// B-spline interpolation, the ZNSSD cost (Eq. (4)) and the shape functions
// (Eq. (5)); Sec. 2.4 the reliability-guided propagation.  The per-subset
// optimiser is inverse-compositional Gauss-Newton (the paper's LM with zero
// damping).
//
// Layout: coefficient arrays are row-major with kPad mirrored samples on
// every side; `coef` pointers address sample (0,0).  One workgroup of T
// threads owns one subset at a time; thread t holds pixels t, t+T, t+2T, ...
// of the subset in row-major order, their reference value and gradient in
// registers.  The deformed coefficients around the warped subset are staged
// in LDS and re-staged only when the warp drifts out of the staged window.
#include "dic_device.h"

#include <algorithm>
#include <climits>
#include <float.h>
#include <math.h>
#include <type_traits>

// Every multiply-add that should fuse is written as fmaf(); nothing else is
// contracted, so identical expressions give identical bits in every kernel.
#pragma clang fp contract(off)

namespace dicmi {

// All-reduce of NV values over the T threads of a workgroup: wavefront totals, then
// summed in a fixed order from LDS (double buffered by `parity`, since one barrier
// separates consecutive uses).
template <int T, int NV, typename V>
__device__ __forceinline__ void block_allreduce(V (&v)[NV], V *red, int &parity)
{
    if constexpr (NV == 1) v[0] = wave_allreduce(v[0]);
    else wave_allreduce_n<NV>(v);
    if constexpr (T > 64) {
        constexpr int NW = T / 64;
        V *buf = red + parity * NW * NV;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) buf[w * NV + i] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            V acc = buf[i];
#pragma unroll
            for (int ww = 1; ww < NW; ++ww) acc += buf[ww * NV + i];
            v[i] = acc;
        }
        parity ^= 1;
    }
}

// Sum of NV values over the T threads of a workgroup, for wavefront 0 only: the
// same wavefront totals and the same fixed-order sum from LDS as block_allreduce
// (so the totals agree with it bitwise); the other wavefronts skip the read-back.
template <int T, int NV, typename V>
__device__ __forceinline__ void block_reduce_first(V (&v)[NV], V *red, int &parity)
{
    if constexpr (NV == 1) v[0] = wave_allreduce(v[0]);
    else wave_allreduce_n<NV>(v);
    if constexpr (T > 64) {
        constexpr int NW = T / 64;
        V *buf = red + parity * NW * NV;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) buf[w * NV + i] = v[i];
        }
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                V acc = buf[i];
#pragma unroll
                for (int ww = 1; ww < NW; ++ww) acc += buf[ww * NV + i];
                v[i] = acc;
            }
        }
        parity ^= 1;
    }
}

// Subset pixels over the T threads of a workgroup, column per thread: thread t owns
// column c = t mod N of the subset and rows r0 + R j (r0 = t div N, R = T div N rows
// per pass) for j < P; threads t >= N R own nothing.  Offsets from the subset centre:
// dx = c - h (fixed per thread), dy = r0 - h + R j.
struct Columns {
    int c, r0, R, jmax;   // jmax: number of valid rows of this thread
    __device__ __forceinline__ Columns(int t, int T, int N)
    {
        R = T / N;
        c = t % N;
        r0 = t / N;
        jmax = t < N * R ? (N - r0 + R - 1) / R : 0;
    }
};

// Per-thread partial sums of one pass over the subset, all in FP32:
//   s[0] = sum g',  s[1] = sum g'^2,  s[2] = sum fbar g',
//   s[3+k] = sum J_k g'  with J = grad f . dW/dp in Eq. (5) order:
//   [fx, fy, fx dx, fx dy, fy dx, fy dy, fx dx^2, fx dx dy, fx dy^2, fy dx^2, fy dx dy, fy dy^2].
// g' is the deformed value minus the reference subset mean.  A thread walks
// the rows of one subset column, so dx is the same for all its pixels: the
// pass accumulates only the terms without a dx factor, and finish_column
// multiplies the others out once at the end.
template <int NP>
__device__ __forceinline__ void accumulate(float (&s)[3 + NP], float g, float fb, float gx, float gy, float dy)
{
    s[0] = s[0] + g;
    s[1] = fmaf(g, g, s[1]);
    s[2] = fmaf(fb, g, s[2]);
    const float a = gx * g;
    const float c = gy * g;
    s[3] = s[3] + a;
    s[4] = s[4] + c;
    s[6] = fmaf(a, dy, s[6]);
    s[8] = fmaf(c, dy, s[8]);
    if constexpr (NP == 12) {
        s[11] = fmaf(a * dy, dy, s[11]);
        s[14] = fmaf(c * dy, dy, s[14]);
    }
}

// the dx-weighted sums of one column, from the sums accumulate kept
template <int NP>
__device__ __forceinline__ void finish_column(float (&s)[3 + NP], float dx)
{
    s[5] = dx * s[3];
    s[7] = dx * s[4];
    if constexpr (NP == 12) {
        s[9] = dx * s[5];
        s[10] = dx * s[6];
        s[12] = dx * s[7];
        s[13] = dx * s[8];
    }
}

// ---------------------------------------------------------------------------
// B-spline prefilter.  The exact inverse of the sampled cubic B-spline
// (c[k-1] + 4c[k] + c[k+1])/6 = s[k] has the two-sided impulse response
// h[n] = sqrt(3) (sqrt(3)-2)^|n| (Unser 1993); truncated at |n| <= 15 its
// tail is below 3.4e-9 of max|s|, far under FP32 resolution.  With the
// mirror-extended input the truncated FIR reproduces the mirror-boundary
// solution.  Separable: rows into an FP32 scratch array, then columns into the
// padded coefficient array (padding filled with the mirrored coefficients,
// the padding rows by a small kernel of their own).
// The stored coefficients are 1/36 of these (1/6 per pass), to match the
// interpolation weights, which are 6 times the B-spline's.
// ---------------------------------------------------------------------------
constexpr int kFir = 15;
__constant__ float c_fir[2 * kFir + 1];

constexpr int kRowBlock = 256;
constexpr int kRowOut = 4;   // consecutive outputs per thread of the row pass

// Rows: a workgroup stages kRowBlock * kRowOut pixels of one row and their
// 15-pixel halos in LDS; each thread reads its kRowOut + 30 inputs as 16-byte
// LDS vectors and evaluates its kRowOut outputs from registers, each the same
// 31-term FMA chain as a direct evaluation.
__global__ __launch_bounds__(kRowBlock) void k_prefilter_rows(const void *src, int64_t sp, int pixel, int W,
                                                               float *tmp, int64_t tp)
{
    constexpr int kSpan = kRowBlock * kRowOut;
    constexpr int kVec = (kRowOut + 2 * kFir + 3) / 4;   // 16-byte reads per thread
    __shared__ float4 s4[kSpan / 4 + kVec];
    float *s = reinterpret_cast<float *>(s4);
    const int y = blockIdx.y;
    const int xb = blockIdx.x * kSpan;
    if (xb >= kFir && xb + kSpan + kFir <= W) {
        for (int i = threadIdx.x; i < kSpan + 2 * kFir; i += kRowBlock) s[i] = load_pixel(src, sp, pixel, xb - kFir + i, y);
    } else {
        for (int i = threadIdx.x; i < kSpan + 2 * kFir; i += kRowBlock)
            s[i] = load_pixel(src, sp, pixel, fold(xb - kFir + i, W), y);
    }
    __syncthreads();
    float v[4 * kVec];
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
        const float4 q = s4[threadIdx.x * (kRowOut / 4) + j];
        v[4 * j] = q.x;
        v[4 * j + 1] = q.y;
        v[4 * j + 2] = q.z;
        v[4 * j + 3] = q.w;
    }
    const int x0 = xb + threadIdx.x * kRowOut;
    float *out = tmp + static_cast<int64_t>(y) * tp + x0;
#pragma unroll
    for (int r = 0; r < kRowOut; ++r) {
        if (x0 + r >= W) break;
        float acc = 0.0f;
#pragma unroll
        for (int n = -kFir; n <= kFir; ++n) acc = fmaf(c_fir[n + kFir], v[r + kFir - n], acc);
        out[r] = acc;
    }
}

__device__ __forceinline__ void store_coef(float *d, float v) { *d = v; }
__device__ __forceinline__ void store_coef(__half *d, float v) { *d = __float2half(v); }

// Columns: a thread walks kColRows consecutive rows of one column with the
// kColRows + 30 input samples in registers (about 3 loads per coefficient instead
// of 31); every coefficient is the same 31-term FMA chain in the same order as a
// direct evaluation, so the result does not depend on the strip it falls in.
constexpr int kColRows = 16;

template <typename OutT>
__global__ __launch_bounds__(256) void k_prefilter_cols(const float *tmp, int64_t tp, int W, int H, OutT *dst,
                                                         int64_t dp)
{
    const int x = blockIdx.x * 64 + threadIdx.x - kPad;
    const int y0 = (blockIdx.y * 4 + threadIdx.y) * kColRows;
    if (x >= W + kPad || y0 >= H) return;
    const int xm = fold(x, W);
    float v[kColRows + 2 * kFir];
    if (y0 >= kFir && y0 + kColRows + kFir <= H) {
        // strip and halo inside the image: consecutive rows, no folding
        const float *q = tmp + static_cast<int64_t>(y0 - kFir) * tp + xm;
#pragma unroll
        for (int i = 0; i < kColRows + 2 * kFir; ++i) {
            v[i] = *q;
            q += tp;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kColRows + 2 * kFir; ++i)
            v[i] = tmp[static_cast<int64_t>(fold(y0 - kFir + i, H)) * tp + xm];
    }
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
        if (y0 + r >= H) break;
        float acc = 0.0f;
#pragma unroll
        for (int n = -kFir; n <= kFir; ++n) acc = fmaf(c_fir[n + kFir], v[r + kFir - n], acc);
        store_coef(dst + static_cast<int64_t>(y0 + r) * dp + x, acc);
    }
}

// The padding rows (kPad above and below the image): each coefficient evaluated
// directly at its mirrored row, the same chain as k_prefilter_cols.
template <typename OutT>
__global__ __launch_bounds__(256) void k_prefilter_pad_rows(const float *tmp, int64_t tp, int W, int H, OutT *dst,
                                                             int64_t dp)
{
    const int x = blockIdx.x * 64 + threadIdx.x - kPad;
    const int i = blockIdx.y * 4 + threadIdx.y;   // 0 .. 2 kPad - 1
    if (x >= W + kPad || i >= 2 * kPad) return;
    const int y = i < kPad ? i - kPad : H + i - kPad;
    const int xm = fold(x, W);
    const int ym = fold(y, H);
    float acc = 0.0f;
#pragma unroll
    for (int n = -kFir; n <= kFir; ++n)
        acc = fmaf(c_fir[n + kFir], tmp[static_cast<int64_t>(fold(ym - n, H)) * tp + xm], acc);
    store_coef(dst + static_cast<int64_t>(y) * dp + x, acc);
}

void launch_prefilter(const void *src, int64_t src_pitch_bytes, int pixel, int W, int H, float *tmp,
                      int64_t tmp_pitch, void *dst, int64_t dst_pitch, bool half, hipStream_t s)
{
    static bool taps_ready[64] = {};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64 || !taps_ready[dev]) {
        float h[2 * kFir + 1];
        const double z = sqrt(3.0) - 2.0;
        // each pass carries the 1/6 of its axis that the scaled interpolation weights leave out
        for (int n = -kFir; n <= kFir; ++n)
            h[n + kFir] = static_cast<float>(sqrt(3.0) * pow(fabs(z), abs(n)) * ((abs(n) & 1) ? -1.0 : 1.0) / 6.0);
        (void)hipMemcpyToSymbol(HIP_SYMBOL(c_fir), h, sizeof(h));
        if (dev >= 0 && dev < 64) taps_ready[dev] = true;
    }
    dim3 g1((W + kRowBlock * kRowOut - 1) / (kRowBlock * kRowOut), H);
    k_prefilter_rows<<<g1, kRowBlock, 0, s>>>(src, src_pitch_bytes, pixel, W, tmp, tmp_pitch);
    dim3 g2((W + 2 * kPad + 63) / 64, (H + 4 * kColRows - 1) / (4 * kColRows));
    dim3 g3((W + 2 * kPad + 63) / 64, (2 * kPad + 3) / 4);
    if (half) {
        k_prefilter_cols<__half><<<g2, dim3(64, 4), 0, s>>>(tmp, tmp_pitch, W, H, static_cast<__half *>(dst),
                                                             dst_pitch);
        k_prefilter_pad_rows<__half><<<g3, dim3(64, 4), 0, s>>>(tmp, tmp_pitch, W, H, static_cast<__half *>(dst),
                                                                 dst_pitch);
    } else {
        k_prefilter_cols<float><<<g2, dim3(64, 4), 0, s>>>(tmp, tmp_pitch, W, H, static_cast<float *>(dst),
                                                            dst_pitch);
        k_prefilter_pad_rows<float><<<g3, dim3(64, 4), 0, s>>>(tmp, tmp_pitch, W, H, static_cast<float *>(dst),
                                                                dst_pitch);
    }
}

// ---------------------------------------------------------------------------
// Reference precompute: the interpolant and its gradient at every pixel
// (t = 0 weights, the same expression the iteration uses for the deformed
// image), then per node the sums the iteration reuses and the inverse of the
// Gauss-Newton Hessian.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ref_pixels(RefView R, float *pa)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= R.W || y >= R.H) return;
    float w0, w1, w2, w3, d0, d1, d2, d3;
    bspline_w(0.0f, w0, w1, w2, w3);
    bspline_dw(0.0f, d0, d1, d2, d3);
    const float *b = R.coef + static_cast<int64_t>(y - 1) * R.cpitch + (x - 1);
    float *o = pa + 3 * (static_cast<int64_t>(y) * R.ppitch + x);
    o[0] = interp16(b, R.cpitch, w0, w1, w2, w3, w0, w1, w2, w3);
    o[1] = interp16(b, R.cpitch, d0, d1, d2, d3, w0, w1, w2, w3);
    o[2] = interp16(b, R.cpitch, w0, w1, w2, w3, d0, d1, d2, d3);
}

void launch_ref_pixels(const RefView &R, float *pa, hipStream_t s)
{
    dim3 g((R.W + 63) / 64, (R.H + 3) / 4);
    k_ref_pixels<<<g, dim3(64, 4), 0, s>>>(R, pa);
}

__global__ __launch_bounds__(256) void k_ref_component(RefView R, int a, float *out)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= R.W || y >= R.H) return;
    out[static_cast<int64_t>(y) * R.W + x] = R.pa[3 * (static_cast<int64_t>(y) * R.ppitch + x) + a];
}

void launch_ref_component(const RefView &R, int a, float *out, hipStream_t s)
{
    dim3 g((R.W + 63) / 64, (R.H + 3) / 4);
    k_ref_component<<<g, dim3(64, 4), 0, s>>>(R, a, out);
}

// A node is active iff all N^2 pixels of its subset are inside the ROI.
__global__ void k_active(const uint8_t *roi, RefView R, int8_t *flag)
{
    const int64_t node = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (node >= R.nodes) return;
    const int ix = static_cast<int>(node % R.nx), iy = static_cast<int>(node / R.nx);
    const int x0 = ix * R.step, y0 = iy * R.step;
    bool ok = true;
    if (roi) {
        for (int y = 0; y < R.N && ok; ++y) {
            const uint8_t *row = roi + static_cast<int64_t>(y0 + y) * R.W + x0;
            for (int x = 0; x < R.N; ++x) ok = ok && row[x] != 0;
        }
    }
    flag[node] = ok ? 0 : -1;
}

void launch_active(const uint8_t *roi, const RefView &R, int8_t *flag, hipStream_t s)
{
    const int64_t blocks = (R.nodes + 255) / 256;
    k_active<<<static_cast<unsigned>(blocks), 256, 0, s>>>(roi, R, flag);
}

template <int NP>
__device__ __forceinline__ void steepest(double (&J)[NP], double gx, double gy, double dx, double dy)
{
    J[0] = gx;
    J[1] = gy;
    J[2] = gx * dx;
    J[3] = gx * dy;
    J[4] = gy * dx;
    J[5] = gy * dy;
    if constexpr (NP == 12) {
        J[6] = gx * dx * dx;
        J[7] = gx * dx * dy;
        J[8] = gx * dy * dy;
        J[9] = gy * dx * dx;
        J[10] = gy * dx * dy;
        J[11] = gy * dy * dy;
    }
}


// Slot of sum-group B entry i in the per-node cache: entries 0..NP-1 (sum J) go
// to slots 3..3+NP-1, entries NP.. (sum J J^T, upper triangle by rows) to the
// Hessian slots 3+2NP.. .
template <int NP> __device__ __forceinline__ int slot_b(int i) { return i < NP ? 3 + i : 3 + NP + i; }

// Per-node sums over the reference subset, written raw to the cache (slot
// layout as read by the wave kernel; k_ref_factor then turns them into the
// cached quantities).  Group A, the sums the iteration recomputes for the
// deformed subset (sum fbar, sum fbar^2, sum J fbar), is reduced exactly as the
// iteration reduces its own, so that an identical deformed subset reproduces
// them bitwise.  Group B (sum J and sum J J^T, FP64 per lane) is reduced by a
// pair exchange and an LDS transpose, in a fixed order.
template <int NP, int T, int P>
__global__ __launch_bounds__(T) void k_ref_nodes(RefView R, double *cache, int8_t *flag)
{
    constexpr int NH = NP * (NP + 1) / 2;
    constexpr int NB = NP + NH;
    constexpr int kNC = 3 + 2 * NP + NH;        // per-node cache slots, contiguous per node
    constexpr int NW = T / 64;
    constexpr int CH = NB < 32 ? NB : 32;      // group-B entries per LDS pass
    constexpr int LS = 33;                      // LDS row stride (doubles) of one entry
    __shared__ double red[2 * NW * (3 + NP)];
    __shared__ double tr[NW * CH * LS];
    __shared__ double part[NW * CH];
    int parity = 0;
    const int N = R.N, h = (N - 1) / 2, n = N * N;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const Columns L(t, T, N);
    const float dxf = static_cast<float>(L.c - h);
    const float dy0 = static_cast<float>(L.r0 - h), dyR = static_cast<float>(L.R);
    const int64_t nn = R.nodes;
    const int64_t rstep = static_cast<int64_t>(L.R) * R.ppitch;
    for (int64_t node = blockIdx.x; node < nn; node += gridDim.x) {
        if (flag[node] < 0) continue;
        const int xc = h + static_cast<int>(node % R.nx) * R.step;
        const int yc = h + static_cast<int>(node / R.nx) * R.step;
        const int64_t o0 = static_cast<int64_t>(yc - h + L.r0) * R.ppitch + xc - h + L.c;
        double sf[1] = {0.0};
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (j < L.jmax) sf[0] += static_cast<double>(R.pa[3 * (o0 + j * rstep)]);
        block_allreduce<T, 1>(sf, red, parity);
        const double fm = sf[0] / n;
        const float fm32 = static_cast<float>(fm);
        float s[3 + NP];
#pragma unroll
        for (int i = 0; i < 3 + NP; ++i) s[i] = 0.0f;
        double vb[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) vb[i] = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (j < L.jmax) {
                const float *a = R.pa + 3 * (o0 + j * rstep);
                const float fb = a[0] - fm32;
                const float gx = a[1], gy = a[2];
                const float dyf = fmaf(static_cast<float>(j), dyR, dy0);
                accumulate<NP>(s, fb, fb, gx, gy, dyf);
                double J[NP];
                steepest<NP>(J, gx, gy, dxf, dyf);
                int q = NP;
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    vb[a] += J[a];
#pragma unroll
                    for (int b = a; b < NP; ++b) {
                        vb[q] = fma(J[a], J[b], vb[q]);
                        ++q;
                    }
                }
            }
        }
        finish_column<NP>(s, dxf);
        double va[3 + NP];
#pragma unroll
        for (int i = 0; i < 3 + NP; ++i) va[i] = static_cast<double>(s[i]);
        block_allreduce<T, 3 + NP>(va, red, parity);
        if (t == 0) {
            double *cn = cache + node * kNC;
            cn[0] = fm;
            cn[1] = va[1];
            cn[2] = va[0];
#pragma unroll
            for (int a = 0; a < NP; ++a) cn[3 + NP + a] = va[3 + a];
        }
        // group B: lanes 2k and 2k+1 pair up, then entry i of the 32 pair sums of
        // every wavefront sits in an LDS row that one lane adds up
#pragma unroll
        for (int i = 0; i < NB; ++i) vb[i] += dpp_read<0xB1>(vb[i]);
#pragma unroll
        for (int c0 = 0; c0 < NB; c0 += CH) {
            if ((lane & 1) == 0) {
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    if (c0 + i < NB) tr[(w * CH + i) * LS + (lane >> 1)] = vb[c0 + i];
            }
            __syncthreads();
            double tot = 0.0;
            if (lane < CH && c0 + lane < NB) {
                const double *row = tr + (w * CH + lane) * LS;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                for (int k = 0; k < 32; k += 4) {
                    a0 += row[k];
                    a1 += row[k + 1];
                    a2 += row[k + 2];
                    a3 += row[k + 3];
                }
                tot = (a0 + a1) + (a2 + a3);
            }
            if constexpr (NW > 1) {
                if (lane < CH) part[w * CH + lane] = tot;
                __syncthreads();
                if (w == 0 && lane < CH) {
                    tot = part[lane];
#pragma unroll
                    for (int ww = 1; ww < NW; ++ww) tot += part[ww * CH + lane];
                }
            }
            if (w == 0 && lane < CH && c0 + lane < NB)
                cache[node * kNC + slot_b<NP>(c0 + lane)] = tot;
            __syncthreads();
        }
    }
}

// Packed lower-triangle index (row i, column j <= i).
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// One thread per node: from the raw sums, the reference deviation, the
// centred sums sum J fbar, the flat and singular checks, and the inverse of
// the centred Gauss-Newton Hessian (Cholesky, inverse of the factor, product),
// all in FP64 and fully unrolled.
template <int NP>
__global__ __launch_bounds__(256) void k_ref_factor(RefView R, double *cache, int8_t *flag)
{
    constexpr int NH = NP * (NP + 1) / 2;
    const int64_t node = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nn = R.nodes;
    if (node >= nn || flag[node] < 0) return;
    const int N = R.N, h = (N - 1) / 2, n = N * N;
    constexpr int kNC = 3 + 2 * NP + NH;
    double *c = cache + node * kNC;
    const double fm = c[0], S1 = c[1], S0 = c[2];
    // same expressions as the iteration's dg2 and J^T gbar, so that an
    // identical deformed subset gives a bitwise-zero increment
    const double gm = S0 * (1.0 / n);
    const double df2 = S1 - S0 * gm;
    double SJ[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        SJ[a] = c[3 + a];
        c[3 + NP + a] = c[3 + NP + a] - gm * SJ[a];
    }
    c[1] = df2;
    int8_t st = 0;
    const double lev = fmax(1.0, fabs(fm));
    if (isnan(df2)) st = kNan;
    else if (df2 <= n * (kFlatRel * lev) * (kFlatRel * lev)) st = kFlatRef;
    // centred Hessian H = sum J J^T - SJ SJ^T / n, lower triangle
    double Lm[NH];
    {
        int q = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a)
#pragma unroll
            for (int b = a; b < NP; ++b) {
                Lm[tri(b, a)] = c[3 + 2 * NP + q] - SJ[a] * SJ[b] / n;
                ++q;
            }
    }
    double hmax = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        const double scl = a < 2 ? 1.0 : (a < 6 ? static_cast<double>(h) * h : static_cast<double>(h) * h * h * h);
        hmax = fmax(hmax, Lm[tri(a, a)] / scl);
    }
    // in-place Cholesky; the first failing pivot sets the status and the rest
    // runs on a unit pivot (its output is discarded)
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        const double scl = a < 2 ? 1.0 : (a < 6 ? static_cast<double>(h) * h : static_cast<double>(h) * h * h * h);
        double d = Lm[tri(a, a)];
#pragma unroll
        for (int k = 0; k < a; ++k) d -= Lm[tri(a, k)] * Lm[tri(a, k)];
        if (st == 0) {
            if (isnan(d)) st = kNan;
            else if (!(d > kSingularRel * scl * hmax)) st = kSingular;
        }
        const double la = st == 0 ? sqrt(d) : 1.0;
        Lm[tri(a, a)] = la;
#pragma unroll
        for (int i = a + 1; i < NP; ++i) {
            double x = Lm[tri(i, a)];
#pragma unroll
            for (int k = 0; k < a; ++k) x -= Lm[tri(i, k)] * Lm[tri(a, k)];
            Lm[tri(i, a)] = x / la;
        }
    }
    // L^{-1} in place, column by column; then H^{-1} = L^{-T} L^{-1} (upper, by rows)
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const double dj = 1.0 / Lm[tri(j, j)];
#pragma unroll
        for (int i = j + 1; i < NP; ++i) {
            double x = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) x -= Lm[tri(i, k)] * (k == j ? dj : Lm[tri(k, j)]);
            Lm[tri(i, j)] = x / Lm[tri(i, i)];
        }
        Lm[tri(j, j)] = dj;
    }
    int q = 3 + 2 * NP;
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int b = a; b < NP; ++b) {
            double x = 0.0;
#pragma unroll
            for (int k = b; k < NP; ++k) x += Lm[tri(k, a)] * Lm[tri(k, b)];
            c[q++] = st == 0 ? x : 0.0;
        }
    flag[node] = st;
}

template <int NP, int T, int P>
static void ref_nodes_inst(const RefView &R, double *cache, int8_t *flag, hipStream_t s)
{
    const int64_t blocks = R.nodes < 8192 ? R.nodes : 8192;
    k_ref_nodes<NP, T, P><<<static_cast<unsigned>(blocks < 1 ? 1 : blocks), T, 0, s>>>(R, cache, flag);
    k_ref_factor<NP><<<static_cast<unsigned>((R.nodes + 255) / 256), 256, 0, s>>>(R, cache, flag);
}

// ---------------------------------------------------------------------------
// Seed initialisation: ZNCC of the raw reference subset against the raw
// deformed subset at every integer shift of round(u0, v0) + [-R, R]^2 (shifts
// leaving the image are skipped).  Integer pixels are summed exactly in int64,
// the ZNCC formed in FP64; the best shift wins, exact ties going to the
// smaller du^2 + dv^2, then smaller dv, then smaller du.
// ---------------------------------------------------------------------------
constexpr int kSeedBlock = 256;

__global__ __launch_bounds__(kSeedBlock) void k_seed_search(RefView R, const FrameState *frames, int nseeds,
                                                            int radius, const int32_t *centre, double *zbuf)
{
    const int side = 2 * radius + 1;
    const int shift = blockIdx.x, si = blockIdx.y, f = blockIdx.z;
    const FrameState &F = frames[f];
    if (si >= F.nseeds) return;
    const int node = F.seed_nodes[si];
    const int du = centre[2 * (f * nseeds + si)] + shift % side - radius;
    const int dv = centre[2 * (f * nseeds + si) + 1] + shift / side - radius;
    const int N = R.N, h = (N - 1) / 2, n = N * N;
    const int xc = h + (node % R.nx) * R.step, yc = h + (node / R.nx) * R.step;
    double *out = zbuf + (static_cast<int64_t>(f) * nseeds + si) * side * side + shift;
    if (xc - h + du < 0 || xc + h + du > R.W - 1 || yc - h + dv < 0 || yc + h + dv > R.H - 1) {
        if (threadIdx.x == 0) *out = -INFINITY;
        return;
    }
    const int64_t rpitch = static_cast<int64_t>(R.W) * (R.pixel == 0 ? 1 : (R.pixel == 1 ? 2 : 4));
    __shared__ long long si64[kSeedBlock][5];
    __shared__ double sd[kSeedBlock][5];
    const bool integer = R.pixel != 2;
    long long a[5] = {0, 0, 0, 0, 0};
    double d[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < n; i += kSeedBlock) {
        const int x = xc + i % N - h, y = yc + i / N - h;
        const float fv = load_pixel(R.raw, rpitch, R.pixel, x, y);
        const float gv = load_pixel(F.draw, F.draw_pitch, F.dpixel, x + du, y + dv);
        if (integer) {
            const long long fi = static_cast<long long>(fv), gi = static_cast<long long>(gv);
            a[0] += fi; a[1] += fi * fi; a[2] += gi; a[3] += gi * gi; a[4] += fi * gi;
        } else {
            const double fd = fv, gd = gv;
            d[0] += fd; d[1] += fd * fd; d[2] += gd; d[3] += gd * gd; d[4] += fd * gd;
        }
    }
    for (int k = 0; k < 5; ++k) { si64[threadIdx.x][k] = a[k]; sd[threadIdx.x][k] = d[k]; }
    __syncthreads();
    for (int m = kSeedBlock / 2; m > 0; m >>= 1) {
        if (threadIdx.x < m)
            for (int k = 0; k < 5; ++k) {
                si64[threadIdx.x][k] += si64[threadIdx.x + m][k];
                sd[threadIdx.x][k] += sd[threadIdx.x + m][k];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double num, A, B;
        if (integer) {
            const long long sf = si64[0][0], sff = si64[0][1], sg = si64[0][2], sgg = si64[0][3], sfg = si64[0][4];
            num = static_cast<double>(static_cast<long long>(n) * sfg - sf * sg);
            A = static_cast<double>(static_cast<long long>(n) * sff - sf * sf);
            B = static_cast<double>(static_cast<long long>(n) * sgg - sg * sg);
        } else {
            num = n * sd[0][4] - sd[0][0] * sd[0][2];
            A = n * sd[0][1] - sd[0][0] * sd[0][0];
            B = n * sd[0][3] - sd[0][2] * sd[0][2];
        }
        *out = (A > 0.0 && B > 0.0) ? num / sqrt(A * B) : -INFINITY;
    }
}

void launch_seed_search(const RefView &R, const FrameState *F_dev, int nframes, int nseeds, int radius,
                        const int32_t *centre, double *zbuf, hipStream_t s)
{
    const int side = 2 * radius + 1;
    dim3 g(side * side, nseeds, nframes);
    k_seed_search<<<g, kSeedBlock, 0, s>>>(R, F_dev, nseeds, radius, centre, zbuf);
}

__global__ void k_seed_pick(RefView R, const FrameState *frames, int nseeds, int radius, const int32_t *centre,
                            const double *zbuf)
{
    const int si = threadIdx.x + blockIdx.x * blockDim.x, f = blockIdx.y;
    const FrameState &F = frames[f];
    if (si >= F.nseeds) return;
    const int side = 2 * radius + 1;
    const double *z = zbuf + (static_cast<int64_t>(f) * nseeds + si) * side * side;
    int bu = 0, bv = 0, found = 0;
    double bz = 0.0;
    for (int q = 0; q < side * side; ++q) {
        if (z[q] == -INFINITY) continue;
        const int du = centre[2 * (f * nseeds + si)] + q % side - radius;
        const int dv = centre[2 * (f * nseeds + si) + 1] + q / side - radius;
        bool better = !found || z[q] > bz;
        if (found && z[q] == bz) {
            const long d2 = static_cast<long>(du) * du + static_cast<long>(dv) * dv;
            const long b2 = static_cast<long>(bu) * bu + static_cast<long>(bv) * bv;
            better = d2 < b2 || (d2 == b2 && (dv < bv || (dv == bv && du < bu)));
        }
        if (better) { found = 1; bz = z[q]; bu = du; bv = dv; }
    }
    if (si == 0) F.counts[0] = F.nseeds;
    F.seed_p[2 * si] = bu;
    F.seed_p[2 * si + 1] = bv;
    F.wave[F.seed_nodes[si]] = 0;
    F.list0[si] = F.seed_nodes[si];
}

void launch_seed_pick(const RefView &R, const FrameState *F_dev, int nframes, int nseeds, int radius,
                      const int32_t *centre, const double *zbuf, hipStream_t s)
{
    dim3 g((nseeds + 63) / 64, nframes);
    k_seed_pick<<<g, 64, 0, s>>>(R, F_dev, nseeds, radius, centre, zbuf);
}

// ---------------------------------------------------------------------------
// Per-frame initialisation and finalisation.
// ---------------------------------------------------------------------------
__global__ void k_init_frame(RefView R, FrameState F, int np)
{
    const int64_t node = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (node >= R.nodes) return;
    for (int j = 0; j < np; ++j) F.p[j * R.nodes + node] = 0.0f;
    F.zncc[node] = 0.0f;
    F.iters[node] = 0;
    F.status[node] = R.flag[node] < 0 ? kNotInRoi : kNotReached;
    F.wave[node] = -1;
    F.pkey[node] = 0;
    F.counts[node] = 0;
    if (node == 0) {
        F.counts[R.nodes] = 0;
        F.counts[R.nodes + 1] = 0;
    }
}

void launch_init_frame(const RefView &R, const FrameState &F, int np, hipStream_t s)
{
    k_init_frame<<<static_cast<unsigned>((R.nodes + 255) / 256), 256, 0, s>>>(R, F, np);
}

__global__ void k_finalize(RefView R, FrameState F, int np)
{
    const int64_t node = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (node >= R.nodes) return;
    if (F.status[node] != kConverged)
        for (int j = 0; j < np; ++j) F.p[j * R.nodes + node] = __int_as_float(0x7fc00000);
}

// Per-frame counters from the results: nodes computed (wave >= 0), converged,
// and IC-GN iterations; one atomic per block and counter.
__global__ __launch_bounds__(256) void k_frame_stats(RefView R, FrameState F)
{
    // stat[0] computed nodes, [1] converged, [2] iterations, [3] waves (largest wave index + 1)
    unsigned long long a = 0, b = 0, c = 0, d = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < R.nodes;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const int wv = F.wave[i];
        a += wv >= 0 ? 1 : 0;
        b += F.status[i] == kConverged ? 1 : 0;
        c += static_cast<unsigned long long>(F.iters[i]);
        d = max(d, static_cast<unsigned long long>(wv + 1));
    }
    for (int m = 1; m < 64; m <<= 1) {
        a += __shfl_xor(a, m);
        b += __shfl_xor(b, m);
        c += __shfl_xor(c, m);
        d = max(d, __shfl_xor(d, m));
    }
    __shared__ unsigned long long part[4][4];
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6][0] = a;
        part[threadIdx.x >> 6][1] = b;
        part[threadIdx.x >> 6][2] = c;
        part[threadIdx.x >> 6][3] = d;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const unsigned long long v = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                                     part[3][threadIdx.x];
        atomicAdd(F.stat + threadIdx.x, v);
    } else if (threadIdx.x == 3) {
        const unsigned long long v = max(max(part[0][3], part[1][3]), max(part[2][3], part[3][3]));
        atomicMax(F.stat + 3, v);
    }
}

void launch_frame_stats(const RefView &R, const FrameState &F, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((R.nodes + 255) / 256, 1024);
    k_frame_stats<<<static_cast<unsigned>(blocks), 256, 0, s>>>(R, F);
}

// Zero `words` 32-bit words (a kernel rather than a memset node, so the same
// sequence may also run inside a captured graph).
__global__ void k_zero32(uint32_t *p, int64_t words)
{
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

void launch_zero32(void *p, int64_t words, hipStream_t s)
{
    if (words <= 0) return;
    const int64_t blocks = std::min<int64_t>((words + 255) / 256, 1024);
    k_zero32<<<static_cast<unsigned>(blocks), 256, 0, s>>>(static_cast<uint32_t *>(p), words);
}

// For each of n frames (device array), the size of the wave it runs at launch step
// `step` (0 before its start or past its counts).
__global__ void k_gather_next(const FrameState *frames, int n, int step, int32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int kf = step - frames[i].k_base;
    out[i] = (kf >= 0 && kf <= frames[i].kmax) ? frames[i].counts[kf] : 0;
}

void launch_gather_next(const FrameState *F_dev, int n, int step, int32_t *out, hipStream_t s)
{
    if (n > 0) k_gather_next<<<(n + 63) / 64, 64, 0, s>>>(F_dev, n, step, out);
}

// Size of wave k summed over the frames (read by the host once per chunk).
__global__ void k_count_wave(const FrameState *frames, int nframes, int k, int32_t *out)
{
    if (threadIdx.x != 0) return;
    int acc = 0;
    for (int f = 0; f < nframes; ++f) acc += frames[f].counts[k];
    out[k] = acc;
}

void launch_count_wave(const FrameState *F_dev, int nframes, int k, int32_t *out, hipStream_t s)
{
    k_count_wave<<<1, 64, 0, s>>>(F_dev, nframes, k, out);
}

void launch_finalize(const RefView &R, const FrameState &F, int np, bool nan_unconverged, hipStream_t s)
{
    if (!nan_unconverged) return;
    k_finalize<<<static_cast<unsigned>((R.nodes + 255) / 256), 256, 0, s>>>(R, F, np);
}

// ---------------------------------------------------------------------------
// One frontier wave: every subset of wave k of every frame.
// ---------------------------------------------------------------------------
// Affine register blocks of at most 4 rows fit three wavefronts per SIMD without
// spilling, quadratic ones of at most 8 rows two (a few bytes of the FP64 tail
// spill for 8 rows, far cheaper than running one wavefront per SIMD); ask the
// compiler for that occupancy there.
template <int NP, int P> constexpr int wave_occupancy_hint() { return NP == 6 ? (P <= 4 ? 3 : 1) : (P <= 8 ? 2 : 1); }

// Row software pipelining needs 16 more registers; blocks of 11 to 16 rows run two
// wavefronts per SIMD either way, smaller ones would lose their third.
template <int P> constexpr bool kPipelineRows() { return P >= 11; }

template <int NP, int T, int P, bool F64>
__global__ __launch_bounds__(T, (wave_occupancy_hint<NP, P>())) void k_wave(const FrameTable frames, int step)
{
    using Acc = typename std::conditional<F64, double, float>::type;
    constexpr int NS = 3 + NP;
    constexpr int NH = NP * (NP + 1) / 2;
    constexpr int NC = 3 + 2 * NP + NH;   // per-node reference cache slots
    extern __shared__ float tile[];  // ts * ts deformed coefficients
    __shared__ Acc red[2 * (T / 64) * NS];
    __shared__ int prefix[kMaxFrames + 1];
    __shared__ int owned[kMaxFrames + 1];
    __shared__ double cache[NC];      // this subset's reference cache
    __shared__ float qa[4 * NP];      // the four possible parents' parameters
    __shared__ double pub_p[NP];      // parameters published by the first wavefront
    __shared__ double qwork[NP == 12 ? 48 : 1];   // quadratic composition's working matrix
    __shared__ int pub_stop;
    const int nframes = frames.n;

    // Frame affinity: workgroups are placed on the 8 XCDs round-robin by index, so
    // with a multiple of 8 frames the workgroups of one XCD (index mod 8) take every
    // 8th frame and that XCD's L2 holds only those frames' coefficient windows.
    const int G = (nframes % 8 == 0 && gridDim.x % 8 == 0) ? 8 : 1;
    const int grp = static_cast<int>(blockIdx.x) % G;
    const int gb = static_cast<int>(blockIdx.x) / G, gstride = static_cast<int>(gridDim.x) / G;
    const int t = threadIdx.x;
    const int wid = t >> 6;   // wavefront index in the workgroup
    if (t == 0) {
        int acc = 0, m = 0;
        for (int f = grp; f < nframes; f += G, ++m) {
            owned[m] = f;
            prefix[m] = acc;
            const int kf = step - frames.f[f].k_base;   // this frame's wave
            acc += (kf >= 0 && kf <= frames.f[f].kmax) ? frames.f[f].counts[kf] : 0;
        }
        owned[kMaxFrames] = m;
        prefix[m] = acc;
    }
    __syncthreads();
    const int nown = __builtin_amdgcn_readfirstlane(owned[kMaxFrames]);
    const int total = __builtin_amdgcn_readfirstlane(prefix[nown]);
    if (gb >= total) return;
    int parity = 0;

    for (int gi = gb; gi < total; gi += gstride) {
        int m = 0;
        while (m + 1 < nown && prefix[m + 1] <= gi) ++m;
        m = __builtin_amdgcn_readfirstlane(m);
        const int f = __builtin_amdgcn_readfirstlane(owned[m]);
        const WaveFrame &F = frames.f[f];
        const RefView R = *F.ref;                 // this frame's reference (uniform loads)
        const int k = step - F.k_base;            // this frame's wave
        const int ts = R.ts, lp = R.lp, half = R.half;
        const int N = R.N, h = (N - 1) / 2, n = N * N;
        const double inv_n = R.inv_n;
        const int64_t nn = R.nodes;
        const Columns L(t, T, N);
        const float dxf = static_cast<float>(L.c - h);
        const float dy0 = static_cast<float>(L.r0 - h), dyR = static_cast<float>(L.R);
        const int li = __builtin_amdgcn_readfirstlane(gi - prefix[m]);
        const int32_t *lin = (k & 1) ? F.list1 : F.list0;
        int32_t *lout = (k & 1) ? F.list0 : F.list1;
        const int node = __builtin_amdgcn_readfirstlane(lin[li]);
        const int ix = node % R.nx, iy = node / R.nx;
        const int xc = h + ix * R.step, yc = h + iy * R.step;

        // ---- the subset's metadata: flag, parent key, the four possible parents'
        // parameters (the key selects one; reading all four saves a dependent round
        // trip) and the reference cache.  Small register blocks take the parents'
        // parameters straight into LDS and load the reference pixels afterwards, which
        // keeps them at three wavefronts per SIMD; the 16-row block (two wavefronts
        // either way) requests everything at once into registers.
        constexpr bool kQaInLds = P <= 12;
        const int8_t rf = R.flag[node];
        const uint64_t key = k > 0 ? F.pkey[node] : 0;
        float qr[kQaInLds ? 1 : 4][NP];
        if constexpr (!kQaInLds) {
            if (k > 0) {
                const int64_t nb[4] = {static_cast<int64_t>(iy) * R.nx + max(ix - 1, 0),
                                       static_cast<int64_t>(iy) * R.nx + min(ix + 1, R.nx - 1),
                                       static_cast<int64_t>(max(iy - 1, 0)) * R.nx + ix,
                                       static_cast<int64_t>(min(iy + 1, R.ny - 1)) * R.nx + ix};
#pragma unroll
                for (int d = 0; d < 4; ++d)
#pragma unroll
                    for (int j = 0; j < NP; ++j) qr[d][j] = F.p[j * nn + nb[d]];
            }
        }
        __syncthreads();   // the previous subset is done with the LDS cache and window
        if constexpr (kQaInLds) {
            if (k > 0 && t < 4 * NP) {
                const int dd = t / NP, j = t - dd * NP;
                const int64_t nb = dd == 0 ? static_cast<int64_t>(iy) * R.nx + max(ix - 1, 0)
                                 : dd == 1 ? static_cast<int64_t>(iy) * R.nx + min(ix + 1, R.nx - 1)
                                 : dd == 2 ? static_cast<int64_t>(max(iy - 1, 0)) * R.nx + ix
                                           : static_cast<int64_t>(min(iy + 1, R.ny - 1)) * R.nx + ix;
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(F.p + j * nn + nb),
                    (__attribute__((address_space(3))) void *)(qa), 4, 0, 0);
            }
        }
        for (int q = t; q < NC; q += T) cache[q] = R.cache[static_cast<int64_t>(node) * NC + q];
        if constexpr (kQaInLds) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();   // metadata visible to every wavefront
        }
        // rows per thread of this subset (a launch may mix subset sizes, P is the
        // largest); uniform across the workgroup
        const int JM = __builtin_amdgcn_readfirstlane((N + L.R - 1) / L.R);
        // reference intensities and gradients, interleaved per pixel, so one 12-byte
        // load per row brings all three.  Row j of every thread lies at the uniform
        // address of subset row R j plus a fixed per-thread byte offset, so the loads
        // take a scalar base and no vector address arithmetic.  Threads past
        // the subset's rows (the last row of some threads, all rows of the spare
        // threads) read a row inside the subset instead; the pixel loop weights those
        // entries by zero.
        float fb[P], gx[P], gy[P];
        {
            const int64_t top = static_cast<int64_t>(yc - h) * R.ppitch + (xc - h);
            const int rown = L.jmax > 0 ? L.r0 : 0;
            const int rlast = min(rown + L.R * (JM - 1), N - 1) - L.R * (JM - 1);
            const int lo = 12 * (rown * static_cast<int>(R.ppitch) + L.c);
            const int lo_last = 12 * (rlast * static_cast<int>(R.ppitch) + L.c);
            const int rsb = 12 * L.R * static_cast<int>(R.ppitch);
            const __amdgpu_buffer_rsrc_t ba =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(R.pa + 3 * top), 0, 0x7fffffff, kBufferWord3);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                if (j < JM) {
                    int o = j < JM - 1 ? lo : lo_last;
                    // opaque to the optimiser, so that +4 and +8 stay constant offsets of
                    // one address and the three loads merge into one 12-byte load
                    asm volatile("" : "+v"(o));
                    fb[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ba, o, j * rsb, 0));
                    gx[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ba, o + 4, j * rsb, 0));
                    gy[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ba, o + 8, j * rsb, 0));
                } else {
                    fb[j] = gx[j] = gy[j] = 0.0f;
                }
            }
        }
        if constexpr (!kQaInLds) __syncthreads();   // cache visible to every wavefront

        // ---- initial guess
        double p[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) p[j] = 0.0;
        if (k == 0) {
            p[0] = F.seed_p[2 * li];
            p[1] = F.seed_p[2 * li + 1];
        } else {
            const uint32_t dir = static_cast<uint32_t>(key & 3u);
            // priority 3: parent on the left, 2: right, 1: above, 0: below
            const int px = ix + (dir == 3 ? -1 : (dir == 2 ? 1 : 0));
            const int py = iy + (dir == 1 ? -1 : (dir == 0 ? 1 : 0));
            const int sel = dir == 3 ? 0 : (dir == 2 ? 1 : (dir == 1 ? 2 : 3));
            double q[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                if constexpr (kQaInLds)
                    q[j] = static_cast<double>(qa[sel * NP + j]);
                else
                    q[j] = static_cast<double>(sel == 0 ? qr[0][j] : (sel == 1 ? qr[1][j] : (sel == 2 ? qr[2][j] : qr[3][j])));
            }
#pragma unroll
            for (int j = 0; j < NP; ++j) p[j] = q[j];
            if (!R.guess_copy) {
                const double ex = static_cast<double>((ix - px) * R.step);
                const double ey = static_cast<double>((iy - py) * R.step);
                p[0] = q[0] + q[2] * ex + q[3] * ey;
                p[1] = q[1] + q[4] * ex + q[5] * ey;
                if constexpr (NP == 12) {
                    p[0] += q[6] * ex * ex + q[7] * ex * ey + q[8] * ey * ey;
                    p[1] += q[9] * ex * ex + q[10] * ex * ey + q[11] * ey * ey;
                    p[2] = q[2] + 2.0 * q[6] * ex + q[7] * ey;
                    p[3] = q[3] + q[7] * ex + 2.0 * q[8] * ey;
                    p[4] = q[4] + 2.0 * q[9] * ex + q[10] * ey;
                    p[5] = q[5] + q[10] * ex + 2.0 * q[11] * ey;
                }
            }
        }

        int status = kMaxIter;
        int iters = 0;
        float zncc_out = 0.0f;
        if (rf != 0) {
            status = rf;
        } else {
            const float fm32 = static_cast<float>(cache[0]);
#pragma unroll
            for (int j = 0; j < P; ++j)
                if (j < JM) fb[j] -= fm32;
            const double hd = static_cast<double>(h);
            int tox = INT_MIN / 2, toy = INT_MIN / 2;   // staged window origin (global sample coords)

            for (int it = 1; it <= R.max_iter; ++it) {
                iters = it;
                // ---- bounding box of the warped subset (exact for affine: its corners)
                double xmin, xmax, ymin, ymax;
                {
                    const double ux = (1.0 + p[2]) * hd, uy = p[3] * hd;
                    const double vx = p[4] * hd, vy = (1.0 + p[5]) * hd;
                    const double cx = xc + p[0], cy = yc + p[1];
                    const double rx = fabs(ux) + fabs(uy), ry = fabs(vx) + fabs(vy);
                    xmin = cx - rx; xmax = cx + rx; ymin = cy - ry; ymax = cy + ry;
                    if constexpr (NP == 12) {
                        const double qx = (fabs(p[6]) + fabs(p[7]) + fabs(p[8])) * hd * hd;
                        const double qy = (fabs(p[9]) + fabs(p[10]) + fabs(p[11])) * hd * hd;
                        xmin -= qx; xmax += qx; ymin -= qy; ymax += qy;
                    }
                }
                if (isnan(xmin + xmax + ymin + ymax)) { status = kNan; break; }
                if (!(xmin >= 0.0 && xmax <= R.W - 1.0 && ymin >= 0.0 && ymax <= R.H - 1.0)) {
                    bool oob = true;
                    if constexpr (NP == 12) {
                        // the box is conservative for the quadratic shape: check every point
                        int any = 0;
#pragma unroll 1
                        for (int j = 0; j < P; ++j) {
                            if (j < L.jmax) {
                                const double dx = dxf, dy = static_cast<double>(L.r0 - h + L.R * j);
                                const double X = xc + dx + p[0] + p[2] * dx + p[3] * dy + p[6] * dx * dx +
                                                 p[7] * dx * dy + p[8] * dy * dy;
                                const double Y = yc + dy + p[1] + p[4] * dx + p[5] * dy + p[9] * dx * dx +
                                                 p[10] * dx * dy + p[11] * dy * dy;
                                any |= !(X >= 0.0 && X <= R.W - 1.0 && Y >= 0.0 && Y <= R.H - 1.0);
                            }
                        }
                        oob = __syncthreads_or(any) != 0;
                        // the exact extent is still within the image: use a box clipped to it
                        xmin = fmax(xmin, 0.0); ymin = fmax(ymin, 0.0);
                        xmax = fmin(xmax, R.W - 1.0); ymax = fmin(ymax, R.H - 1.0);
                    }
                    if (oob) { status = kOutOfBounds; zncc_out = 0.0f; break; }
                }
                // ---- deformed coefficients: LDS window if the taps fit, else global
                // taps of every warped point; the 1e-3 px slack covers the FP32 rounding of
                // the per-pixel coordinates (far below it) so no tap leaves the window
                const int tx0 = static_cast<int>(floor(xmin - 1e-3)) - 1, tx1 = static_cast<int>(floor(xmax + 1e-3)) + 2;
                const int ty0 = static_cast<int>(floor(ymin - 1e-3)) - 1, ty1 = static_cast<int>(floor(ymax + 1e-3)) + 2;
                const bool fits = (tx1 - tx0 < ts) && (ty1 - ty0 < ts) && (R.W + 2 * kPad >= ts) &&
                                  (R.H + 2 * kPad >= ts);
                if (fits && !(tx0 >= tox && tx1 < tox + ts && ty0 >= toy && ty1 < toy + ts)) {
                    // split the spare room evenly: the window covers [tx0, tx1] x [ty0, ty1]
                    int ox = tx0 - (ts - (tx1 - tx0 + 1)) / 2;
                    int oy = ty0 - (ts - (ty1 - ty0 + 1)) / 2;
                    ox = max(-kPad, min(ox, R.W + kPad - ts));
                    oy = max(-kPad, min(oy, R.H + kPad - ts));
                    tox = ox;
                    toy = oy;
                    __syncthreads();   // previous window no longer read
                    if (!half) {
                        // one buffer request per window row (and 64-column segment),
                        // straight into LDS: the descriptor holds the window origin, the
                        // row offset and the LDS destination are uniform and step in
                        // scalar registers, and a lane's column offset stays fixed, so
                        // the loop issues no vector instruction (row offsets fit 32 bits:
                        // the set-up bounds the row pitch)
                        const int lane = t & 63;
                        const int nw = T / 64;
                        const int w0 = __builtin_amdgcn_readfirstlane(wid);
                        const int oxu = __builtin_amdgcn_readfirstlane(ox);
                        const int oyu = __builtin_amdgcn_readfirstlane(oy);
                        const int64_t dpitch = F.dpitch;
                        const float *origin = static_cast<const float *>(F.dcoef) + static_cast<int64_t>(oyu) * dpitch + oxu;
                        const __amdgpu_buffer_rsrc_t win =
                            __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(origin), 0, 0x7fffffff, kBufferWord3);
                        const int rstride = static_cast<int>(4 * nw * dpitch);
                        for (int c0 = 0; c0 < ts; c0 += 64) {
                            if (lane < ts - c0) {
                                const int vo = 4 * (c0 + lane);
                                int so = static_cast<int>(4 * w0 * dpitch);
                                float *d = tile + w0 * lp + c0;
                                for (int r = w0; r < ts; r += nw) {
                                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                        win, (__attribute__((address_space(3))) void *)(d), 4, vo, so, 0, 0);
                                    so += rstride;
                                    d += nw * lp;
                                }
                            }
                        }
                        __builtin_amdgcn_s_waitcnt(0);
                    } else {
                        // FP16 storage: widen to FP32 on the way into LDS
                        const int dr = T / ts, dc = T - (T / ts) * ts;
                        int r = t / ts, c = t - (t / ts) * ts;
                        for (int e = t; e < ts * ts; e += T) {
                            const int64_t go = static_cast<int64_t>(oy + r) * F.dpitch + (ox + c);
                            tile[r * lp + c] = to_f32(static_cast<const __half *>(F.dcoef)[go]);
                            r += dr;
                            c += dc;
                            if (c >= ts) {
                                c -= ts;
                                ++r;
                            }
                        }
                    }
                    __syncthreads();
                }
                // local frame: LDS window origin, or a point near the subset for global reads
                const int ox = fits ? tox : static_cast<int>(floor(xc + p[0])) - h - 4;
                const int oy = fits ? toy : static_cast<int>(floor(yc + p[1])) - h - 4;
                const float A0 = static_cast<float>(static_cast<double>(xc - ox) + p[0]);
                const float A1 = static_cast<float>(1.0 + p[2]);
                const float A2 = static_cast<float>(p[3]);
                const float B0 = static_cast<float>(static_cast<double>(yc - oy) + p[1]);
                const float B1 = static_cast<float>(p[4]);
                const float B2 = static_cast<float>(1.0 + p[5]);
                float Q[6];
                if constexpr (NP == 12) {
#pragma unroll
                    for (int q = 0; q < 6; ++q) Q[q] = static_cast<float>(p[6 + q]);
                }
                float s[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) s[i] = 0.0f;
                if (fits) {
                    // LDS window, branch-free: an entry past this thread's rows samples
                    // the subset's last row in its column (inside the window) and is
                    // weighted by zero, so every lane runs the same instruction stream
                    const float dyl = static_cast<float>(N - 1 - h);
                    const float Xc = fmaf(A1, dxf, A0), Yc = fmaf(B1, dxf, B0);
                    const float *tb = tile - lp - 1;
                    const float tsf = static_cast<float>(lp);
                    auto pixel_row = [&](int j) {
                        const bool on = j < L.jmax;
                        const float dy = on ? fmaf(static_cast<float>(j), dyR, dy0) : dyl;
                        float X = fmaf(A2, dy, Xc);
                        float Y = fmaf(B2, dy, Yc);
                        if constexpr (NP == 12) {
                            const float xx = dxf * dxf, xy = dxf * dy, yy = dy * dy;
                            X = fmaf(Q[2], yy, fmaf(Q[1], xy, fmaf(Q[0], xx, X)));
                            Y = fmaf(Q[5], yy, fmaf(Q[4], xy, fmaf(Q[3], xx, Y)));
                        }
                        const float fx0 = floorf(X), fy0 = floorf(Y);
                        float wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3;
                        bspline_w(X - fx0, wx0, wx1, wx2, wx3);
                        bspline_w(Y - fy0, wy0, wy1, wy2, wy3);
                        // tap offset in the window: exact in FP32 (|values| < 2^24), which
                        // avoids a quarter-rate integer multiply per pixel
                        const int off = static_cast<int>(fmaf(fy0, tsf, fx0));
                        const float g = interp16(tb + off, lp, wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3);
                        // a weight rather than a select: the row is then computed on every
                        // lane instead of under a branch, which keeps the rows in one block
                        accumulate<NP>(s, (g - fm32) * (on ? 1.0f : 0.0f), fb[j], gx[j], gy[j], dy);
                    };
                    if (kPipelineRows<P>() && JM == P) {
                        // every row of the register block is in use (the usual case): one
                        // straight-line block, software-pipelined by a row: the 16 window
                        // reads of row j+1 are issued before row j is computed, so their
                        // latency hides behind that arithmetic
                        float tap[2][16], frx[2], fry[2], dyv[2];
                        auto fetch_row = [&](int j, int b) {
                            const bool on = j < L.jmax;
                            const float dy = on ? fmaf(static_cast<float>(j), dyR, dy0) : dyl;
                            float X = fmaf(A2, dy, Xc);
                            float Y = fmaf(B2, dy, Yc);
                            if constexpr (NP == 12) {
                                const float xx = dxf * dxf, xy = dxf * dy, yy = dy * dy;
                                X = fmaf(Q[2], yy, fmaf(Q[1], xy, fmaf(Q[0], xx, X)));
                                Y = fmaf(Q[5], yy, fmaf(Q[4], xy, fmaf(Q[3], xx, Y)));
                            }
                            const float fx0 = floorf(X), fy0 = floorf(Y);
                            frx[b] = X - fx0;
                            fry[b] = Y - fy0;
                            dyv[b] = dy;
                            const float *q = tb + static_cast<int>(fmaf(fy0, tsf, fx0));
#pragma unroll
                            for (int r = 0; r < 4; ++r)
#pragma unroll
                                for (int c = 0; c < 4; ++c) tap[b][4 * r + c] = q[r * lp + c];
                        };
                        fetch_row(0, 0);
#pragma unroll
                        for (int j = 0; j < P; ++j) {
                            const int b = j & 1;
                            if (j + 1 < P) fetch_row(j + 1, b ^ 1);
                            float wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3;
                            bspline_w(frx[b], wx0, wx1, wx2, wx3);
                            bspline_w(fry[b], wy0, wy1, wy2, wy3);
                            const float *v = tap[b];
                            const float r0 = fmaf(wx3, v[3], fmaf(wx2, v[2], fmaf(wx1, v[1], wx0 * v[0])));
                            const float r1 = fmaf(wx3, v[7], fmaf(wx2, v[6], fmaf(wx1, v[5], wx0 * v[4])));
                            const float r2 = fmaf(wx3, v[11], fmaf(wx2, v[10], fmaf(wx1, v[9], wx0 * v[8])));
                            const float r3 = fmaf(wx3, v[15], fmaf(wx2, v[14], fmaf(wx1, v[13], wx0 * v[12])));
                            const float g = fmaf(wy3, r3, fmaf(wy2, r2, fmaf(wy1, r1, wy0 * r0)));
                            const bool on = j < L.jmax;
                            accumulate<NP>(s, (g - fm32) * (on ? 1.0f : 0.0f), fb[j], gx[j], gy[j], dyv[b]);
                        }
                    } else if (JM == P) {
#pragma unroll
                        for (int j = 0; j < P; ++j) pixel_row(j);
                    } else {
#pragma unroll
                        for (int j = 0; j < P; ++j)
                            if (j < JM) pixel_row(j);
                    }
                } else {
                    // taps straight from global memory (a window that does not fit)
                    const float X0 = fmaf(A2, dy0, fmaf(A1, dxf, A0)), XR = A2 * dyR;
                    const float Y0 = fmaf(B2, dy0, fmaf(B1, dxf, B0)), YR = B2 * dyR;
                    for (int j = 0; j < L.jmax; ++j) {
                        const float dx = dxf, dy = fmaf(static_cast<float>(j), dyR, dy0);
                        float X = fmaf(static_cast<float>(j), XR, X0);
                        float Y = fmaf(static_cast<float>(j), YR, Y0);
                        if constexpr (NP == 12) {
                            const float xx = dx * dx, xy = dx * dy, yy = dy * dy;
                            X = fmaf(Q[2], yy, fmaf(Q[1], xy, fmaf(Q[0], xx, X)));
                            Y = fmaf(Q[5], yy, fmaf(Q[4], xy, fmaf(Q[3], xx, Y)));
                        }
                        const float fx0 = floorf(X), fy0 = floorf(Y);
                        float wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3;
                        bspline_w(X - fx0, wx0, wx1, wx2, wx3);
                        bspline_w(Y - fy0, wy0, wy1, wy2, wy3);
                        const int ixl = static_cast<int>(fx0) - 1, iyl = static_cast<int>(fy0) - 1;
                        const int64_t go = static_cast<int64_t>(oy + iyl) * F.dpitch + (ox + ixl);
                        float g;
                        if (half)
                            g = interp16(static_cast<const __half *>(F.dcoef) + go, F.dpitch, wx0, wx1, wx2, wx3, wy0,
                                         wy1, wy2, wy3);
                        else
                            g = interp16(static_cast<const float *>(F.dcoef) + go, F.dpitch, wx0, wx1, wx2, wx3, wy0,
                                         wy1, wy2, wy3);
                        float fbj = 0.0f, gxj = 0.0f, gyj = 0.0f;
#pragma unroll
                        for (int q = 0; q < P; ++q)
                            if (q == j) {
                                fbj = fb[q];
                                gxj = gx[q];
                                gyj = gy[q];
                            }
                        accumulate<NP>(s, g - fm32, fbj, gxj, gyj, dy);
                    }
                }
                finish_column<NP>(s, dxf);
                // ---- reduce; the rest of the iteration (checks, increment, composition,
                // convergence) is scalar FP64 work that the first wavefront does alone and
                // publishes through LDS, so the other wavefronts do not repeat it
                Acc v[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) v[i] = static_cast<Acc>(s[i]);
                block_reduce_first<T, NS>(v, red, parity);
                int stop = 0;
                if (wid == 0) {
                    do {
                        const Acc S0 = v[0], S1 = v[1];
                        const Acc gm = S0 * static_cast<Acc>(inv_n);
                        const Acc dg2 = S1 - S0 * gm;
                        if (isnan(static_cast<double>(dg2))) { status = kNan; stop = 1; break; }
                        const double lev = fmax(1.0, fabs(cache[0] + static_cast<double>(gm)));
                        if (static_cast<double>(dg2) <= n * (kFlatRel * lev) * (kFlatRel * lev)) {
                            status = kFlatDef;
                            zncc_out = 0.0f;
                            stop = 1;
                            break;
                        }
                        // The sums cancel in FP64 (or FP32); the ratio df/dg and the ZNCC need
                        // only FP32 accuracy: an FP32 ratio moves b by ~1e-7 of |sum J fbar|,
                        // i.e. the increment by ~1e-8 px.  Equal reference and deformed sums
                        // give ratio 1 and ZNCC 1 exactly.
                        const Acc sfg = v[2] - gm * static_cast<Acc>(cache[2]);
                        const float ratio_f = sqrtf(static_cast<float>(cache[1]) / static_cast<float>(dg2));
                        const float zn = static_cast<float>(sfg) / (static_cast<float>(dg2) * ratio_f);
                        const Acc ratio = static_cast<Acc>(ratio_f);
                        Acc b[NP];
#pragma unroll
                        for (int a = 0; a < NP; ++a)
                            b[a] = static_cast<Acc>(cache[3 + NP + a]) -
                                   ratio * (v[3 + a] - gm * static_cast<Acc>(cache[3 + a]));
                        // up to b, the same expressions as the reference precompute (an
                        // identical subset gives b = 0 exactly); from here on FP64 contraction
                        // is allowed, since b = 0 still gives a zero increment and unchanged p
                        {
#pragma clang fp contract(fast)
                        double dp[NP];
                        if constexpr (T <= 128 || (NP == 12 && F64)) {
                            // lane a < NP forms row a of H^{-1} b (terms in column order) and
                            // the rows are read back from their lanes; the packed upper
                            // triangle holds H[r][c], r <= c, at r NP - r (r - 1) / 2 + c - r
                            const int ra = t < NP ? t : 0;
                            Acc acc = 0;
#pragma unroll
                            for (int c = 0; c < NP; ++c) {
                                const int r0 = min(ra, c), c0 = max(ra, c);
                                const int q = r0 * NP - (r0 * (r0 - 1)) / 2 + c0 - r0;
                                acc += static_cast<Acc>(cache[3 + 2 * NP + q]) * b[c];
                            }
#pragma unroll
                            for (int a = 0; a < NP; ++a) dp[a] = -static_cast<double>(read_lane(acc, a));
                        } else {
                            // every lane forms every row, walking the packed triangle once; the
                            // terms of each row still add in column order, so the result is
                            // bitwise that of the form above (which, at 256 threads, costs the
                            // 8-row affine block its third wavefront per SIMD; the quadratic
                            // blocks with FP64 sums run at most two either way and spill less
                            // with it)
                            int q = 0;
                            Acc acc[NP];
#pragma unroll
                            for (int a = 0; a < NP; ++a) acc[a] = 0;
#pragma unroll
                            for (int a = 0; a < NP; ++a)
#pragma unroll
                                for (int c = a; c < NP; ++c) {
                                    const Acc hv = static_cast<Acc>(cache[3 + 2 * NP + q]);
                                    ++q;
                                    acc[a] += hv * b[c];
                                    if (c != a) acc[c] += hv * b[a];
                                }
#pragma unroll
                            for (int a = 0; a < NP; ++a) dp[a] = -static_cast<double>(acc[a]);
                        }
                        zncc_out = zn;
                        if constexpr (NP == 6) compose_affine(p, dp);
                        else compose_quadratic(p, dp, qwork);
                        double nrm = dp[0] * dp[0] + dp[1] * dp[1];
                        {
                            double s1 = 0.0, s2 = 0.0;
#pragma unroll
                            for (int a = 2; a < 6; ++a) s1 += dp[a] * dp[a];
#pragma unroll
                            for (int a = 6; a < NP; ++a) s2 += dp[a] * dp[a];
                            nrm += hd * hd * s1 + hd * hd * hd * hd * s2;
                        }
                        bool bad = isnan(zn) || isnan(nrm);
#pragma unroll
                        for (int a = 0; a < NP; ++a) bad = bad || isnan(p[a]);
                        if (bad) { status = kNan; stop = 1; break; }
                        if (nrm < R.tol2) {
                            status = zncc_out >= R.zncc_min ? kConverged : kLowZncc;
                            stop = 1;
                        }
                        }
                    } while (false);
                }
                if constexpr (T > 64) {
                    if (t == 0) {
#pragma unroll
                        for (int a = 0; a < NP; ++a) pub_p[a] = p[a];
                        pub_stop = stop;
                    }
                    __syncthreads();
                    if (wid != 0) {
#pragma unroll
                        for (int a = 0; a < NP; ++a) p[a] = pub_p[a];
                        stop = pub_stop;
                    }
                }
                if (stop) break;
            }
        }

        // ---- results (one thread) and propagation (one lane per direction)
        if (t == 0) {
#pragma unroll
            for (int j = 0; j < NP; ++j) F.p[j * nn + node] = static_cast<float>(p[j]);
            F.zncc[node] = zncc_out;
            F.iters[node] = static_cast<int16_t>(iters);
            F.status[node] = static_cast<int8_t>(status);
        }
        if (status == kConverged && t < 64) push_children(F, R, ix, iy, k, zncc_out, lout, t);
    }
}

// ---------------------------------------------------------------------------
// Packed subsets: for small subsets (N <= 16, affine) one wavefront carries
// 64 / LS subsets, LS lanes each (column-per-thread inside its lane group).
// The per-iteration scalar work (reductions, checks, solve, composition) is
// then shared by the subsets of the wavefront instead of repeated per subset.
// The group's sums use the first steps of the wavefront reduction (the lanes
// of one 16- or 32-lane segment), in the same order on the reference side.
// ---------------------------------------------------------------------------
template <int LS, typename V> __device__ __forceinline__ V seg_allreduce(V v)
{
    v += dpp_read<0xB1>(v);
    v += dpp_read<0x4E>(v);
    v += dpp_read<0x141>(v);
    v += dpp_read<0x140>(v);
    if constexpr (LS >= 32) v = pair_sum16(v);
    return v;
}

template <int LS, int P>
__global__ __launch_bounds__(64) void k_ref_nodes_packed(RefView R, double *cache, int8_t *flag)
{
    constexpr int NP = 6, NH = NP * (NP + 1) / 2, NB = NP + NH, G = 64 / LS;
    constexpr int kNC = 3 + 2 * NP + NH;
    const int t = threadIdx.x, g = t / LS, tl = t - g * LS;
    const int N = R.N, h = (N - 1) / 2, n = N * N;
    const Columns L(tl, LS, N);
    const float dxf = static_cast<float>(L.c - h);
    const float dy0 = static_cast<float>(L.r0 - h), dyR = static_cast<float>(L.R);
    const int64_t nn = R.nodes;
    const int64_t rstep = static_cast<int64_t>(L.R) * R.ppitch;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * G; base < nn; base += static_cast<int64_t>(gridDim.x) * G) {
        const int64_t node = base + g;
        const bool valid = node < nn && flag[node] >= 0;
        const int xc = h + static_cast<int>((valid ? node : 0) % R.nx) * R.step;
        const int yc = h + static_cast<int>((valid ? node : 0) / R.nx) * R.step;
        const int64_t o0 = static_cast<int64_t>(yc - h + L.r0) * R.ppitch + xc - h + L.c;
        double sf = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (valid && j < L.jmax) sf += static_cast<double>(R.pa[3 * (o0 + j * rstep)]);
        sf = seg_allreduce<LS>(sf);
        const double fm = sf / n;
        const float fm32 = static_cast<float>(fm);
        float s[3 + NP];
#pragma unroll
        for (int i = 0; i < 3 + NP; ++i) s[i] = 0.0f;
        double vb[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) vb[i] = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (valid && j < L.jmax) {
                const float *a = R.pa + 3 * (o0 + j * rstep);
                const float fb = a[0] - fm32;
                const float gx = a[1], gy = a[2];
                const float dyf = fmaf(static_cast<float>(j), dyR, dy0);
                accumulate<NP>(s, fb, fb, gx, gy, dyf);
                double J[NP];
                steepest<NP>(J, gx, gy, dxf, dyf);
                int q = NP;
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    vb[a] += J[a];
#pragma unroll
                    for (int b = a; b < NP; ++b) {
                        vb[q] = fma(J[a], J[b], vb[q]);
                        ++q;
                    }
                }
            }
        }
        finish_column<NP>(s, dxf);
        double va[3 + NP];
#pragma unroll
        for (int i = 0; i < 3 + NP; ++i) va[i] = seg_allreduce<LS>(static_cast<double>(s[i]));
#pragma unroll
        for (int i = 0; i < NB; ++i) vb[i] = seg_allreduce<LS>(vb[i]);
        if (valid && tl == 0) {
            double *cn = cache + node * kNC;
            cn[0] = fm;
            cn[1] = va[1];
            cn[2] = va[0];
#pragma unroll
            for (int a = 0; a < NP; ++a) cn[3 + NP + a] = va[3 + a];
#pragma unroll
            for (int i = 0; i < NB; ++i) cn[slot_b<NP>(i)] = vb[i];
        }
    }
}

template <int LS, int P, bool F64>
__global__ __launch_bounds__(64) void k_wave_packed(const FrameTable frames, int step)
{
    using Acc = typename std::conditional<F64, double, float>::type;
    constexpr int NP = 6, NS = 3 + NP, NH = NP * (NP + 1) / 2, NC = 3 + 2 * NP + NH, G = 64 / LS;
    extern __shared__ float tiles[];   // G windows of ts * ts deformed coefficients
    __shared__ double cache[G][NC];
    __shared__ int prefix[kMaxFrames + 1];
    __shared__ int owned[kMaxFrames + 1];
    __shared__ int cnt[kMaxFrames];
    const int nframes = frames.n;
    // frame affinity as in k_wave; the work items are slots of G subsets of one frame
    const int XG = (nframes % 8 == 0 && gridDim.x % 8 == 0) ? 8 : 1;
    const int grp = static_cast<int>(blockIdx.x) % XG;
    const int gb = static_cast<int>(blockIdx.x) / XG, gstride = static_cast<int>(gridDim.x) / XG;
    const int t = threadIdx.x, g = t / LS, tl = t - g * LS;
    if (t == 0) {
        int acc = 0, m = 0;
        for (int f = grp; f < nframes; f += XG, ++m) {
            owned[m] = f;
            prefix[m] = acc;
            const int kf = step - frames.f[f].k_base;
            const int c = (kf >= 0 && kf <= frames.f[f].kmax) ? frames.f[f].counts[kf] : 0;
            cnt[m] = c;
            acc += (c + G - 1) / G;
        }
        owned[kMaxFrames] = m;
        prefix[m] = acc;
    }
    __syncthreads();
    const int nown = __builtin_amdgcn_readfirstlane(owned[kMaxFrames]);
    const int total = __builtin_amdgcn_readfirstlane(prefix[nown]);
    if (gb >= total) return;

    for (int si = gb; si < total; si += gstride) {
        int m = 0;
        while (m + 1 < nown && prefix[m + 1] <= si) ++m;
        m = __builtin_amdgcn_readfirstlane(m);
        const int f = __builtin_amdgcn_readfirstlane(owned[m]);
        const WaveFrame &F = frames.f[f];
        const RefView R = *F.ref;
        const int k = step - F.k_base;
        const int ts = R.ts, half = R.half;
        const int N = R.N, h = (N - 1) / 2, n = N * N;
        const double inv_n = 1.0 / n;
        const int64_t nn = R.nodes;
        const Columns L(tl, LS, N);
        const float dxf = static_cast<float>(L.c - h);
        const float dy0 = static_cast<float>(L.r0 - h), dyR = static_cast<float>(L.R);
        const int li = (si - prefix[m]) * G + g;   // this group's position in the frame's list
        const bool act = li < cnt[m];
        const int32_t *lin = (k & 1) ? F.list1 : F.list0;
        int32_t *lout = (k & 1) ? F.list0 : F.list1;
        const int node = act ? lin[li] : 0;
        const int ix = node % R.nx, iy = node / R.nx;
        const int xc = h + ix * R.step, yc = h + iy * R.step;
        const int8_t rf = act ? R.flag[node] : static_cast<int8_t>(-1);
        const uint64_t key = (act && k > 0) ? F.pkey[node] : 0;
        float qa[4][NP];
        if (act && k > 0) {
            const int64_t nb[4] = {static_cast<int64_t>(iy) * R.nx + max(ix - 1, 0),
                                   static_cast<int64_t>(iy) * R.nx + min(ix + 1, R.nx - 1),
                                   static_cast<int64_t>(max(iy - 1, 0)) * R.nx + ix,
                                   static_cast<int64_t>(min(iy + 1, R.ny - 1)) * R.nx + ix};
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int j = 0; j < NP; ++j) qa[d][j] = F.p[j * nn + nb[d]];
        }
        __syncthreads();   // the previous slot is done with the LDS cache and windows
        if (act)
            for (int q = tl; q < NC; q += LS) cache[g][q] = R.cache[static_cast<int64_t>(node) * NC + q];
        float fb[P], gx[P], gy[P];
        {
            const int64_t o0 = static_cast<int64_t>(yc - h + L.r0) * R.ppitch + xc - h + L.c;
            const int64_t rs = static_cast<int64_t>(L.R) * R.ppitch;
            const float *a = R.pa + 3 * o0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                fb[j] = gx[j] = gy[j] = 0.0f;
                if (act && j < L.jmax) {
                    fb[j] = a[0];
                    gx[j] = a[1];
                    gy[j] = a[2];
                }
                a += 3 * rs;
            }
        }
        double p[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) p[j] = 0.0;
        if (act && k == 0) {
            p[0] = F.seed_p[2 * li];
            p[1] = F.seed_p[2 * li + 1];
        } else if (act) {
            const uint32_t dir = static_cast<uint32_t>(key & 3u);
            const int px = ix + (dir == 3 ? -1 : (dir == 2 ? 1 : 0));
            const int py = iy + (dir == 1 ? -1 : (dir == 0 ? 1 : 0));
            const int sel = dir == 3 ? 0 : (dir == 2 ? 1 : (dir == 1 ? 2 : 3));
            double q[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j)
                q[j] = static_cast<double>(sel == 0 ? qa[0][j] : (sel == 1 ? qa[1][j] : (sel == 2 ? qa[2][j] : qa[3][j])));
#pragma unroll
            for (int j = 0; j < NP; ++j) p[j] = q[j];
            if (!R.guess_copy) {
                const double ex = static_cast<double>((ix - px) * R.step);
                const double ey = static_cast<double>((iy - py) * R.step);
                p[0] = q[0] + q[2] * ex + q[3] * ey;
                p[1] = q[1] + q[4] * ex + q[5] * ey;
            }
        }
        __syncthreads();   // caches visible
        int status = act ? (rf != 0 ? static_cast<int>(rf) : kMaxIter) : kMaxIter;
        int iters = 0;
        float zncc_out = 0.0f;
        bool live = act && rf == 0;
        const double *cg = cache[g];
        float *tile = tiles + g * ts * ts;
        const float fm32 = static_cast<float>(cg[0]);
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (live && j < L.jmax) fb[j] -= fm32;
        const double hd = static_cast<double>(h);
        int tox = INT_MIN / 2, toy = INT_MIN / 2;
        for (int it = 1; it <= R.max_iter; ++it) {
            if (__ballot(live) == 0) break;
            bool fits = false;
            int ox = 0, oy = 0;
            if (live) {
                iters = it;
                const double ux = (1.0 + p[2]) * hd, uy = p[3] * hd;
                const double vx = p[4] * hd, vy = (1.0 + p[5]) * hd;
                const double cx = xc + p[0], cy = yc + p[1];
                const double rx = fabs(ux) + fabs(uy), ry = fabs(vx) + fabs(vy);
                const double xmin = cx - rx, xmax = cx + rx, ymin = cy - ry, ymax = cy + ry;
                if (isnan(xmin + xmax + ymin + ymax)) {
                    status = kNan;
                    live = false;
                } else if (!(xmin >= 0.0 && xmax <= R.W - 1.0 && ymin >= 0.0 && ymax <= R.H - 1.0)) {
                    status = kOutOfBounds;
                    zncc_out = 0.0f;
                    live = false;
                } else {
                    const int tx0 = static_cast<int>(floor(xmin - 1e-3)) - 1, tx1 = static_cast<int>(floor(xmax + 1e-3)) + 2;
                    const int ty0 = static_cast<int>(floor(ymin - 1e-3)) - 1, ty1 = static_cast<int>(floor(ymax + 1e-3)) + 2;
                    fits = (tx1 - tx0 < ts) && (ty1 - ty0 < ts) && (R.W + 2 * kPad >= ts) && (R.H + 2 * kPad >= ts);
                    if (fits && !(tx0 >= tox && tx1 < tox + ts && ty0 >= toy && ty1 < toy + ts)) {
                        int nx0 = tx0 - (ts - (tx1 - tx0 + 1)) / 2;
                        int ny0 = ty0 - (ts - (ty1 - ty0 + 1)) / 2;
                        nx0 = max(-kPad, min(nx0, R.W + kPad - ts));
                        ny0 = max(-kPad, min(ny0, R.H + kPad - ts));
                        tox = nx0;
                        toy = ny0;
                        // this group's lanes restage its own window
                        for (int e = tl; e < ts * ts; e += LS) {
                            const int r = e / ts, c = e - r * ts;
                            const int64_t go = static_cast<int64_t>(toy + r) * F.dpitch + (tox + c);
                            tile[e] = half ? to_f32(static_cast<const __half *>(F.dcoef)[go])
                                           : static_cast<const float *>(F.dcoef)[go];
                        }
                    }
                    ox = fits ? tox : static_cast<int>(floor(xc + p[0])) - h - 4;
                    oy = fits ? toy : static_cast<int>(floor(yc + p[1])) - h - 4;
                }
            }
            __syncthreads();   // windows written
            float s[NS];
#pragma unroll
            for (int i = 0; i < NS; ++i) s[i] = 0.0f;
            if (live) {
                const float A0 = static_cast<float>(static_cast<double>(xc - ox) + p[0]);
                const float A1 = static_cast<float>(1.0 + p[2]);
                const float A2 = static_cast<float>(p[3]);
                const float B0 = static_cast<float>(static_cast<double>(yc - oy) + p[1]);
                const float B1 = static_cast<float>(p[4]);
                const float B2 = static_cast<float>(1.0 + p[5]);
                const float X0 = fmaf(A2, dy0, fmaf(A1, dxf, A0)), XR = A2 * dyR;
                const float Y0 = fmaf(B2, dy0, fmaf(B1, dxf, B0)), YR = B2 * dyR;
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    if (j < L.jmax) {
                        const float dy = fmaf(static_cast<float>(j), dyR, dy0);
                        const float X = fmaf(static_cast<float>(j), XR, X0);
                        const float Y = fmaf(static_cast<float>(j), YR, Y0);
                        const float fx0 = floorf(X), fy0 = floorf(Y);
                        float wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3;
                        bspline_w(X - fx0, wx0, wx1, wx2, wx3);
                        bspline_w(Y - fy0, wy0, wy1, wy2, wy3);
                        const int ixl = static_cast<int>(fx0) - 1, iyl = static_cast<int>(fy0) - 1;
                        float gv;
                        if (fits) {
                            gv = interp16(tile + iyl * ts + ixl, ts, wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3);
                        } else {
                            const int64_t go = static_cast<int64_t>(oy + iyl) * F.dpitch + (ox + ixl);
                            gv = half ? interp16(static_cast<const __half *>(F.dcoef) + go, F.dpitch, wx0, wx1, wx2,
                                                 wx3, wy0, wy1, wy2, wy3)
                                      : interp16(static_cast<const float *>(F.dcoef) + go, F.dpitch, wx0, wx1, wx2,
                                                 wx3, wy0, wy1, wy2, wy3);
                        }
                        accumulate<NP>(s, gv - fm32, fb[j], gx[j], gy[j], dy);
                    }
                }
            }
            finish_column<NP>(s, dxf);
            // segmented sums over each group's lanes (every lane takes part)
            Acc v[NS];
#pragma unroll
            for (int i = 0; i < NS; ++i) v[i] = seg_allreduce<LS>(static_cast<Acc>(s[i]));
            if (live) {
                do {
                    const Acc S0 = v[0], S1 = v[1];
                    const Acc gm = S0 * static_cast<Acc>(inv_n);
                    const Acc dg2 = S1 - S0 * gm;
                    if (isnan(static_cast<double>(dg2))) { status = kNan; live = false; break; }
                    const double lev = fmax(1.0, fabs(cg[0] + static_cast<double>(gm)));
                    if (static_cast<double>(dg2) <= n * (kFlatRel * lev) * (kFlatRel * lev)) {
                        status = kFlatDef;
                        zncc_out = 0.0f;
                        live = false;
                        break;
                    }
                    const Acc sfg = v[2] - gm * static_cast<Acc>(cg[2]);
                    const float ratio_f = sqrtf(static_cast<float>(cg[1]) / static_cast<float>(dg2));
                    const float zn = static_cast<float>(sfg) / (static_cast<float>(dg2) * ratio_f);
                    const Acc ratio = static_cast<Acc>(ratio_f);
                    Acc b[NP];
#pragma unroll
                    for (int a = 0; a < NP; ++a)
                        b[a] = static_cast<Acc>(cg[3 + NP + a]) - ratio * (v[3 + a] - gm * static_cast<Acc>(cg[3 + a]));
                    {
#pragma clang fp contract(fast)
                        double dp[NP];
                        {
                            int q = 0;
                            Acc acc[NP];
#pragma unroll
                            for (int a = 0; a < NP; ++a) acc[a] = 0;
#pragma unroll
                            for (int a = 0; a < NP; ++a)
#pragma unroll
                                for (int c = a; c < NP; ++c) {
                                    const Acc hv = static_cast<Acc>(cg[3 + 2 * NP + q]);
                                    ++q;
                                    acc[a] += hv * b[c];
                                    if (c != a) acc[c] += hv * b[a];
                                }
#pragma unroll
                            for (int a = 0; a < NP; ++a) dp[a] = -static_cast<double>(acc[a]);
                        }
                        zncc_out = zn;
                        compose_affine(p, dp);
                        double s1 = 0.0;
#pragma unroll
                        for (int a = 2; a < 6; ++a) s1 += dp[a] * dp[a];
                        const double nrm = dp[0] * dp[0] + dp[1] * dp[1] + hd * hd * s1;
                        bool bad = isnan(zn) || isnan(nrm);
#pragma unroll
                        for (int a = 0; a < NP; ++a) bad = bad || isnan(p[a]);
                        if (bad) { status = kNan; live = false; break; }
                        if (nrm < R.tol2) {
                            status = zncc_out >= R.zncc_min ? kConverged : kLowZncc;
                            live = false;
                        }
                    }
                } while (false);
            }
        }
        if (act && tl == 0) {
#pragma unroll
            for (int j = 0; j < NP; ++j) F.p[j * nn + node] = static_cast<float>(p[j]);
            F.zncc[node] = zncc_out;
            F.iters[node] = static_cast<int16_t>(iters);
            F.status[node] = static_cast<int8_t>(status);
        }
        // propagation: lanes 0..3 of each group visit the group's four neighbours
        int64_t mnb = -1;
        bool inserted = false;
        if (act && status == kConverged && tl < 4) {
            const int cx = ix + (tl == 0 ? 1 : (tl == 1 ? -1 : 0));
            const int cy = iy + (tl == 2 ? 1 : (tl == 3 ? -1 : 0));
            if (cx >= 0 && cy >= 0 && cx < R.nx && cy < R.ny) {
                mnb = static_cast<int64_t>(cy) * R.nx + cx;
                if (R.flag[mnb] >= 0) {
                    const int old = atomicCAS(F.wave + mnb, -1, k + 1);
                    inserted = old == -1;
                    if (old == -1 || old == k + 1)
                        atomicMax(reinterpret_cast<unsigned long long *>(F.pkey + mnb),
                                  static_cast<unsigned long long>(
                                      (static_cast<uint64_t>(ordered_bits(zncc_out)) << 2) | (3u - tl)));
                }
            }
        }
        const uint64_t bal = __ballot(inserted);
        if (bal != 0) {
            int basei = 0;
            if (t == 0) basei = atomicAdd(F.counts + k + 1, __popcll(bal));
            basei = __shfl(basei, 0);
            if (inserted) lout[basei + __popcll(bal & ((1ull << t) - 1))] = static_cast<int32_t>(mnb);
        }
    }
}

template <int LS, int P>
static void wave_packed_inst(const FrameTable &F, int step, bool f64, int max_ts, int grid, hipStream_t s)
{
    const size_t lds = static_cast<size_t>(64 / LS) * max_ts * max_ts * sizeof(float);
    if (f64)
        k_wave_packed<LS, P, true><<<grid, 64, lds, s>>>(F, step);
    else
        k_wave_packed<LS, P, false><<<grid, 64, lds, s>>>(F, step);
}

#define DIC_PACKED_CASES(X) X(16, 8) X(16, 12) X(16, 16) X(32, 2) X(32, 4) X(32, 8)

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int NP, int T, int P>
static void wave_inst(const FrameTable &F, int step, bool f64, int lds_floats, int grid, hipStream_t s)
{
    const size_t lds = static_cast<size_t>(lds_floats) * sizeof(float);
    if (f64)
        k_wave<NP, T, P, true><<<grid, T, lds, s>>>(F, step);
    else
        k_wave<NP, T, P, false><<<grid, T, lds, s>>>(F, step);
}

// Rows per thread for subset size N at T threads (column-per-thread layout,
// R = T div N rows per pass): the smallest supported register block holding
// ceil(N / R) rows; -1 if T < N or none is large enough.  Besides the powers of
// two and 12, the 14-row block at 128 threads and the 11-row block at 256 are
// exact fits for subsets of 41 and 51 pixels (full blocks take the
// software-pipelined pixel loop).
int pixels_per_thread(int N, int T)
{
    if (T < N) return -1;
    const int R = T / N;
    const int need = (N + R - 1) / R;
    const int opts[] = {2, 4, 8, 11, 12, 14, 16};
    for (int o : opts) {
        if ((o == 14 && T != 128) || (o == 11 && T != 256)) continue;
        if (o >= need) return o;
    }
    return -1;
}

#define DIC_TP_CASES(NP, X)                                                                                           \
    X(NP, 64, 4) X(NP, 64, 8) X(NP, 64, 12) X(NP, 64, 16) X(NP, 128, 2) X(NP, 128, 4) X(NP, 128, 8) X(NP, 128, 12)    \
    X(NP, 128, 14) X(NP, 128, 16) X(NP, 256, 2) X(NP, 256, 4) X(NP, 256, 8) X(NP, 256, 11) X(NP, 256, 12)            \
    X(NP, 256, 16)

int tile_side(int N)
{
    // the warped subset, its 4-tap reach (3 samples) and 3 samples of room to drift
    // on each side; a window that no longer holds the taps is restaged, and one the
    // warped subset outgrows sends the subset to the global-memory path
    return N + 9;
}

// One launch for every frame of F at launch step `step`.  All frames must use the
// same shape and threads per subset, and subset sizes whose rows fit the register
// block chosen for N (the largest subset of the launch); the LDS window is sized
// for the largest frame's window side.
bool launch_wave(const FrameTable &F, int step, int np, int N, int tps, bool f64, int max_ts, int lds_floats,
                 int grid, hipStream_t s)
{
    const int P = pixels_per_thread(N, tps);
    if (tps < 64) {
        if (np != 6) return false;
#define X(LS_, P_)                                                                                                    \
    if (tps == LS_ && P == P_) {                                                                                      \
        wave_packed_inst<LS_, P_>(F, step, f64, max_ts, grid, s);                                                     \
        return true;                                                                                                   \
    }
        DIC_PACKED_CASES(X)
#undef X
        return false;
    }
#define X(NP_, T_, P_)                                                                                                \
    if (np == NP_ && tps == T_ && P == P_) {                                                                          \
        wave_inst<NP_, T_, P_>(F, step, f64, lds_floats, grid, s);                                  \
        return true;                                                                                                   \
    }
    DIC_TP_CASES(6, X)
    DIC_TP_CASES(12, X)
#undef X
    return false;
}

// false if no kernel is built for (np, tps, N): nothing is launched then
bool launch_ref_nodes(const RefView &R, int np, int tps, double *cache, int8_t *flag, hipStream_t s)
{
    const int P = pixels_per_thread(R.N, tps);
    if (tps < 64) {
        const int64_t nblk = (R.nodes + 64 / tps - 1) / (64 / tps);
        const unsigned grid = static_cast<unsigned>(nblk < 8192 ? (nblk < 1 ? 1 : nblk) : 8192);
#define X(LS_, P_)                                                                                                    \
    if (np == 6 && tps == LS_ && P == P_) {                                                                           \
        k_ref_nodes_packed<LS_, P_><<<grid, 64, 0, s>>>(R, cache, flag);                                              \
        k_ref_factor<6><<<static_cast<unsigned>((R.nodes + 255) / 256), 256, 0, s>>>(R, cache, flag);               \
        return true;                                                                                                   \
    }
        DIC_PACKED_CASES(X)
#undef X
        return false;
    }
#define X(NP_, T_, P_)                                                                                                \
    if (np == NP_ && tps == T_ && P == P_) {                                                                          \
        ref_nodes_inst<NP_, T_, P_>(R, cache, flag, s);                                                               \
        return true;                                                                                                   \
    }
    DIC_TP_CASES(6, X)
    DIC_TP_CASES(12, X)
#undef X
    return false;
}

bool supported_tps(int N, int tps)
{
    if (tps == 16 || tps == 32) {
        // packed subsets (affine only, checked by the caller)
        const int P = pixels_per_thread(N, tps);
        return tps == 16 ? (P == 8 || P == 12 || P == 16) : (P == 2 || P == 4 || P == 8);
    }
    if (tps != 64 && tps != 128 && tps != 256) return false;
    const int P = pixels_per_thread(N, tps);
    return P > 0 && !(tps == 64 && P < 4);
}

int wave_grid_hint(int np, int tps, int device, int chains)
{
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    // Enough workgroups to keep every SIMD busy.  One launch chain: one-wavefront
    // workgroups 64 per compute unit take about two subsets each of a full 32-frame
    // wave, so their uneven run times even out over many workgroups and no slow one
    // sets the launch time (+2.4 % over 16 with 16 frames per launch, +2.5 % over 32
    // with 32 frames; 128 is no faster).  Two chains: the other chain's launch fills a
    // launch's tail, and 8 per compute unit (all resident from the start, each walking
    // about 8 subsets of a 16-frame wave) is fastest: +4 % over 64, while 4 and 6 leave
    // SIMDs idle (-9 % and -5 %).
    const int per_cu = tps <= 64 ? (chains > 1 ? 8 : 64) : (tps == 128 ? 8 : 4);
    (void)np;
    return cus * per_cu;
}

} // namespace dicmi
