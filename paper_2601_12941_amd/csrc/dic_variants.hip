// Wave kernel of the method's other variants (paper Sec. 2.2): the rigid shape
// function of Eq. (5), the SSD (Eq. (2)) and NSSD (Eq. (3)) costs beside ZNSSD
// (Eq. (4)), and Levenberg-Marquardt damping of the Gauss-Newton step (the
// optimiser the paper names).  The frontier scheduling, seeds, parent rule,
// guess transfer, statuses and result layout are those of the ZNSSD wave
// kernel; what differs is the per-subset arithmetic:
//   * one workgroup of 256 threads per subset, pixels strided over the threads;
//   * the reference side (mean, norms, sum J, sum J J^T, sum J f) is reduced in
//     the subset's prologue (no per-node cache), in FP64;
//   * taps are read straight from the deformed coefficients in global memory
//     (L1/L2 serve the 4x4 neighbourhoods), interpolation and residual terms
//     in FP32, per-thread partial sums in FP32, cross-thread sums in FP64;
//   * the increment solves (H + lambda diag(H)) dp = -b by Cholesky in FP64
//     (lambda = 0: Gauss-Newton) with Marquardt's accept / reject adaptation of
//     lambda; the merit of an evaluation is the convergence norm of the
//     undamped increment there (zero exactly at the inverse-compositional fixed
//     point, which is not exactly the cost's minimiser).
// All sums are taken of values shifted by the reference subset's FP32 mean c:
// f~ = f - c, g~ = g - c, so that 12-bit intensities do not cancel in FP32.
#include "dic_device.h"

#include <climits>

namespace dicmi {

namespace {

constexpr int kVarT = 256;

template <int NV, typename V> __device__ __forceinline__ void var_block_sum(const V *v, double *red, double *out)
{
    // wavefront totals (the values reduced together, as in the tuned kernel), then
    // the 4 wavefront partials summed in a fixed order; `out` (LDS) receives the sums
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double d[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) d[i] = static_cast<double>(v[i]);
    if constexpr (NV == 1) d[0] = wave_allreduce(d[0]);
    else wave_allreduce_n<NV>(d);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[w * NV + i] = d[i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NV; i += kVarT) {
        double acc = red[i];
        for (int ww = 1; ww < kVarT / 64; ++ww) acc += red[ww * NV + i];
        out[i] = acc;
    }
    __syncthreads();
}

// Steepest-descent terms of Eq. (5) at offset (dx, dy) for gradient (gx, gy).
template <int NP, typename T> __device__ __forceinline__ void sd_terms(T (&J)[NP], T gx, T gy, T dx, T dy)
{
    J[0] = gx;
    J[1] = gy;
    if constexpr (NP >= 6) {
        J[2] = gx * dx;
        J[3] = gx * dy;
        J[4] = gy * dx;
        J[5] = gy * dy;
    }
    if constexpr (NP == 12) {
        J[6] = gx * dx * dx;
        J[7] = gx * dx * dy;
        J[8] = gx * dy * dy;
        J[9] = gy * dx * dx;
        J[10] = gy * dx * dy;
        J[11] = gy * dy * dy;
    }
}

// Weights of the convergence norm (translation 1, gradient h^2, curvature h^4).
__device__ __forceinline__ double norm_weight(int j, double h)
{
    return j < 2 ? 1.0 : (j < 6 ? h * h : h * h * h * h);
}

// In-place Cholesky of the NP x NP matrix A (row-major, lower part used) with
// A_jj scaled by (1 + lam); false if a pivot fails `d > thr_j`.
template <int NP> __device__ bool cholesky(double *A, double lam, const double *thr)
{
    for (int j = 0; j < NP; ++j) {
        double d = A[j * NP + j] * (1.0 + lam);
        for (int k = 0; k < j; ++k) d -= A[j * NP + k] * A[j * NP + k];
        if (!(d > thr[j])) return false;
        const double l = sqrt(d);
        A[j * NP + j] = l;
        for (int i = j + 1; i < NP; ++i) {
            double x = A[i * NP + j];
            for (int k = 0; k < j; ++k) x -= A[i * NP + k] * A[j * NP + k];
            A[i * NP + j] = x / l;
        }
    }
    return true;
}

// dp = -(L L^T)^{-1} b with the Cholesky factor L (row-major, lower part)
template <int NP> __device__ void chol_solve(const double *L, const double *b, double *dp)
{
    double y[NP];
    for (int j = 0; j < NP; ++j) {
        double x = -b[j];
        for (int q = 0; q < j; ++q) x -= L[j * NP + q] * y[q];
        y[j] = x / L[j * NP + j];
    }
    for (int j = NP - 1; j >= 0; --j) {
        double x = y[j];
        for (int q = j + 1; q < NP; ++q) x -= L[q * NP + j] * dp[q];
        dp[j] = x / L[j * NP + j];
    }
}

template <int NP>
__global__ __launch_bounds__(kVarT) void k_wave_var(const FrameTable frames, int step)
{
    constexpr int NH = NP * (NP + 1) / 2;
    constexpr int NR = 2 + NP + NH + NP;   // prologue: S f~, S f~^2, S J, S J J^T, S J f~
    constexpr int NI = 3 + NP;             // iteration: S g~, S g~^2, S f~ g~, S J g~
    __shared__ double red[(kVarT / 64) * NR];
    __shared__ double sums[NR];
    __shared__ double isums[NI];
    __shared__ double Hs[NP * NP];         // H (row-major; the reference side)
    __shared__ double LH[NP * NP];         // Cholesky factor of H
    __shared__ double Ls[NP * NP];         // Cholesky work matrix of H + lambda diag H
    __shared__ double qwork[NP == 12 ? 48 : 1];
    __shared__ double pub_p[NP];
    __shared__ double pub_fm;
    __shared__ float pub_z;
    __shared__ int pub_stop, pub_status;
    __shared__ int prefix[kMaxFrames + 1];

    const int t = threadIdx.x;
    const int nframes = frames.n;
    if (t == 0) {
        int acc = 0;
        for (int f = 0; f < nframes; ++f) {
            prefix[f] = acc;
            const int kf = step - frames.f[f].k_base;
            acc += (kf >= 0 && kf <= frames.f[f].kmax) ? frames.f[f].counts[kf] : 0;
        }
        prefix[nframes] = acc;
    }
    __syncthreads();
    const int total = __builtin_amdgcn_readfirstlane(prefix[nframes]);

    for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
        int m = 0;
        while (m + 1 < nframes && prefix[m + 1] <= gi) ++m;
        m = __builtin_amdgcn_readfirstlane(m);
        const WaveFrame &F = frames.f[m];
        const RefView R = *F.ref;
        const int k = step - F.k_base;
        const int N = R.N, h = (N - 1) / 2, n = N * N;
        const double hd = static_cast<double>(h);
        const int64_t nn = R.nodes;
        const int li = __builtin_amdgcn_readfirstlane(gi - prefix[m]);
        const int32_t *lin = (k & 1) ? F.list1 : F.list0;
        int32_t *lout = (k & 1) ? F.list0 : F.list1;
        const int node = __builtin_amdgcn_readfirstlane(lin[li]);
        const int ix = node % R.nx, iy = node / R.nx;
        const int xc = h + ix * R.step, yc = h + iy * R.step;

        // ---- initial guess: the seed's integer shift, or the parent's shape
        // function (Eq. (5)) re-expanded at this node's centre
        double p[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) p[j] = 0.0;
        if (k == 0) {
            p[0] = F.seed_p[2 * li];
            p[1] = F.seed_p[2 * li + 1];
        } else {
            const uint32_t dir = static_cast<uint32_t>(F.pkey[node] & 3u);
            const int px = ix + (dir == 3 ? -1 : (dir == 2 ? 1 : 0));
            const int py = iy + (dir == 1 ? -1 : (dir == 0 ? 1 : 0));
            const int64_t pn = static_cast<int64_t>(py) * R.nx + px;
            double q[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) q[j] = static_cast<double>(F.p[j * nn + pn]);
#pragma unroll
            for (int j = 0; j < NP; ++j) p[j] = q[j];
            if constexpr (NP >= 6) {
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
        }

        // ---- reference side: mean, then the shifted sums
        const int64_t obase = static_cast<int64_t>(yc - h) * R.ppitch + (xc - h);
        {
            double sf = 0.0;
            for (int i = t; i < n; i += kVarT) sf += static_cast<double>(R.pa[3 * (obase + (i / N) * R.ppitch + i % N)]);
            var_block_sum<1>(&sf, red, sums);
        }
        if (t == 0) pub_fm = sums[0] / n;
        __syncthreads();
        const double fm = pub_fm;
        const float c32 = static_cast<float>(fm);
        {
            double v[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) v[i] = 0.0;
            for (int i = t; i < n; i += kVarT) {
                const float *a = R.pa + 3 * (obase + (i / N) * R.ppitch + i % N);
                const double ft = static_cast<double>(a[0] - c32);
                double J[NP];
                sd_terms<NP, double>(J, a[1], a[2], static_cast<double>(i % N - h),
                                     static_cast<double>(i / N - h));
                v[0] += ft;
                v[1] += ft * ft;
                int q = 2 + NP;
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    v[2 + a] += J[a];
#pragma unroll
                    for (int b = a; b < NP; ++b) v[q++] += J[a] * J[b];
                    v[2 + NP + NH + a] += J[a] * ft;
                }
            }
            var_block_sum<NR>(v, red, sums);
        }
        const double S0 = sums[0], S1 = sums[1];
        const double *SJ = sums + 2, *SJJ = sums + 2 + NP, *SJf = sums + 2 + NP + NH;
        const double df2 = S1 - S0 * S0 / n;   // sum of squared deviations from the mean
        int status = kMaxIter, iters = 0;
        float zncc_out = 0.0f;
        if (t == 0) {
            int st = 0;
            const double lev = fmax(1.0, fabs(static_cast<double>(c32) + S0 / n));
            if (isnan(df2)) st = kNan;
            else if (df2 <= n * (kFlatRel * lev) * (kFlatRel * lev)) st = kFlatRef;
            // Gauss-Newton Hessian: mean-centred steepest-descent terms for ZNSSD
            double hmax = 0.0;
            int q = 0;
            for (int a = 0; a < NP; ++a)
                for (int b = a; b < NP; ++b) {
                    double hv = SJJ[q++];
                    if (R.cost == 0) hv -= SJ[a] * SJ[b] / n;
                    Hs[a * NP + b] = hv;
                    Hs[b * NP + a] = hv;
                }
            for (int a = 0; a < NP; ++a) hmax = fmax(hmax, Hs[a * NP + a] / norm_weight(a, hd));
            double thr[NP];
            for (int a = 0; a < NP; ++a) thr[a] = kSingularRel * norm_weight(a, hd) * hmax;
            for (int i = 0; i < NP * NP; ++i) LH[i] = Hs[i];
            if (st == 0 && !cholesky<NP>(LH, 0.0, thr)) st = kSingular;
            pub_status = st;
        }
        __syncthreads();
        if (pub_status != 0) status = pub_status;

        if (status == kMaxIter) {
            // per-thread FP32 window of the iteration: this thread's pixels
            double lam = R.lm_lambda, best = 0.0, p_acc[NP], b_acc[NP];
            float z_acc = 0.0f;
            for (int it = 1; it <= R.max_iter; ++it) {
                iters = it;
                // split p0, p1 into integer and fraction parts so the FP32 local
                // displacement stays small at any image size
                const double fx0 = floor(p[0]), fy0 = floor(p[1]);
                const float U0 = static_cast<float>(p[0] - fx0), V0 = static_cast<float>(p[1] - fy0);
                const int bx = xc + static_cast<int>(fx0), by = yc + static_cast<int>(fy0);
                float pf_[NP];
#pragma unroll
                for (int j = 0; j < NP; ++j) pf_[j] = static_cast<float>(p[j]);
                float v[NI];
#pragma unroll
                for (int i = 0; i < NI; ++i) v[i] = 0.0f;
                int bad = 0;
                for (int i = t; i < n; i += kVarT) {
                    const float dx = static_cast<float>(i % N - h), dy = static_cast<float>(i / N - h);
                    float U = U0, V = V0;
                    if constexpr (NP >= 6) {
                        U = fmaf(pf_[2], dx, fmaf(pf_[3], dy, U));
                        V = fmaf(pf_[4], dx, fmaf(pf_[5], dy, V));
                    }
                    if constexpr (NP == 12) {
                        U = fmaf(pf_[6], dx * dx, fmaf(pf_[7], dx * dy, fmaf(pf_[8], dy * dy, U)));
                        V = fmaf(pf_[9], dx * dx, fmaf(pf_[10], dx * dy, fmaf(pf_[11], dy * dy, V)));
                    }
                    const float fu = floorf(U), fv = floorf(V);
                    const int x0 = bx + (i % N - h) + static_cast<int>(fu);
                    const int y0 = by + (i / N - h) + static_cast<int>(fv);
                    const float tx = U - fu, ty = V - fv;
                    // a warped point outside [0, W-1] x [0, H-1] ends the subset
                    if (!(x0 >= 0 && y0 >= 0 && (x0 < R.W - 1 || (x0 == R.W - 1 && tx == 0.0f)) &&
                          (y0 < R.H - 1 || (y0 == R.H - 1 && ty == 0.0f)))) {
                        bad |= isnan(U) || isnan(V) ? 2 : 1;
                        continue;
                    }
                    float wx0, wx1, wx2, wx3, wy0, wy1, wy2, wy3;
                    bspline_w(tx, wx0, wx1, wx2, wx3);
                    bspline_w(ty, wy0, wy1, wy2, wy3);
                    const int64_t go = static_cast<int64_t>(y0 - 1) * F.dpitch + (x0 - 1);
                    const float g = R.half ? interp16(static_cast<const __half *>(F.dcoef) + go, F.dpitch, wx0, wx1,
                                                      wx2, wx3, wy0, wy1, wy2, wy3)
                                           : interp16(static_cast<const float *>(F.dcoef) + go, F.dpitch, wx0, wx1,
                                                      wx2, wx3, wy0, wy1, wy2, wy3);
                    const float *a = R.pa + 3 * (obase + (i / N) * R.ppitch + i % N);
                    const float ft = a[0] - c32, gt = g - c32;
                    float J[NP];
                    sd_terms<NP, float>(J, a[1], a[2], dx, dy);
                    v[0] += gt;
                    v[1] = fmaf(gt, gt, v[1]);
                    v[2] = fmaf(ft, gt, v[2]);
#pragma unroll
                    for (int a = 0; a < NP; ++a) v[3 + a] = fmaf(J[a], gt, v[3 + a]);
                }
                const int anybad = __syncthreads_or(bad);
                if (anybad) {
                    status = __syncthreads_or(bad & 2) ? kNan : kOutOfBounds;
                    zncc_out = 0.0f;
                    break;
                }
                var_block_sum<NI>(v, red, isums);
                const double *I = isums;
                if (t == 0) {
                    int stop = 0, st = kMaxIter;
                    do {
                        const double Sg = I[0], Sgg = I[1], Sfg = I[2];
                        const double *SJg = I + 3;
                        const double gm = Sg / n;
                        const double dg2 = Sgg - Sg * gm;
                        if (isnan(dg2)) { st = kNan; stop = 1; break; }
                        const double lev = fmax(1.0, fabs(static_cast<double>(c32) + gm));
                        if (dg2 <= n * (kFlatRel * lev) * (kFlatRel * lev)) {
                            st = kFlatDef;
                            zncc_out = 0.0f;
                            stop = 1;
                            break;
                        }
                        const double sfg = Sfg - gm * S0;       // sum (f - f_m)(g - g_m)
                        const double zn = sfg / sqrt(df2 * dg2);
                        double b[NP];
                        if (R.cost == 0) {          // ZNSSD: r = fbar - (|fbar| / |gbar|) gbar
                            const double ratio = sqrt(df2 / dg2);
                            for (int a = 0; a < NP; ++a)
                                b[a] = (SJf[a] - S0 / n * SJ[a]) - ratio * (SJg[a] - gm * SJ[a]);
                        } else if (R.cost == 1) {   // NSSD: r = f - (|f| / |g|) g
                            const double c = static_cast<double>(c32);
                            const double ff = S1 + 2.0 * c * S0 + n * c * c;
                            const double gg = Sgg + 2.0 * c * Sg + n * c * c;
                            const double ratio = sqrt(ff / gg);
                            for (int a = 0; a < NP; ++a) b[a] = (SJf[a] + c * SJ[a]) - ratio * (SJg[a] + c * SJ[a]);
                        } else {                    // SSD: r = f - g
                            for (int a = 0; a < NP; ++a) b[a] = SJf[a] - SJg[a];
                        }
                        float zf = static_cast<float>(zn);
                        double dp[NP];
                        bool damped = false;
                        if (lam > 0.0) {
                            // Marquardt's adaptation, the merit being the undamped
                            // increment's convergence norm at this p
                            chol_solve<NP>(LH, b, dp);
                            double merit = 0.0;
                            for (int a = 0; a < NP; ++a) merit += norm_weight(a, hd) * dp[a] * dp[a];
                            if (it == 1 || merit <= best) {
                                if (it > 1) lam *= 0.1;
                                best = merit;
                                z_acc = zf;
                                for (int a = 0; a < NP; ++a) {
                                    p_acc[a] = p[a];
                                    b_acc[a] = b[a];
                                }
                                damped = !(merit < R.tol2);
                            } else {
                                lam *= 10.0;
                                zf = z_acc;
                                for (int a = 0; a < NP; ++a) {
                                    p[a] = p_acc[a];
                                    b[a] = b_acc[a];
                                }
                                damped = true;
                            }
                        }
                        zncc_out = zf;
                        if (damped) {
                            // (H + lam diag H) dp = -b
                            double thr[NP];
                            for (int a = 0; a < NP; ++a) thr[a] = 0.0;
                            for (int i = 0; i < NP * NP; ++i) Ls[i] = Hs[i];
                            if (!cholesky<NP>(Ls, lam, thr)) { st = kSingular; stop = 1; break; }
                            chol_solve<NP>(Ls, b, dp);
                        } else {
                            chol_solve<NP>(LH, b, dp);
                        }
                        if constexpr (NP == 2) {
                            p[0] -= dp[0];
                            p[1] -= dp[1];
                        } else if constexpr (NP == 6) {
                            compose_affine(p, dp);
                        } else {
                            compose_quadratic(p, dp, qwork);
                        }
                        double nrm = 0.0;
                        for (int a = 0; a < NP; ++a) nrm += norm_weight(a, hd) * dp[a] * dp[a];
                        bool isbad = isnan(zn) || isnan(nrm);
                        for (int a = 0; a < NP; ++a) isbad = isbad || isnan(p[a]);
                        if (isbad) { st = kNan; stop = 1; break; }
                        if (!damped && nrm < R.tol2) {
                            st = zncc_out >= R.zncc_min ? kConverged : kLowZncc;
                            stop = 1;
                        }
                    } while (false);
                    for (int a = 0; a < NP; ++a) pub_p[a] = p[a];
                    pub_stop = stop;
                    pub_status = st;
                    pub_z = zncc_out;
                }
                __syncthreads();
#pragma unroll
                for (int a = 0; a < NP; ++a) p[a] = pub_p[a];
                const int stop = pub_stop;
                status = pub_status;
                zncc_out = pub_z;
                __syncthreads();   // LDS sums and published values are rewritten next iteration
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
        __syncthreads();   // LDS reused by the next subset
    }
}

} // namespace

bool launch_wave_var(const FrameTable &F, int step, int np, int grid, hipStream_t s)
{
    if (np == 2) k_wave_var<2><<<grid, kVarT, 0, s>>>(F, step);
    else if (np == 6) k_wave_var<6><<<grid, kVarT, 0, s>>>(F, step);
    else if (np == 12) k_wave_var<12><<<grid, kVarT, 0, s>>>(F, step);
    else return false;
    return true;
}

} // namespace dicmi
