// Strain post-processing (paper Sec. 2.3): least-squares polynomial smoothing
// of the displacement over a square window of N x N grid nodes (Eq. (8)-(9)),
// the deformation gradient F = I + grad u at the window centre (Eq. (6)), and
// one of the five strain measures of Sec. 2.3.
//
// On a complete window the basis and the node offsets are the same for every
// node, so the least-squares derivative at the centre is a fixed linear
// combination of the window's values: the host solves the normal equations
// once (FP64) for the weights of d/dx and d/dy, and the kernel applies them.
// One thread per output node; a 16 x 16 block of nodes stages its
// (16 + N - 1)^2 input window of u, v and validity in LDS.  HBM-bound: 9 bytes
// read and 28 written per node.
#include "dic_context.h"

#include <cmath>

using namespace dicmi;

namespace {

constexpr int kStrainMaxWin = 15;
constexpr int kStrainTile = 16;

// Column basis terms at offset (x, y): bilinear [1, x, y, xy]; biquadratic the
// 9-term tensor product [1, x, y, xy, x^2, y^2, x^2 y, x y^2, x^2 y^2].
void basis_terms(int m, double x, double y, double *t)
{
    t[0] = 1.0;
    t[1] = x;
    t[2] = y;
    t[3] = x * y;
    if (m == 9) {
        t[4] = x * x;
        t[5] = y * y;
        t[6] = x * x * y;
        t[7] = x * y * y;
        t[8] = x * x * y * y;
    }
}

// Weights wx, wy [N*N] (row-major window, rows = y) with d/dx u(0,0) = sum wx u
// and d/dy u(0,0) = sum wy u for the least-squares fit: rows 1 and 2 of
// (A^T A)^{-1} A^T, by Gauss-Jordan elimination with partial pivoting on
// [A^T A | e1 e2] (the matrix is symmetric, so its inverse's rows are columns).
bool fit_weights(int N, int step, int m, double *wx, double *wy)
{
    const int r = (N - 1) / 2;
    double G[9][11] = {};
    for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b) {
            double t[9];
            basis_terms(m, static_cast<double>(b) * step, static_cast<double>(a) * step, t);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) G[i][j] += t[i] * t[j];
        }
    for (int i = 0; i < m; ++i) {
        G[i][m] = i == 1 ? 1.0 : 0.0;
        G[i][m + 1] = i == 2 ? 1.0 : 0.0;
    }
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int i = col + 1; i < m; ++i)
            if (std::fabs(G[i][col]) > std::fabs(G[piv][col])) piv = i;
        if (!(std::fabs(G[piv][col]) > 0.0)) return false;
        if (piv != col)
            for (int j = 0; j < m + 2; ++j) std::swap(G[col][j], G[piv][j]);
        const double inv = 1.0 / G[col][col];
        for (int i = 0; i < m; ++i) {
            if (i == col) continue;
            const double f = G[i][col] * inv;
            for (int j = col; j < m + 2; ++j) G[i][j] -= f * G[col][j];
        }
    }
    // z = G^{-1} e1 and G^{-1} e2: the x and y rows of G^{-1} (symmetric)
    double zx[9], zy[9];
    for (int i = 0; i < m; ++i) {
        zx[i] = G[i][m] / G[i][i];
        zy[i] = G[i][m + 1] / G[i][i];
    }
    for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b) {
            double t[9];
            basis_terms(m, static_cast<double>(b) * step, static_cast<double>(a) * step, t);
            double sx = 0.0, sy = 0.0;
            for (int i = 0; i < m; ++i) {
                sx += zx[i] * t[i];
                sy += zy[i] * t[i];
            }
            wx[(a + r) * N + (b + r)] = sx;
            wy[(a + r) * N + (b + r)] = sy;
        }
    return true;
}

// f(C) = alpha I + beta C for a symmetric positive-definite 2x2 C and
// f = ln: beta = (ln l1 - ln l2) / (l1 - l2) = atanh(x) / (x m) with the
// eigenvalues l = m +- r, x = r / m (series for small x), alpha = ln l1 - beta l1.
__device__ void log_spd(double c00, double c01, double c11, double &o00, double &o01, double &o11)
{
    const double m = 0.5 * (c00 + c11), q = 0.5 * (c00 - c11);
    const double r = sqrt(q * q + c01 * c01);
    const double x = r / m;
    const double ax = x < 1e-3 ? 1.0 + x * x * (1.0 / 3.0 + x * x * 0.2) : atanh(x) / x;
    const double beta = ax / m;
    const double l1 = m + r;
    const double alpha = log(l1) - beta * l1;
    o00 = alpha + beta * c00;
    o01 = beta * c01;
    o11 = alpha + beta * c11;
}

// sqrt of a symmetric positive-definite 2x2 matrix: (C + sqrt(det C) I) / sqrt(tr C + 2 sqrt(det C)).
__device__ void sqrt_spd(double c00, double c01, double c11, double &o00, double &o01, double &o11)
{
    const double s = sqrt(c00 * c11 - c01 * c01);
    const double t = 1.0 / sqrt(c00 + c11 + 2.0 * s);
    o00 = (c00 + s) * t;
    o01 = c01 * t;
    o11 = (c11 + s) * t;
}

__global__ __launch_bounds__(kStrainTile *kStrainTile) void k_strain(const float *u, const float *v,
                                                                      const int8_t *status, int nx, int ny, int N,
                                                                      const double *w, int measure, float *Fo,
                                                                      float *eo)
{
    constexpr int TS = kStrainTile + kStrainMaxWin - 1;
    __shared__ float su[TS * TS], sv[TS * TS];
    __shared__ unsigned char sok[TS * TS];
    const int r = (N - 1) / 2, side = kStrainTile + N - 1;
    const int i0 = blockIdx.x * kStrainTile - r, j0 = blockIdx.y * kStrainTile - r;
    const int t = threadIdx.y * kStrainTile + threadIdx.x;
    for (int e = t; e < side * side; e += kStrainTile * kStrainTile) {
        const int a = e / side, b = e - (e / side) * side;
        const int gi = i0 + b, gj = j0 + a;
        float uu = 0.0f, vv = 0.0f;
        unsigned char ok = 0;
        if (gi >= 0 && gj >= 0 && gi < nx && gj < ny) {
            const int64_t o = static_cast<int64_t>(gj) * nx + gi;
            uu = u[o];
            vv = v[o];
            ok = isfinite(uu) && isfinite(vv) && (!status || status[o] == kConverged);
        }
        su[a * TS + b] = uu;
        sv[a * TS + b] = vv;
        sok[a * TS + b] = ok;
    }
    __syncthreads();
    const int i = blockIdx.x * kStrainTile + threadIdx.x, j = blockIdx.y * kStrainTile + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const int64_t nn = static_cast<int64_t>(nx) * ny, o = static_cast<int64_t>(j) * nx + i;
    bool ok = i >= r && j >= r && i < nx - r && j < ny - r;
    double ux = 0.0, uy = 0.0, vx = 0.0, vy = 0.0;
    if (ok) {
        const double *wx = w, *wy = w + N * N;
        for (int a = 0; a < N && ok; ++a) {
            const int row = (threadIdx.y + a) * TS + threadIdx.x;
            for (int b = 0; b < N; ++b) {
                ok = ok && sok[row + b];
                const double uu = su[row + b], vv = sv[row + b];
                const double cx = wx[a * N + b], cy = wy[a * N + b];
                ux = fma(cx, uu, ux);
                uy = fma(cy, uu, uy);
                vx = fma(cx, vv, vx);
                vy = fma(cy, vv, vy);
            }
        }
    }
    if (!ok) {
        const float qn = __int_as_float(0x7fc00000);
        for (int k = 0; k < 4; ++k) Fo[k * nn + o] = qn;
        for (int k = 0; k < 3; ++k) eo[k * nn + o] = qn;
        return;
    }
    const double a = 1.0 + ux, b = uy, c = vx, d = 1.0 + vy;   // F = [[a, b], [c, d]]
    double e00, e01, e11;
    if (measure == DIC_STRAIN_GREEN_LAGRANGE) {
        e00 = 0.5 * (a * a + c * c - 1.0);
        e01 = 0.5 * (a * b + c * d);
        e11 = 0.5 * (b * b + d * d - 1.0);
    } else if (measure == DIC_STRAIN_HENCKY) {
        // ln sqrt(C) = ln(C) / 2, C = F^T F
        log_spd(a * a + c * c, a * b + c * d, b * b + d * d, e00, e01, e11);
        e00 *= 0.5;
        e01 *= 0.5;
        e11 *= 0.5;
    } else if (measure == DIC_STRAIN_EULER_ALMANSI) {
        // (I - B^{-1}) / 2, B = F F^T
        const double b00 = a * a + b * b, b01 = a * c + b * d, b11 = c * c + d * d;
        const double id = 1.0 / (b00 * b11 - b01 * b01);
        e00 = 0.5 * (1.0 - b11 * id);
        e01 = 0.5 * (b01 * id);
        e11 = 0.5 * (1.0 - b00 * id);
    } else if (measure == DIC_STRAIN_BIOT_RIGHT) {
        sqrt_spd(a * a + c * c, a * b + c * d, b * b + d * d, e00, e01, e11);
        e00 -= 1.0;
        e11 -= 1.0;
    } else {
        sqrt_spd(a * a + b * b, a * c + b * d, c * c + d * d, e00, e01, e11);
        e00 -= 1.0;
        e11 -= 1.0;
    }
    Fo[o] = static_cast<float>(a);
    Fo[nn + o] = static_cast<float>(b);
    Fo[2 * nn + o] = static_cast<float>(c);
    Fo[3 * nn + o] = static_cast<float>(d);
    eo[o] = static_cast<float>(e00);
    eo[nn + o] = static_cast<float>(e01);
    eo[2 * nn + o] = static_cast<float>(e11);
}

} // namespace

extern "C" {

int32_t dic_vsg(int32_t window, int32_t step, int32_t subset_size) { return (window - 1) * step + subset_size; }

dic_status dic_strain(dic_ctx *c, const float *u, const float *v, const int8_t *status, int32_t nx, int32_t ny,
                      int32_t step, const dic_strain_params *prm, float *F_out, float *eps_out)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    if (!prm) FAIL(DIC_E_INVAL, "strain params is NULL");
    if (!u || !v || !F_out || !eps_out) FAIL(DIC_E_INVAL, "NULL displacement or output array");
    if (nx < 1 || ny < 1) FAIL(DIC_E_INVAL, "grid %dx%d", nx, ny);
    if (step < 1) FAIL(DIC_E_INVAL, "step %d", step);
    const int N = prm->window;
    if (N < 3 || N > kStrainMaxWin || (N & 1) == 0) FAIL(DIC_E_INVAL, "window %d (odd, 3..%d)", N, kStrainMaxWin);
    if (prm->basis != DIC_STRAIN_BILINEAR && prm->basis != DIC_STRAIN_BIQUADRATIC)
        FAIL(DIC_E_INVAL, "basis %d (4: bilinear, 9: biquadratic)", prm->basis);
    if (prm->measure < DIC_STRAIN_GREEN_LAGRANGE || prm->measure > DIC_STRAIN_BIOT_LEFT)
        FAIL(DIC_E_INVAL, "strain measure %d", prm->measure);
    std::vector<double> w(2 * N * N);
    if (!fit_weights(N, step, prm->basis, w.data(), w.data() + N * N))
        FAIL(DIC_E_INVAL, "the %d-term basis is singular on a %dx%d window", prm->basis, N, N);
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    if (!c->d_strain_w) HIPCHK(hipMalloc(&c->d_strain_w, sizeof(double) * 2 * kStrainMaxWin * kStrainMaxWin));
    HIPCHK(hipMemcpyAsync(c->d_strain_w, w.data(), sizeof(double) * 2 * N * N, hipMemcpyHostToDevice, s));
    dim3 grid((nx + kStrainTile - 1) / kStrainTile, (ny + kStrainTile - 1) / kStrainTile);
    k_strain<<<grid, dim3(kStrainTile, kStrainTile), 0, s>>>(u, v, status, nx, ny, N, c->d_strain_w, prm->measure,
                                                             F_out, eps_out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return DIC_OK;
}

} // extern "C"
