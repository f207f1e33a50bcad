// Device helpers shared by the gfx950 kernel sources: raw pixel loads, the
// scaled cubic B-spline weights and 4x4 interpolation, the ordered key of a
// ZNCC, cross-lane FP64/FP32 sums, the degenerate-case thresholds and the
// inverse-compositional updates of Eq. (5)'s shape functions.
#pragma once

#include "dic_internal.h"

#include <math.h>

// Every multiply-add that should fuse is written as fmaf(); nothing else is
// contracted, so identical expressions give identical bits in every kernel.
#pragma clang fp contract(off)

namespace dicmi {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float load_pixel(const void *base, int64_t pitch_bytes, int pixel, int x, int y)
{
    const char *row = static_cast<const char *>(base) + static_cast<int64_t>(y) * pitch_bytes;
    if (pixel == 0) return static_cast<float>(reinterpret_cast<const uint8_t *>(row)[x]);
    if (pixel == 1) return static_cast<float>(reinterpret_cast<const uint16_t *>(row)[x]);
    return reinterpret_cast<const float *>(row)[x];
}

// whole-sample mirror fold of k onto [0, n)
__device__ __forceinline__ int fold(int k, int n)
{
    if (n == 1) return 0;
    const int P = 2 * n - 2;
    k %= P;
    if (k < 0) k += P;
    return k < n ? k : P - k;
}

// Cubic B-spline weights of taps x0-1 .. x0+2 at fraction t (beta3 sampled at
// t+1, t, t-1, t-2), scaled by 6: (1-t)^3, 4 - 6t^2 + 3t^3, the same polynomial
// at 1-t, and t^3.  The prefilter folds the 1/6 of each axis into the
// coefficients, so the tensor product of the scaled weights with them is the
// interpolant itself; the scaling saves the divisions by 6 and lets the mirror
// symmetry w2(t) = w1(1-t) share the second cubic's form.
__device__ __forceinline__ void bspline_w(float t, float &w0, float &w1, float &w2, float &w3)
{
    const float s = 1.0f - t;
    const float t2 = t * t;
    const float s2 = s * s;
    w0 = s2 * s;
    w1 = fmaf(fmaf(3.0f, t, -6.0f), t2, 4.0f);
    w2 = fmaf(fmaf(3.0f, s, -6.0f), s2, 4.0f);
    w3 = t2 * t;
}

// their derivatives with respect to t, scaled by 6 like the weights
__device__ __forceinline__ void bspline_dw(float t, float &d0, float &d1, float &d2, float &d3)
{
    const float s = 1.0f - t;
    const float t2 = t * t;
    d0 = -3.0f * (s * s);
    d1 = fmaf(9.0f, t2, -12.0f * t);
    d2 = fmaf(-9.0f, t2, fmaf(6.0f, t, 3.0f));
    d3 = 3.0f * t2;
}

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__half v) { return __half2float(v); }

// 4x4 tensor-product interpolation; b points at tap (x0-1, y0-1).
template <typename Ptr>
__device__ __forceinline__ float interp16(Ptr b, int64_t pitch, float x0, float x1, float x2, float x3, float y0,
                                          float y1, float y2, float y3)
{
    const float r0 = fmaf(x3, to_f32(b[3]), fmaf(x2, to_f32(b[2]), fmaf(x1, to_f32(b[1]), x0 * to_f32(b[0]))));
    b += pitch;
    const float r1 = fmaf(x3, to_f32(b[3]), fmaf(x2, to_f32(b[2]), fmaf(x1, to_f32(b[1]), x0 * to_f32(b[0]))));
    b += pitch;
    const float r2 = fmaf(x3, to_f32(b[3]), fmaf(x2, to_f32(b[2]), fmaf(x1, to_f32(b[1]), x0 * to_f32(b[0]))));
    b += pitch;
    const float r3 = fmaf(x3, to_f32(b[3]), fmaf(x2, to_f32(b[2]), fmaf(x1, to_f32(b[1]), x0 * to_f32(b[0]))));
    return fmaf(y3, r3, fmaf(y2, r2, fmaf(y1, r1, y0 * r0)));
}

// Map a ZNCC to an unsigned key whose integer order is the float order.
__device__ __forceinline__ uint32_t ordered_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Value of the lane chosen by DPP control CTRL (quad_perm, row mirrors), per 32-bit half.
// (every control used here has a source lane for every lane and the row and bank
// masks are full, so each lane is written and no previous value needs setting)
template <int CTRL>
__device__ __forceinline__ double dpp_read(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_read(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v + (v of the partner lane) where the partner sits in the other 16-lane row of a row
// pair (permlane16 swap) or in the other 32-lane half (permlane32 swap).  The swap
// returns the even-row (lower-half) value in one result and the odd-row (upper-half)
// value in the other on every lane, so their sum is formed in the same order everywhere.
__device__ __forceinline__ float pair_sum16(float v)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum32(float v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ double pair_sum16(double v)
{
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double pair_sum32(double v)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Sum over the 64 lanes of a wavefront, left in every lane.  Each step adds the value
// of a partner lane under an involution (quad xor 1, quad xor 2, half-row mirror, row
// mirror, row pairs, halves), so both partners form the same sum: every lane ends
// with bitwise the same total.  No LDS traffic.
template <typename V>
__device__ __forceinline__ V wave_allreduce(V v)
{
    v += dpp_read<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_read<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_read<0x141>(v);  // row_half_mirror
    v += dpp_read<0x140>(v);  // row_mirror
    v = pair_sum16(v);
    v = pair_sum32(v);
    return v;
}

// After a permlane32 swap of (a, b), the sum of the two results is a(lane) + a(lane + 32)
// on lanes 0-31 and b(lane - 32) + b(lane) on lanes 32-63;
// the permlane16 form does the same for even and odd 16-lane rows.  One swap and one add
// reduce two values over a lane pair, each kept by one side.
__device__ __forceinline__ float swap_sum32(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(a), __float_as_int(b), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ float swap_sum16(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(a), __float_as_int(b), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ double swap_sum32(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double swap_sum16(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ float read_lane(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ __forceinline__ double read_lane(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l), __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sums over the 64 lanes of a wavefront of NV values at once, left in every lane as
// uniform values.  Halves and then row pairs reduce the values two at a time (value
// 2i kept by the lower half / even rows, 2i+1 by the upper half / odd rows; an odd one
// out is summed on both sides), each 16-lane row then sums its remaining values with
// the four row steps of wave_allreduce, and every total is read from a lane of the
// class that holds it.  About a third of the instructions of NV separate all-reduces;
// the order of the additions is fixed, so equal inputs give bitwise equal totals.
template <int NV, typename V>
__device__ __forceinline__ void wave_allreduce_n(V (&v)[NV])
{
    constexpr int N1 = (NV + 1) / 2, N2 = (N1 + 1) / 2;
    V a[N1];
#pragma unroll
    for (int i = 0; i < NV / 2; ++i) a[i] = swap_sum32(v[2 * i], v[2 * i + 1]);
    if constexpr (NV & 1) a[N1 - 1] = swap_sum32(v[NV - 1], v[NV - 1]);
    V b[N2];
#pragma unroll
    for (int i = 0; i < N1 / 2; ++i) b[i] = swap_sum16(a[2 * i], a[2 * i + 1]);
    if constexpr (N1 & 1) b[N2 - 1] = swap_sum16(a[N1 - 1], a[N1 - 1]);
#pragma unroll
    for (int i = 0; i < N2; ++i) {
        b[i] += dpp_read<0xB1>(b[i]);
        b[i] += dpp_read<0x4E>(b[i]);
        b[i] += dpp_read<0x141>(b[i]);
        b[i] += dpp_read<0x140>(b[i]);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        // value k: step-1 slot k/2 on the half (k odd: upper), step-2 slot k/4 on the
        // row parity (slot k/2 odd: odd rows)
        const int lane = ((k & 1) ? 32 : 0) + (((k >> 1) & 1) ? 16 : 0);
        v[k] = read_lane(b[k >> 2], lane);
    }
}

// Degenerate-case thresholds: a subset is flat when its RMS deviation is below
// 1e-6 of its mean level; a Cholesky pivot is singular below 1e-10 of the
// largest Hessian diagonal, each entry taken in the units of the convergence
// norm (weights 1, h^2, h^4 for translation, gradient and curvature terms).
constexpr double kFlatRel = 1e-6;
constexpr double kSingularRel = 1e-10;

// ---------------------------------------------------------------------------
// Inverse-compositional update p <- p o dp^{-1} (FP64).
// ---------------------------------------------------------------------------
// Affine: with M(q) = [[1+q2, q3, q0], [q4, 1+q5, q1], [0, 0, 1]], the product
// M(p) M(dp)^{-1} written so that every entry is formed from differences
// p_j - dp_j (no "(1 + small) - 1" cancellation; exact when dp = 0).
__device__ __forceinline__ void compose_affine(double (&p)[6], const double (&d)[6])
{
    // contraction is free here: d = 0 leaves p unchanged with or without it
#pragma clang fp contract(fast)
    const double a = 1.0 + d[2], b = d[3], c = d[4], e = 1.0 + d[5];
    const double det = a * e - b * c;
    // the reciprocal scales terms that are differences of order |dp|: FP32 suffices
    const double r = static_cast<double>(1.0f / static_cast<float>(det));
    // translation part of M(dp)^{-1}: -(M2^{-1}) (d0, d1)
    const double tx = (b * d[1] - e * d[0]) * r;
    const double ty = (c * d[0] - a * d[1]) * r;
    const double n2 = (e * (p[2] - d[2]) - c * (p[3] - d[3])) * r;
    const double n3 = ((p[3] - d[3]) + p[3] * d[2] - p[2] * d[3]) * r;
    const double n4 = ((p[4] - d[4]) + p[4] * d[5] - p[5] * d[4]) * r;
    const double n5 = (a * (p[5] - d[5]) - b * (p[4] - d[4])) * r;
    const double n0 = p[0] + (1.0 + p[2]) * tx + p[3] * ty;
    const double n1 = p[1] + p[4] * tx + (1.0 + p[5]) * ty;
    p[0] = n0; p[1] = n1; p[2] = n2; p[3] = n3; p[4] = n4; p[5] = n5;
}

// Quadratic: lift q to the 6x6 matrix Q(q) acting on the monomials
// [dx^2, dx dy, dy^2, dx, dy, 1] (each image monomial truncated at second
// order); the update keeps the X and Y rows of Q(p) Q(dp)^{-1}, found by
// solving Q(dp)^T r = (row of Q(p))^T with partial pivoting.
__device__ __forceinline__ void lift(const double (&q)[12], double (&Q)[6][6])
{
    const double U = q[0], V = q[1], A = 1.0 + q[2], B = q[3], C = q[4], D = 1.0 + q[5];
    const double a0 = q[6], a1 = q[7], a2 = q[8], b0 = q[9], b1 = q[10], b2 = q[11];
    // X^2
    Q[0][0] = A * A + 2.0 * U * a0; Q[0][1] = 2.0 * (A * B + U * a1); Q[0][2] = B * B + 2.0 * U * a2;
    Q[0][3] = 2.0 * U * A; Q[0][4] = 2.0 * U * B; Q[0][5] = U * U;
    // X Y
    Q[1][0] = A * C + U * b0 + V * a0; Q[1][1] = A * D + B * C + U * b1 + V * a1; Q[1][2] = B * D + U * b2 + V * a2;
    Q[1][3] = U * C + V * A; Q[1][4] = U * D + V * B; Q[1][5] = U * V;
    // Y^2
    Q[2][0] = C * C + 2.0 * V * b0; Q[2][1] = 2.0 * (C * D + V * b1); Q[2][2] = D * D + 2.0 * V * b2;
    Q[2][3] = 2.0 * V * C; Q[2][4] = 2.0 * V * D; Q[2][5] = V * V;
    // X, Y, 1
    Q[3][0] = a0; Q[3][1] = a1; Q[3][2] = a2; Q[3][3] = A; Q[3][4] = B; Q[3][5] = U;
    Q[4][0] = b0; Q[4][1] = b1; Q[4][2] = b2; Q[4][3] = C; Q[4][4] = D; Q[4][5] = V;
    Q[5][0] = 0.0; Q[5][1] = 0.0; Q[5][2] = 0.0; Q[5][3] = 0.0; Q[5][4] = 0.0; Q[5][5] = 1.0;
}

// The elimination runs on a 6 x 8 working matrix in LDS (M, 48 doubles, one per
// workgroup): its rows are picked by the pivot search at run time, which in
// registers would force the whole matrix out to scratch memory.
__device__ __forceinline__ void compose_quadratic(double (&p)[12], const double (&d)[12], double *M)
{
    {
        double Qd[6][6];
        lift(d, Qd);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int j = 0; j < 6; ++j) M[i * 8 + j] = Qd[j][i];   // transpose
        }
    }
    // right-hand sides: the X and Y rows of Q(p), i.e. (a0, a1, a2, A, B, U) and
    // (b0, b1, b2, C, D, V) in the monomial order
    M[0 * 8 + 6] = p[6];  M[1 * 8 + 6] = p[7];  M[2 * 8 + 6] = p[8];
    M[3 * 8 + 6] = 1.0 + p[2]; M[4 * 8 + 6] = p[3]; M[5 * 8 + 6] = p[0];
    M[0 * 8 + 7] = p[9];  M[1 * 8 + 7] = p[10]; M[2 * 8 + 7] = p[11];
    M[3 * 8 + 7] = p[4];  M[4 * 8 + 7] = 1.0 + p[5]; M[5 * 8 + 7] = p[1];
#pragma unroll
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = fabs(M[col * 8 + col]);
#pragma unroll
        for (int r = col + 1; r < 6; ++r) {
            const double v = fabs(M[r * 8 + col]);
            if (v > best) { best = v; piv = r; }
        }
        if (piv != col) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double tv = M[col * 8 + k];
                M[col * 8 + k] = M[piv * 8 + k];
                M[piv * 8 + k] = tv;
            }
        }
        const double inv = 1.0 / M[col * 8 + col];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            if (r == col) continue;
            const double fct = M[r * 8 + col] * inv;
#pragma unroll
            for (int k = col; k < 8; ++k) M[r * 8 + k] -= fct * M[col * 8 + k];
        }
    }
    double x[6], y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        x[i] = M[i * 8 + 6] / M[i * 8 + i];
        y[i] = M[i * 8 + 7] / M[i * 8 + i];
    }
    p[0] = x[5]; p[1] = y[5];
    p[2] = x[3] - 1.0; p[3] = x[4];
    p[4] = y[3]; p[5] = y[4] - 1.0;
    p[6] = x[0]; p[7] = x[1]; p[8] = x[2];
    p[9] = y[0]; p[10] = y[1]; p[11] = y[2];
}

// Propagation from a CONVERGED node (ix, iy) of wave k, run by one wavefront
// (lane t of it): lane d < 4 visits the neighbour in direction d (right, left,
// below, above) if it is active; the first visitor claims it for wave k + 1
// and appends it to the next frontier list `lout`, and every visitor of this
// wave raises the child's parent key to (ordered ZNCC << 2 | priority), where
// the priority 3, 2, 1, 0 says that the child sees this node on its left,
// right, above or below: the exact-tie order of the parent rule.
__device__ __forceinline__ void push_children(const WaveFrame &F, const RefView &R, int ix, int iy, int k,
                                              float zncc, int32_t *lout, int t)
{
    int64_t m = -1;
    bool inserted = false;
    if (t < 4) {
        const int cx = ix + (t == 0 ? 1 : (t == 1 ? -1 : 0));
        const int cy = iy + (t == 2 ? 1 : (t == 3 ? -1 : 0));
        if (cx >= 0 && cy >= 0 && cx < R.nx && cy < R.ny) {
            m = static_cast<int64_t>(cy) * R.nx + cx;
            if (R.flag[m] >= 0) {
                const int old = atomicCAS(F.wave + m, -1, k + 1);
                inserted = old == -1;
                if (old == -1 || old == k + 1)
                    atomicMax(reinterpret_cast<unsigned long long *>(F.pkey + m),
                              static_cast<unsigned long long>((static_cast<uint64_t>(ordered_bits(zncc)) << 2) |
                                                              (3u - t)));
            }
        }
    }
    const uint64_t bal = __ballot(inserted);
    if (bal != 0) {
        int base = 0;
        if (t == 0) base = atomicAdd(F.counts + k + 1, __popcll(bal));
        base = __shfl(base, 0);
        if (inserted) lout[base + __popcll(bal & ((1ull << t) - 1))] = static_cast<int32_t>(m);
    }
}

} // namespace dicmi
