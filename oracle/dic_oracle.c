/*
 * FP64 reference ("oracle") of reliability-guided local-subset 2D DIC.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, single-threaded
 * definition that the GPU library is checked against.  Only the tests, the
 * package's smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant generator with the GPU path.
 *
 * What it computes (paper: Hirst et al., "Pyvale: a fast, scalable,
 * open-source 2D DIC engine", arXiv 2601.12941):
 *   - cubic B-spline gray-level interpolation ("bicubic b-spline", Sec. 2.2),
 *     coefficients by the exact recursive prefilter with mirror boundaries;
 *   - the ZNSSD cost, Eq. (4), and the rigid / affine / quadratic shape
 *     functions of Eq. (5) with its parameter order p0..p11;
 *   - per-subset minimisation by inverse-compositional Gauss-Newton (the
 *     paper names Levenberg-Marquardt, Sec. 2.2; Gauss-Newton is the
 *     zero-damping case), with the convergence threshold and iteration cap
 *     of Sec. 2.2 / Sec. 4;
 *   - reliability-guided propagation from a seed to 4-neighbours ranked by
 *     the correlation coefficient with a global visited mask (Sec. 2.4 and
 *     the RG schematic figure), in two orders: WAVE (breadth-first frontier
 *     waves, every node of a wave independent) and SEQUENTIAL (one max-heap,
 *     the single-thread case).
 * Readings where the paper is silent are listed in the design notes; each
 * function below states the one it uses.
 *
 * Parity-unpinned parts: iteration counts (path dependent) and which fixed
 * point is reached on ill-posed subsets.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared [-fopenmp]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ST_CONVERGED = 0,
    ST_NOT_REACHED = 1,
    ST_NOT_IN_ROI = 2,
    ST_MAX_ITER = 3,
    ST_LOW_ZNCC = 4,
    ST_OUT_OF_BOUNDS = 5,
    ST_FLAT_REF = 6,
    ST_FLAT_DEF = 7,
    ST_SINGULAR = 8,
    ST_NAN = 9
};

enum { ORDER_WAVE = 0, ORDER_SEQUENTIAL = 1 };
enum { GUESS_EXTRAPOLATE = 0, GUESS_COPY = 1 };
/* cost functions of Sec. 2.2: Eq. (4) (the default), Eq. (3), Eq. (2) */
enum { COST_ZNSSD = 0, COST_NSSD = 1, COST_SSD = 2 };

#define NPMAX 12 /* quadratic shape: p0..p11 */

/* Relative thresholds for the degenerate cases (reading: "flat" is an RMS
 * deviation below 1e-6 of the subset's mean level; "singular" is a Cholesky
 * pivot below 1e-10 of the largest diagonal entry of the Hessian measured in
 * the same units as the convergence norm, i.e. H_jj / s_j with s_j = 1 for
 * p0, p1, h^2 for p2..p5 and h^4 for p6..p11). */
#define FLAT_REL 1e-6
#define SINGULAR_REL 1e-10

/* ------------------------------------------------------------------ */
/* B-spline prefilter and evaluation                                   */
/* ------------------------------------------------------------------ */

/* Whole-sample mirror extension of index k on [0, n): period 2n-2. */
static long mirror_index(long k, long n)
{
    if (n == 1) return 0;
    long P = 2 * n - 2;
    k %= P;
    if (k < 0) k += P;
    return k < n ? k : P - k;
}

/*
 * Interpolation coefficients of one line: solve (c[k-1] + 4c[k] + c[k+1])/6
 * = s[k] for all k with the mirror extension c[-1] = c[1], c[n] = c[n-2].
 * Exact recursive algorithm (Unser 1993): the inverse filter
 * 6/(z + 4 + 1/z) factors into a causal and an anti-causal first-order
 * recursion with pole z1 = sqrt(3) - 2 and gain 6.
 *   causal:      c+[k] = s[k] + z1 c+[k-1],
 *                c+[0] = sum_k z1^k s~[k] / (1 - z1^(2n-2))  (s~ mirrored,
 *                periodic; terms below 1e-300 are dropped: they are zero in
 *                double precision),
 *   anti-causal: c-[k] = z1 (c-[k+1] - c+[k]),
 *                c-[n-1] = z1/(z1^2 - 1) (c+[n-1] + z1 c+[n-2]),
 *   c = 6 c-.
 */
void orc_prefilter_line(double *s, long n, long stride)
{
    if (n < 2) return;
    const double z = sqrt(3.0) - 2.0;
    const long P = 2 * n - 2;
    double acc = 0.0, zk = 1.0;
    for (long k = 0; k < P; ++k) {
        acc += zk * s[mirror_index(k, n) * stride];
        zk *= z;
        if (fabs(zk) < 1e-300) break;
    }
    double zP = pow(z, (double)P);
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    cp[0] = acc / (1.0 - zP);
    for (long k = 1; k < n; ++k) cp[k] = s[k * stride] + z * cp[k - 1];
    double cm = z / (z * z - 1.0) * (cp[n - 1] + z * cp[n - 2]);
    s[(n - 1) * stride] = 6.0 * cm;
    for (long k = n - 2; k >= 0; --k) {
        cm = z * (cm - cp[k]);
        s[k * stride] = 6.0 * cm;
    }
    free(cp);
}

/* Separable 2-D prefilter: rows, then columns.  img, coef: [H][W]. */
void orc_prefilter_2d(const double *img, int W, int H, double *coef)
{
    memcpy(coef, img, sizeof(double) * (size_t)W * (size_t)H);
    for (long y = 0; y < H; ++y) orc_prefilter_line(coef + y * (long)W, W, 1);
    for (long x = 0; x < W; ++x) orc_prefilter_line(coef + x, H, W);
}

/* Cubic B-spline weights for taps x0-1 .. x0+2 at fraction t = x - x0. */
static void bspline_weights(double t, double w[4])
{
    double s = 1.0 - t;
    w[0] = s * s * s / 6.0;
    w[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    w[3] = t * t * t / 6.0;
}

/* d/dt of the weights above. */
static void bspline_dweights(double t, double d[4])
{
    d[0] = -(1.0 - t) * (1.0 - t) / 2.0;
    d[1] = (3.0 * t * t - 4.0 * t) / 2.0;
    d[2] = (-3.0 * t * t + 2.0 * t + 1.0) / 2.0;
    d[3] = t * t / 2.0;
}

/*
 * Value (and, if gx/gy are non-null, the x and y derivatives) of the
 * interpolant sum_{a,b} c[y0-1+a][x0-1+b] w_a(ty) w_b(tx) at (x, y), with
 * mirror indices at the image edges.  Pixel (row i, col j) sits at x=j, y=i.
 */
double orc_eval(const double *c, int W, int H, double x, double y, double *gx, double *gy)
{
    double fx0 = floor(x), fy0 = floor(y);
    long x0 = (long)fx0, y0 = (long)fy0;
    double tx = x - fx0, ty = y - fy0;
    double wx[4], wy[4], dx[4], dy[4];
    bspline_weights(tx, wx);
    bspline_weights(ty, wy);
    bspline_dweights(tx, dx);
    bspline_dweights(ty, dy);
    double v = 0.0, vx = 0.0, vy = 0.0;
    const int grad = gx != NULL || gy != NULL;
    for (int a = 0; a < 4; ++a) {
        long yy = mirror_index(y0 - 1 + a, H);
        for (int b = 0; b < 4; ++b) {
            long xx = mirror_index(x0 - 1 + b, W);
            double cv = c[yy * W + xx];
            v += wy[a] * wx[b] * cv;
            if (grad) {
                vx += wy[a] * dx[b] * cv;
                vy += dy[a] * wx[b] * cv;
            }
        }
    }
    if (gx) *gx = vx;
    if (gy) *gy = vy;
    return v;
}

/* ------------------------------------------------------------------ */
/* Shape functions, Eq. (5)                                            */
/* ------------------------------------------------------------------ */

/* Displacement of local offset (dx, dy) under p (Eq. (5), x and y read as
 * offsets from the subset centre): returns (u, v) so that the warped point is
 * (x_c + dx + u, y_c + dy + v). */
static void shape_disp(const double *p, int np, double dx, double dy, double *u, double *v)
{
    double uu = p[0], vv = p[1];
    if (np >= 6) {
        uu += p[2] * dx + p[3] * dy;
        vv += p[4] * dx + p[5] * dy;
    }
    if (np >= 12) {
        uu += p[6] * dx * dx + p[7] * dx * dy + p[8] * dy * dy;
        vv += p[9] * dx * dx + p[10] * dx * dy + p[11] * dy * dy;
    }
    *u = uu;
    *v = vv;
}

/* Derivative of the warped point with respect to p at p = 0 (the steepest
 * descent directions): row x and row y of dW/dp. */
static void shape_jac(int np, double dx, double dy, double jx[NPMAX], double jy[NPMAX])
{
    memset(jx, 0, sizeof(double) * NPMAX);
    memset(jy, 0, sizeof(double) * NPMAX);
    jx[0] = 1.0;
    jy[1] = 1.0;
    if (np >= 6) {
        jx[2] = dx; jx[3] = dy;
        jy[4] = dx; jy[5] = dy;
    }
    if (np >= 12) {
        jx[6] = dx * dx; jx[7] = dx * dy; jx[8] = dy * dy;
        jy[9] = dx * dx; jy[10] = dx * dy; jy[11] = dy * dy;
    }
}

/* Solve A x = b (n x n, row-major) by Gauss-Jordan elimination with partial
 * pivoting, in place; A is destroyed.  Returns 0 on a zero pivot. */
static int gauss_solve(double *A, double *B, int n, int nrhs)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0) return 0;
        if (piv != col) {
            for (int k = 0; k < n; ++k) { double t = A[col * n + k]; A[col * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            for (int k = 0; k < nrhs; ++k) { double t = B[col * nrhs + k]; B[col * nrhs + k] = B[piv * nrhs + k]; B[piv * nrhs + k] = t; }
        }
        double d = A[col * n + col];
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = A[r * n + col] / d;
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
            for (int k = 0; k < nrhs; ++k) B[r * nrhs + k] -= f * B[col * nrhs + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < nrhs; ++k) B[r * nrhs + k] /= A[r * n + r];
    return 1;
}

/*
 * Lift of a quadratic warp to the 6x6 matrix that maps the monomial vector
 * m = [dx^2, dx dy, dy^2, dx, dy, 1] of a point to that of its image, each
 * entry truncated at second order.  With X = U + A dx + B dy + q_x(dx,dy),
 * Y = V + C dx + D dy + q_y(dx,dy) (A = 1+p2, B = p3, C = p4, D = 1+p5,
 * U = p0, V = p1, q_x = p6 dx^2 + p7 dx dy + p8 dy^2, q_y likewise p9..p11),
 * the rows are X^2, XY, Y^2, X, Y, 1 expanded in m.
 */
static void quad_lift(const double *p, double Q[36])
{
    double U = p[0], V = p[1], A = 1.0 + p[2], B = p[3], C = p[4], D = 1.0 + p[5];
    double a0 = p[6], a1 = p[7], a2 = p[8], b0 = p[9], b1 = p[10], b2 = p[11];
    double r[6][6] = {
        {A * A + 2.0 * U * a0, 2.0 * A * B + 2.0 * U * a1, B * B + 2.0 * U * a2, 2.0 * U * A, 2.0 * U * B, U * U},
        {A * C + U * b0 + V * a0, A * D + B * C + U * b1 + V * a1, B * D + U * b2 + V * a2, U * C + V * A,
         U * D + V * B, U * V},
        {C * C + 2.0 * V * b0, 2.0 * C * D + 2.0 * V * b1, D * D + 2.0 * V * b2, 2.0 * V * C, 2.0 * V * D, V * V},
        {a0, a1, a2, A, B, U},
        {b0, b1, b2, C, D, V},
        {0.0, 0.0, 0.0, 0.0, 0.0, 1.0}};
    memcpy(Q, r, sizeof(r));
}

/*
 * Inverse-compositional update p <- p o dp^{-1}.
 *   rigid:     p - dp;
 *   affine:    M(p) M(dp)^{-1}, M(p) = [[1+p2, p3, p0], [p4, 1+p5, p1], [0,0,1]];
 *   quadratic: Q(p) Q(dp)^{-1} with the lift above, parameters read back
 *              from the X and Y rows.
 * Returns 0 if the increment warp is not invertible.
 */
int orc_compose(const double *p, const double *dp, int np, double *out)
{
    if (np == 2) {
        out[0] = p[0] - dp[0];
        out[1] = p[1] - dp[1];
        return 1;
    }
    if (np == 6) {
        double a = 1.0 + dp[2], b = dp[3], c = dp[4], d = 1.0 + dp[5];
        double det = a * d - b * c;
        if (det == 0.0) return 0;
        /* inverse of [[a, b, e], [c, d, f], [0, 0, 1]] */
        double ia = d / det, ib = -b / det, ic = -c / det, id = a / det;
        double ie = -(ia * dp[0] + ib * dp[1]);
        double iff = -(ic * dp[0] + id * dp[1]);
        double A = 1.0 + p[2], B = p[3], C = p[4], D = 1.0 + p[5];
        double nA = A * ia + B * ic, nB = A * ib + B * id, nE = A * ie + B * iff + p[0];
        double nC = C * ia + D * ic, nD = C * ib + D * id, nF = C * ie + D * iff + p[1];
        out[0] = nE;
        out[1] = nF;
        out[2] = nA - 1.0;
        out[3] = nB;
        out[4] = nC;
        out[5] = nD - 1.0;
        return 1;
    }
    /* quadratic: R = Q(p) Q(dp)^{-1}  <=>  R Q(dp) = Q(p)  <=>  Q(dp)^T R^T = Q(p)^T */
    double Qp[36], Qd[36], At[36], Bt[36];
    quad_lift(p, Qp);
    quad_lift(dp, Qd);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            At[i * 6 + j] = Qd[j * 6 + i];
            Bt[i * 6 + j] = Qp[j * 6 + i];
        }
    if (!gauss_solve(At, Bt, 6, 6)) return 0;
    /* R^T is in Bt: R[i][j] = Bt[j][i]. Row 3 = X, row 4 = Y. */
    double R3[6], R4[6];
    for (int j = 0; j < 6; ++j) {
        R3[j] = Bt[j * 6 + 3];
        R4[j] = Bt[j * 6 + 4];
    }
    out[0] = R3[5];
    out[1] = R4[5];
    out[2] = R3[3] - 1.0;
    out[3] = R3[4];
    out[4] = R4[3];
    out[5] = R4[4] - 1.0;
    out[6] = R3[0];
    out[7] = R3[1];
    out[8] = R3[2];
    out[9] = R4[0];
    out[10] = R4[1];
    out[11] = R4[2];
    return 1;
}

/* ------------------------------------------------------------------ */
/* One subset                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int W, H;
    const double *fc; /* reference coefficients [H][W] */
    const double *gc; /* deformed coefficients  [H][W] */
    const double *fraw, *graw; /* raw pixel values (seed search) */
    int int_pixels; /* raw values are integers: sums are exact in int64 */
    int N, step, np, nx, ny;
    double tol;
    int max_iter;
    double zncc_min;
    int seed_radius;
    int guess_mode;
    int cost;          /* COST_* */
    double lm_lambda;  /* 0: Gauss-Newton; > 0: initial Levenberg-Marquardt damping */
} orc_problem;

typedef struct {
    double p[NPMAX];
    double zncc;
    int iters;
    int status;
} orc_node_result;

/*
 * Convergence norm of an increment (reading: the largest-scale displacement
 * change over the subset): sqrt(dp0^2 + dp1^2 + h^2 sum_{2..5} dpj^2
 * + h^4 sum_{6..11} dpj^2), h = (N-1)/2, in pixels.
 */
static double dp_norm(const double *dp, int np, double h)
{
    double s = dp[0] * dp[0] + dp[1] * dp[1];
    double s1 = 0.0, s2 = 0.0;
    for (int j = 2; j < np && j < 6; ++j) s1 += dp[j] * dp[j];
    for (int j = 6; j < np; ++j) s2 += dp[j] * dp[j];
    return sqrt(s + h * h * s1 + h * h * h * h * s2);
}

/*
 * Inverse-compositional Gauss-Newton on the ZNSSD cost of Eq. (4) for the
 * subset centred at node (xc, yc), starting from p_init.
 *
 * Reference side (fixed over the iterations):
 *   f_i  = reference interpolant at the subset's integer pixels,
 *   f_m  = mean f_i, fbar_i = f_i - f_m, df = sqrt(sum fbar_i^2),
 *   J_i  = grad f_i . dW/dp (Eq. (5) parameter order),
 *   H    = sum J_i^T J_i (uncentred), Cholesky-factorised.
 * Iteration k = 1..max_iter:
 *   1. warp every pixel with p; any point outside [0,W-1]x[0,H-1] -> OUT_OF_BOUNDS;
 *   2. g_i = deformed interpolant at the warped point;
 *   3. g_m = mean g_i, gbar_i = g_i - g_m, dg = sqrt(sum gbar_i^2) (two passes);
 *   4. r_i = fbar_i - (df/dg) gbar_i;
 *   5. ZNSSD = sum r_i^2 / df^2  (= Eq. (4)),  ZNCC = 1 - ZNSSD/2;
 *   6. dp = -H^{-1} sum J_i^T r_i;
 *   7. p <- p o dp^{-1};
 *   8. NaN anywhere -> NAN; |dp| < tol -> converged (LOW_ZNCC if ZNCC < zncc_min).
 * Without convergence after max_iter iterations -> MAX_ITER.
 *
 * Other costs of Sec. 2.2 (same loop, same Gauss-Newton structure):
 *   NSSD, Eq. (3):  r_i = f_i - (|f|/|g|) g_i with |f| = sqrt(sum f_i^2) (no
 *                   mean removed), cost sum r_i^2 / |f|^2, H = sum J_i^T J_i;
 *   SSD,  Eq. (2):  r_i = f_i - g_i, cost sum r_i^2, H = sum J_i^T J_i.
 * The reported coefficient is the ZNCC of step 5 for every cost.
 *
 * Levenberg-Marquardt (Sec. 2.2 names it as the optimiser; Gauss-Newton is
 * its zero-damping case), with lambda > 0: the increment solves
 * (H + lambda diag(H)) dp = -b, and lambda adapts by Marquardt's rule: an
 * evaluation that improves on the last accepted one is accepted and divides
 * lambda by 10; one that does not is rejected: lambda is multiplied by 10 and
 * the step is retaken from the last accepted p and b.  Reading of "improves":
 * the merit is the convergence norm of the undamped Gauss-Newton increment at
 * the evaluated p, zero exactly at the inverse-compositional fixed point.  (The
 * cost itself is not used: that fixed point is not exactly the cost's
 * minimiser, and a cost test makes the iteration cycle between the two points
 * near convergence.)  An accepted evaluation whose merit is below tol takes the
 * undamped step and is CONVERGED; the ZNCC reported is the last accepted one.
 */
void orc_icgn_node(const orc_problem *P, double xc, double yc, const double *p_init, orc_node_result *res)
{
    const int N = P->N, np = P->np, n = N * N;
    const int h = (N - 1) / 2;
    double *fbar = (double *)malloc(sizeof(double) * (size_t)n);
    double *fraw = (double *)malloc(sizeof(double) * (size_t)n);
    double *graw = (double *)malloc(sizeof(double) * (size_t)n);
    double *J = (double *)malloc(sizeof(double) * (size_t)n * NPMAX);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double Hm[NPMAX * NPMAX], L[NPMAX * NPMAX], Ld[NPMAX * NPMAX];
    double p[NPMAX], p_acc[NPMAX], b_acc[NPMAX];
    double lam = P->lm_lambda, best = 0.0, z_acc = 0.0;
    int damped = 0; /* this iteration takes the damped step */
    memset(p, 0, sizeof(p));
    for (int j = 0; j < np; ++j) p[j] = p_init[j];
    res->zncc = 0.0;
    res->iters = 0;

    /* reference subset */
    double fsum = 0.0;
    for (int i = 0; i < n; ++i) {
        int dy = i / N - h, dx = i % N - h;
        double gx, gy;
        fbar[i] = orc_eval(P->fc, P->W, P->H, xc + dx, yc + dy, &gx, &gy);
        fraw[i] = fbar[i];
        fsum += fbar[i];
        double jx[NPMAX], jy[NPMAX];
        shape_jac(np, dx, dy, jx, jy);
        for (int k = 0; k < np; ++k) J[i * NPMAX + k] = gx * jx[k] + gy * jy[k];
    }
    double fm = fsum / n;
    double ss = 0.0;
    for (int i = 0; i < n; ++i) {
        fbar[i] -= fm;
        ss += fbar[i] * fbar[i];
    }
    double df = sqrt(ss);
    if (isnan(df)) { res->status = ST_NAN; goto done; }
    if (ss <= n * (FLAT_REL * fmax(1.0, fabs(fm))) * (FLAT_REL * fmax(1.0, fabs(fm)))) {
        res->status = ST_FLAT_REF;
        goto done;
    }
    /* Gauss-Newton Hessian of the zero-mean criterion: the warped reference
     * subset's mean moves with the increment, so its Jacobian is the
     * mean-centred J.  b = sum J^T r needs no centring because sum r = 0.
     * NSSD and SSD remove no mean: their Hessian is the uncentred sum. */
    double Jm[NPMAX];
    for (int k = 0; k < np; ++k) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += J[i * NPMAX + k];
        Jm[k] = P->cost == COST_ZNSSD ? s / n : 0.0;
    }
    double ff = 0.0; /* |f|^2 of NSSD */
    for (int i = 0; i < n; ++i) ff += fraw[i] * fraw[i];
    for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += (J[i * NPMAX + a] - Jm[a]) * (J[i * NPMAX + b] - Jm[b]);
            Hm[a * np + b] = s;
        }
    /* Cholesky H = L L^T */
    double hs[NPMAX], hmax = 0.0;
    for (int j = 0; j < np; ++j) {
        hs[j] = j < 2 ? 1.0 : (j < 6 ? (double)h * h : (double)h * h * h * h);
        hmax = fmax(hmax, Hm[j * np + j] / hs[j]);
    }
    for (int j = 0; j < np; ++j) {
        double d = Hm[j * np + j];
        for (int k = 0; k < j; ++k) d -= L[j * np + k] * L[j * np + k];
        if (isnan(d)) { res->status = ST_NAN; goto done; }
        if (!(d > SINGULAR_REL * hs[j] * hmax)) { res->status = ST_SINGULAR; goto done; }
        L[j * np + j] = sqrt(d);
        for (int i = j + 1; i < np; ++i) {
            double s = Hm[i * np + j];
            for (int k = 0; k < j; ++k) s -= L[i * np + k] * L[j * np + k];
            L[i * np + j] = s / L[j * np + j];
        }
    }

    for (int it = 1; it <= P->max_iter; ++it) {
        res->iters = it;
        /* 1-2: warp and interpolate */
        for (int i = 0; i < n; ++i) {
            int dy = i / N - h, dx = i % N - h;
            double u, v;
            shape_disp(p, np, dx, dy, &u, &v);
            double x = xc + dx + u, y = yc + dy + v;
            if (!(x >= 0.0 && x <= P->W - 1.0 && y >= 0.0 && y <= P->H - 1.0)) {
                res->status = isnan(x) || isnan(y) ? ST_NAN : ST_OUT_OF_BOUNDS;
                res->zncc = 0.0;
                goto done;
            }
            g[i] = orc_eval(P->gc, P->W, P->H, x, y, NULL, NULL);
        }
        /* 3: two-pass mean and norm */
        double gs = 0.0, gg = 0.0;
        for (int i = 0; i < n; ++i) {
            graw[i] = g[i];
            gs += g[i];
            gg += g[i] * g[i];
        }
        double gm = gs / n;
        double gss = 0.0;
        for (int i = 0; i < n; ++i) {
            g[i] -= gm;
            gss += g[i] * g[i];
        }
        if (isnan(gss)) { res->status = ST_NAN; goto done; }
        if (gss <= n * (FLAT_REL * fmax(1.0, fabs(gm))) * (FLAT_REL * fmax(1.0, fabs(gm)))) {
            res->status = ST_FLAT_DEF;
            res->zncc = 0.0;
            goto done;
        }
        double dg = sqrt(gss);
        /* 4-6 */
        double ratio = df / dg, rr = 0.0, b[NPMAX];
        double nratio = sqrt(ff / gg), cr = 0.0; /* NSSD's |f|/|g|; the chosen cost's sum of r^2 */
        memset(b, 0, sizeof(b));
        for (int i = 0; i < n; ++i) {
            double r = fbar[i] - ratio * g[i];
            rr += r * r;
            if (P->cost == COST_NSSD) r = fraw[i] - nratio * graw[i];
            else if (P->cost == COST_SSD) r = fraw[i] - graw[i];
            cr += r * r;
            for (int k = 0; k < np; ++k) b[k] += J[i * NPMAX + k] * r;
        }
        double znssd = rr / (df * df);
        res->zncc = 1.0 - 0.5 * znssd;
        double y[NPMAX], dp[NPMAX];
        if (lam > 0.0) {
            /* merit: the undamped increment's convergence norm at this p */
            double gd[NPMAX];
            memset(gd, 0, sizeof(gd));
            for (int j = 0; j < np; ++j) {
                double s = b[j];
                for (int k = 0; k < j; ++k) s -= L[j * np + k] * y[k];
                y[j] = s / L[j * np + j];
            }
            for (int j = np - 1; j >= 0; --j) {
                double s = y[j];
                for (int k = j + 1; k < np; ++k) s -= L[k * np + j] * gd[k];
                gd[j] = s / L[j * np + j];
            }
            const double merit = dp_norm(gd, np, h);
            if (it == 1 || merit <= best) {
                if (it > 1) lam *= 0.1;
                best = merit;
                z_acc = res->zncc;
                memcpy(p_acc, p, sizeof(p));
                memcpy(b_acc, b, sizeof(b));
                damped = !(merit < P->tol);
            } else {
                lam *= 10.0;
                res->zncc = z_acc;
                memcpy(p, p_acc, sizeof(p));
                memcpy(b, b_acc, sizeof(b));
                damped = 1;
            }
        }
        memset(dp, 0, sizeof(dp));
        const double *Ls = L;
        if (damped) {
            /* Cholesky of H + lambda diag(H) */
            for (int j = 0; j < np; ++j) {
                double d = Hm[j * np + j] * (1.0 + lam);
                for (int k = 0; k < j; ++k) d -= Ld[j * np + k] * Ld[j * np + k];
                if (!(d > 0.0)) { res->status = ST_SINGULAR; goto done; }
                Ld[j * np + j] = sqrt(d);
                for (int i = j + 1; i < np; ++i) {
                    double t = Hm[i * np + j];
                    for (int k = 0; k < j; ++k) t -= Ld[i * np + k] * Ld[j * np + k];
                    Ld[i * np + j] = t / Ld[j * np + j];
                }
            }
            Ls = Ld;
        }
        for (int j = 0; j < np; ++j) {
            double s = b[j];
            for (int k = 0; k < j; ++k) s -= Ls[j * np + k] * y[k];
            y[j] = s / Ls[j * np + j];
        }
        for (int j = np - 1; j >= 0; --j) {
            double s = y[j];
            for (int k = j + 1; k < np; ++k) s -= Ls[k * np + j] * dp[k];
            dp[j] = s / Ls[j * np + j];
        }
        for (int j = 0; j < np; ++j) dp[j] = -dp[j];
        /* 7: p <- p o dp^-1 */
        double pn[NPMAX];
        memset(pn, 0, sizeof(pn));
        if (!orc_compose(p, dp, np, pn)) { res->status = ST_SINGULAR; goto done; }
        memcpy(p, pn, sizeof(p));
        /* 8 */
        int bad = isnan(res->zncc);
        for (int j = 0; j < np; ++j) bad |= isnan(p[j]) || isnan(dp[j]);
        if (bad) { res->status = ST_NAN; goto done; }
        if (!damped && dp_norm(dp, np, h) < P->tol) {
            res->status = res->zncc >= P->zncc_min ? ST_CONVERGED : ST_LOW_ZNCC;
            goto done;
        }
    }
    res->status = ST_MAX_ITER;
done:
    memset(res->p, 0, sizeof(res->p));
    for (int j = 0; j < np; ++j) res->p[j] = p[j];
    free(fbar);
    free(fraw);
    free(graw);
    free(J);
    free(g);
}

/* ------------------------------------------------------------------ */
/* Grid, ROI, seeds                                                    */
/* ------------------------------------------------------------------ */

/* Nodes x_c = h + i*step, i < nx = floor((W-N)/step)+1 (y likewise); a node is
 * active iff all N^2 pixels of its subset are inside the ROI mask. */
static void active_nodes(const orc_problem *P, const uint8_t *roi, uint8_t *act)
{
    const int N = P->N, h = (N - 1) / 2;
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            int xc = h + i * P->step, yc = h + j * P->step, ok = 1;
            if (roi)
                for (int dy = -h; dy <= h && ok; ++dy)
                    for (int dx = -h; dx <= h; ++dx)
                        if (!roi[(long)(yc + dy) * P->W + (xc + dx)]) { ok = 0; break; }
            act[(long)j * P->nx + i] = (uint8_t)ok;
        }
}

/* Nearest active node to (x, y) (Euclidean), ties to smaller y then smaller
 * x.  Returns -1 if no node is active. */
static long snap_seed(const orc_problem *P, const uint8_t *act, double x, double y)
{
    const int h = (P->N - 1) / 2;
    long best = -1;
    double bd = 0.0;
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            if (!act[(long)j * P->nx + i]) continue;
            double ddx = h + i * P->step - x, ddy = h + j * P->step - y;
            double d = ddx * ddx + ddy * ddy;
            if (best < 0 || d < bd) { best = (long)j * P->nx + i; bd = d; }
        }
    return best;
}

/*
 * Integer-pixel seed initialisation (reading of the seeding step, which the
 * paper does with multi-window FFT correlation): zero-normalised
 * cross-correlation of the raw reference subset with the raw deformed
 * subset shifted by (du, dv) in round(u0, v0) + [-R, R]^2, skipping shifts
 * that leave the image.  ZNCC = (n Sfg - Sf Sg) / sqrt((n Sff - Sf^2)(n Sgg - Sg^2));
 * integer images accumulate the sums exactly in int64.  The maximum wins;
 * exact ties go to smaller du^2+dv^2, then smaller dv, then smaller du.
 * Returns 0 if no shift has a non-flat deformed window.
 */
int orc_seed_search(const orc_problem *P, int xc, int yc, double u0, double v0, int *du_out, int *dv_out,
                    double *zncc_out)
{
    const int N = P->N, h = (N - 1) / 2, R = P->seed_radius;
    const long n = (long)N * N;
    int cu = (int)lround(u0), cv = (int)lround(v0);
    int found = 0, bu = 0, bv = 0;
    double bz = 0.0;
    for (int dv = cv - R; dv <= cv + R; ++dv)
        for (int du = cu - R; du <= cu + R; ++du) {
            if (xc - h + du < 0 || xc + h + du > P->W - 1 || yc - h + dv < 0 || yc + h + dv > P->H - 1) continue;
            double num, A, B;
            if (P->int_pixels) {
                int64_t sf = 0, sff = 0, sg = 0, sgg = 0, sfg = 0;
                for (int y = -h; y <= h; ++y)
                    for (int x = -h; x <= h; ++x) {
                        int64_t f = (int64_t)P->fraw[(long)(yc + y) * P->W + xc + x];
                        int64_t g = (int64_t)P->graw[(long)(yc + y + dv) * P->W + xc + x + du];
                        sf += f; sff += f * f; sg += g; sgg += g * g; sfg += f * g;
                    }
                num = (double)(n * sfg - sf * sg);
                A = (double)(n * sff - sf * sf);
                B = (double)(n * sgg - sg * sg);
            } else {
                double sf = 0, sff = 0, sg = 0, sgg = 0, sfg = 0;
                for (int y = -h; y <= h; ++y)
                    for (int x = -h; x <= h; ++x) {
                        double f = P->fraw[(long)(yc + y) * P->W + xc + x];
                        double g = P->graw[(long)(yc + y + dv) * P->W + xc + x + du];
                        sf += f; sff += f * f; sg += g; sgg += g * g; sfg += f * g;
                    }
                num = n * sfg - sf * sg;
                A = n * sff - sf * sf;
                B = n * sgg - sg * sg;
            }
            if (!(A > 0.0) || !(B > 0.0)) continue;
            double z = num / sqrt(A * B);
            int better = 0;
            if (!found || z > bz) better = 1;
            else if (z == bz) {
                long d2 = (long)du * du + (long)dv * dv, b2 = (long)bu * bu + (long)bv * bv;
                if (d2 < b2 || (d2 == b2 && (dv < bv || (dv == bv && du < bu)))) better = 1;
            }
            if (better) { found = 1; bz = z; bu = du; bv = dv; }
        }
    *du_out = bu;
    *dv_out = bv;
    *zncc_out = bz;
    return found;
}

/*
 * Initial guess for node n from a converged neighbour m, delta = (x_n - x_m,
 * y_n - y_m): the neighbour's shape function extrapolated to n's centre
 * (displacement at the offset, and for the quadratic shape the gradient
 * there); GUESS_COPY copies p_m unchanged.
 */
void orc_transfer_guess(const double *pm, int np, double ddx, double ddy, int mode, double *out)
{
    memset(out, 0, sizeof(double) * NPMAX);
    for (int j = 0; j < np; ++j) out[j] = pm[j];
    if (mode == GUESS_COPY || np == 2) return;
    double u, v;
    shape_disp(pm, np, ddx, ddy, &u, &v);
    out[0] = u;
    out[1] = v;
    if (np >= 12) {
        out[2] = pm[2] + 2.0 * pm[6] * ddx + pm[7] * ddy;
        out[3] = pm[3] + pm[7] * ddx + 2.0 * pm[8] * ddy;
        out[4] = pm[4] + 2.0 * pm[9] * ddx + pm[10] * ddy;
        out[5] = pm[5] + pm[10] * ddx + 2.0 * pm[11] * ddy;
    }
}

/* ------------------------------------------------------------------ */
/* Reliability-guided propagation                                      */
/* ------------------------------------------------------------------ */

/* neighbour directions in tie-break priority: left (-x), right (+x), up (-y), down (+y) */
static const int DIRX[4] = {-1, 1, 0, 0};
static const int DIRY[4] = {0, 0, -1, 1};

typedef struct {
    double key;
    long counter;
    long node;
} heap_item;

static int heap_less(const heap_item *a, const heap_item *b) /* a below b in a max-heap */
{
    if (a->key != b->key) return a->key < b->key;
    return a->counter > b->counter;
}

static void heap_push(heap_item *h, long *sz, heap_item it)
{
    long i = (*sz)++;
    h[i] = it;
    while (i > 0) {
        long par = (i - 1) / 2;
        if (!heap_less(&h[par], &h[i])) break;
        heap_item t = h[par]; h[par] = h[i]; h[i] = t;
        i = par;
    }
}

static heap_item heap_pop(heap_item *h, long *sz)
{
    heap_item top = h[0];
    h[0] = h[--(*sz)];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1, r = l + 1, m = i;
        if (l < *sz && heap_less(&h[m], &h[l])) m = l;
        if (r < *sz && heap_less(&h[m], &h[r])) m = r;
        if (m == i) break;
        heap_item t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

/*
 * Full correlation of one pair.
 *   ref, def: raw pixel values [H][W] (double);  roi: [H][W] 0/1 or NULL;
 *   seeds: nseeds x (x, y, u0, v0);  order: ORDER_WAVE or ORDER_SEQUENTIAL;
 *   outputs (caller-allocated, [ny][nx] row-major): p [12][ny][nx] planar,
 *   zncc, iters, status, wave.
 * Returns the number of distinct seed nodes, or -1 if no seed could be
 * placed on an active node.
 *
 * WAVE: F0 = the seed nodes.  F(k+1) = active, unvisited nodes with at
 * least one CONVERGED 4-neighbour in F(k); the parent is that neighbour with
 * the largest ZNCC, exact ties by direction priority L, R, U, D seen from the
 * child; every node of F(k+1) starts from its parent's transferred guess and
 * is computed independently.  No node is computed twice and failed nodes are
 * not retried (global visited mask).
 * SEQUENTIAL: seeds computed in the given order; CONVERGED nodes go on a
 * max-heap keyed (ZNCC desc, insertion order asc); pop a node, compute its
 * unvisited active neighbours in order L, R, U, D from its guess, push the
 * converged ones.  `wave` then holds the propagation depth.
 */
long orc_correlate(const double *ref, const double *def, int W, int H, const uint8_t *roi, int int_pixels, int N,
                   int step, int np, double tol, int max_iter, double zncc_min, int seed_radius, int guess_mode,
                   int order, const double *seeds, int nseeds, int nthreads, double *p_out, double *zncc_out,
                   int32_t *iters_out, int32_t *status_out, int32_t *wave_out, double *seed_out, int cost,
                   double lm_lambda)
{
    orc_problem P;
    memset(&P, 0, sizeof(P));
    P.W = W; P.H = H; P.N = N; P.step = step; P.np = np;
    P.nx = W >= N ? (W - N) / step + 1 : 0;
    P.ny = H >= N ? (H - N) / step + 1 : 0;
    P.tol = tol; P.max_iter = max_iter; P.zncc_min = zncc_min; P.seed_radius = seed_radius;
    P.guess_mode = guess_mode; P.int_pixels = int_pixels; P.fraw = ref; P.graw = def;
    P.cost = cost; P.lm_lambda = lm_lambda;
    const long nn = (long)P.nx * P.ny;
    const int h = (N - 1) / 2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    double *fc = (double *)malloc(sizeof(double) * (size_t)W * H);
    double *gc = (double *)malloc(sizeof(double) * (size_t)W * H);
    orc_prefilter_2d(ref, W, H, fc);
    orc_prefilter_2d(def, W, H, gc);
    P.fc = fc; P.gc = gc;

    uint8_t *act = (uint8_t *)malloc((size_t)nn + 1);
    active_nodes(&P, roi, act);
    for (long k = 0; k < nn; ++k) {
        for (int j = 0; j < NPMAX; ++j) p_out[j * nn + k] = 0.0;
        zncc_out[k] = 0.0;
        iters_out[k] = 0;
        status_out[k] = act[k] ? ST_NOT_REACHED : ST_NOT_IN_ROI;
        wave_out[k] = -1;
    }

    /* seeds: snap, de-duplicate, integer search */
    long *F = (long *)malloc(sizeof(long) * (size_t)(nn + 1));
    long *G = (long *)malloc(sizeof(long) * (size_t)(nn + 1));
    double *pinit = (double *)malloc(sizeof(double) * NPMAX * (size_t)(nseeds + 1));
    long nf = 0;
    for (int s = 0; s < nseeds; ++s) {
        long node = snap_seed(&P, act, seeds[4 * s], seeds[4 * s + 1]);
        if (node < 0) continue;
        int dup = 0;
        for (long q = 0; q < nf; ++q) dup |= F[q] == node;
        if (dup) continue;
        int xc = h + (int)(node % P.nx) * step, yc = h + (int)(node / P.nx) * step;
        int du = 0, dv = 0;
        double zs = 0.0;
        orc_seed_search(&P, xc, yc, seeds[4 * s + 2], seeds[4 * s + 3], &du, &dv, &zs);
        double *pi = pinit + NPMAX * nf;
        memset(pi, 0, sizeof(double) * NPMAX);
        pi[0] = du;
        pi[1] = dv;
        if (seed_out) {
            seed_out[4 * nf] = (double)node;
            seed_out[4 * nf + 1] = du;
            seed_out[4 * nf + 2] = dv;
            seed_out[4 * nf + 3] = zs;
        }
        F[nf++] = node;
    }
    long nseed_nodes = nf;
    if (nf == 0) {
        free(fc); free(gc); free(act); free(F); free(G); free(pinit);
        return -1;
    }

#define STORE(node, r, wv)                                                        \
    do {                                                                          \
        for (int j_ = 0; j_ < NPMAX; ++j_) p_out[j_ * nn + (node)] = (r).p[j_];   \
        zncc_out[node] = (r).zncc;                                                \
        iters_out[node] = (r).iters;                                              \
        status_out[node] = (r).status;                                            \
        wave_out[node] = (wv);                                                    \
    } while (0)

    if (order == ORDER_WAVE) {
        for (long q = 0; q < nf; ++q) wave_out[F[q]] = 0;
#pragma omp parallel for schedule(dynamic, 1)
        for (long q = 0; q < nf; ++q) {
            long node = F[q];
            orc_node_result r;
            orc_icgn_node(&P, h + (node % P.nx) * step, h + (node / P.nx) * step, pinit + NPMAX * q, &r);
            STORE(node, r, 0);
        }
        for (int k = 0; nf > 0; ++k) {
            /* candidates: unvisited active neighbours of converged wave-k nodes */
            long ng = 0;
            for (long q = 0; q < nf; ++q) {
                long m = F[q];
                if (status_out[m] != ST_CONVERGED) continue;
                int mx = (int)(m % P.nx), my = (int)(m / P.nx);
                for (int d = 0; d < 4; ++d) {
                    int cx = mx + DIRX[d], cy = my + DIRY[d];
                    if (cx < 0 || cy < 0 || cx >= P.nx || cy >= P.ny) continue;
                    long c = (long)cy * P.nx + cx;
                    if (!act[c] || wave_out[c] != -1) continue;
                    wave_out[c] = k + 1;
                    G[ng++] = c;
                }
            }
            /* each candidate's parent and guess, then its subset */
#pragma omp parallel for schedule(dynamic, 1)
            for (long q = 0; q < ng; ++q) {
                long c = G[q];
                int cx = (int)(c % P.nx), cy = (int)(c / P.nx);
                long par = -1;
                for (int d = 0; d < 4; ++d) {
                    int mx = cx + DIRX[d], my = cy + DIRY[d];
                    if (mx < 0 || my < 0 || mx >= P.nx || my >= P.ny) continue;
                    long m = (long)my * P.nx + mx;
                    if (wave_out[m] != k || status_out[m] != ST_CONVERGED) continue;
                    if (par < 0 || zncc_out[m] > zncc_out[par]) par = m; /* earlier d wins exact ties */
                }
                double pm[NPMAX], g0[NPMAX];
                for (int j = 0; j < NPMAX; ++j) pm[j] = p_out[j * nn + par];
                double ddx = (double)(cx - par % P.nx) * step, ddy = (double)(cy - par / P.nx) * step;
                orc_transfer_guess(pm, np, ddx, ddy, guess_mode, g0);
                orc_node_result r;
                orc_icgn_node(&P, h + cx * step, h + cy * step, g0, &r);
                STORE(c, r, k + 1);
            }
            long *t = F; F = G; G = t;
            nf = ng;
        }
    } else {
        heap_item *hp = (heap_item *)malloc(sizeof(heap_item) * (size_t)(nn + 1));
        long hsz = 0, counter = 0;
        for (long q = 0; q < nf; ++q) {
            long node = F[q];
            orc_node_result r;
            orc_icgn_node(&P, h + (node % P.nx) * step, h + (node / P.nx) * step, pinit + NPMAX * q, &r);
            STORE(node, r, 0);
            if (r.status == ST_CONVERGED) {
                heap_item it = {r.zncc, counter++, node};
                heap_push(hp, &hsz, it);
            }
        }
        while (hsz > 0) {
            heap_item top = heap_pop(hp, &hsz);
            long m = top.node;
            int mx = (int)(m % P.nx), my = (int)(m / P.nx);
            double pm[NPMAX];
            for (int j = 0; j < NPMAX; ++j) pm[j] = p_out[j * nn + m];
            for (int d = 0; d < 4; ++d) {
                int cx = mx + DIRX[d], cy = my + DIRY[d];
                if (cx < 0 || cy < 0 || cx >= P.nx || cy >= P.ny) continue;
                long c = (long)cy * P.nx + cx;
                if (!act[c] || wave_out[c] != -1) continue;
                double g0[NPMAX];
                orc_transfer_guess(pm, np, (double)DIRX[d] * step, (double)DIRY[d] * step, guess_mode, g0);
                orc_node_result r;
                orc_icgn_node(&P, h + cx * step, h + cy * step, g0, &r);
                STORE(c, r, wave_out[m] + 1);
                if (r.status == ST_CONVERGED) {
                    heap_item it = {r.zncc, counter++, c};
                    heap_push(hp, &hsz, it);
                }
            }
        }
        free(hp);
    }
#undef STORE
    free(fc); free(gc); free(act); free(F); free(G); free(pinit);
    return nseed_nodes;
}

/* ------------------------------------------------------------------ */
/* Thin entry points for the tests                                     */
/* ------------------------------------------------------------------ */

/* Interpolant value and gradient at m points. */
void orc_eval_many(const double *coef, int W, int H, const double *x, const double *y, long m, double *v, double *gx,
                   double *gy)
{
    for (long i = 0; i < m; ++i) v[i] = orc_eval(coef, W, H, x[i], y[i], gx ? gx + i : NULL, gy ? gy + i : NULL);
}

/* One subset from a given start; images are raw pixels, prefiltered here. */
void orc_icgn_single(const double *ref, const double *def, int W, int H, int N, int np, double tol, int max_iter,
                     double zncc_min, double xc, double yc, const double *p_init, double *p_out, double *zncc,
                     int32_t *iters, int32_t *status, int cost, double lm_lambda)
{
    orc_problem P;
    memset(&P, 0, sizeof(P));
    P.W = W; P.H = H; P.N = N; P.np = np; P.tol = tol; P.max_iter = max_iter; P.zncc_min = zncc_min;
    P.cost = cost; P.lm_lambda = lm_lambda;
    double *fc = (double *)malloc(sizeof(double) * (size_t)W * H);
    double *gc = (double *)malloc(sizeof(double) * (size_t)W * H);
    orc_prefilter_2d(ref, W, H, fc);
    orc_prefilter_2d(def, W, H, gc);
    P.fc = fc; P.gc = gc;
    orc_node_result r;
    orc_icgn_node(&P, xc, yc, p_init, &r);
    for (int j = 0; j < NPMAX; ++j) p_out[j] = r.p[j];
    *zncc = r.zncc;
    *iters = r.iters;
    *status = r.status;
    free(fc);
    free(gc);
}

/* Integer seed search for one node of a raw pair. */
int orc_seed_single(const double *ref, const double *def, int W, int H, int int_pixels, int N, int R, int xc, int yc,
                    double u0, double v0, int32_t *du, int32_t *dv, double *zncc)
{
    orc_problem P;
    memset(&P, 0, sizeof(P));
    P.W = W; P.H = H; P.N = N; P.seed_radius = R; P.int_pixels = int_pixels; P.fraw = ref; P.graw = def;
    int a = 0, b = 0;
    int ok = orc_seed_search(&P, xc, yc, u0, v0, &a, &b, zncc);
    *du = a;
    *dv = b;
    return ok;
}
