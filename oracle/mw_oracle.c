/*
 * FP64 reference ("oracle") of the multi-window FFT initial guess.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the package's smoke check and
 * the benchmark's CPU-baseline leg, never by the library's own path.  Plain,
 * single-threaded, no shared code with the GPU path.
 *
 * Paper: Hirst et al., arXiv 2601.12941, Sec. 2.2 (the multi-window FFT
 * procedure, Eq. (1), the window-size rule, the MULTIWINDOW sub-pixel mode)
 * and Sec. 4 (MAD outlier removal at every window size).  Readings where the
 * paper is silent:
 *   - window sizes: W1 = the smallest power of two above the maximum
 *     displacement (halved while larger than the image), then W1/2, W1/4, ...
 *     while larger than Wf, the smallest power of two at least the subset size;
 *     the last level puts one Wf window on every node of the subset grid;
 *   - level grids: windows fully inside the image, centres W/2 + j W/2 (50 %
 *     overlap); a node-level window's top-left corner is x_c - Wf/2 clamped
 *     into the image;
 *   - the deformed window sits at the reference window shifted by the integer
 *     guess; a window whose shifted copy would leave the image keeps the guess
 *     as its estimate (no correlation); guesses are integers: level 1 starts from
 *     zero, later levels from the bilinear interpolation of the previous
 *     level's integer field at the window centre (the four nearest coarser
 *     points), evaluated exactly in integers and rounded half away from zero;
 *   - both windows are tapered by the separable periodic Hann weight
 *     sin^2(pi x / W) sin^2(pi y / W) before Eq. (1): the bare windows are not
 *     periodic, and their own edges give the map a peak at zero shift that
 *     outweighs the true one (the usual apodisation of PIV correlation);
 *   - the displacement of a window is the shift plus minus the peak of
 *     Eq. (1)'s map, the peak index q taken in [-W/2, W/2) (ties: smaller
 *     |q|^2, then smaller q_y, then smaller q_x);
 *   - MAD outlier removal: a window whose u or v differs from the median of its
 *     existing 3x3 neighbours by more than thr (MAD + 1 px) (MAD = median
 *     absolute deviation of those neighbours, at least 3 of them; the 1 px is the
 *     resolution of the integer peaks the test sees) takes the neighbours'
 *     medians, rounded half away from zero; every value in the test is a
 *     multiple of 1/4, so it is exact in any floating-point precision;
 *   - MULTIWINDOW sub-pixel: on the node level, a 3-point Gaussian fit per axis
 *     through the peak and its two neighbours on the map (a parabola when a
 *     value is not positive; no shift when the fit is degenerate or more than
 *     half a pixel away).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (with dic_oracle.c)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* In-place radix-2 complex FFT of length n (a power of two): decimation in
 * time with bit-reversed input order.  sign -1: forward exp(-2 pi i k j / n);
 * +1: inverse without the 1/n scale. */
void orc_fft(double *re, double *im, int n, int sign)
{
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        const double ang = sign * 2.0 * M_PI / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const double wr = cos(ang * k), wi = sin(ang * k);
                const int a = i + k, b = i + k + len / 2;
                const double xr = re[b] * wr - im[b] * wi, xi = re[b] * wi + im[b] * wr;
                re[b] = re[a] - xr;
                im[b] = im[a] - xi;
                re[a] += xr;
                im[a] += xi;
            }
    }
}

/* 2-D transform of a W x W array (row-major): every row, then every column. */
void orc_fft2(double *re, double *im, int W, int sign)
{
    double *cr = (double *)malloc(sizeof(double) * W), *ci = (double *)malloc(sizeof(double) * W);
    for (int y = 0; y < W; ++y) orc_fft(re + (long)y * W, im + (long)y * W, W, sign);
    for (int x = 0; x < W; ++x) {
        for (int y = 0; y < W; ++y) { cr[y] = re[(long)y * W + x]; ci[y] = im[(long)y * W + x]; }
        orc_fft(cr, ci, W, sign);
        for (int y = 0; y < W; ++y) { re[(long)y * W + x] = cr[y]; im[(long)y * W + x] = ci[y]; }
    }
    free(cr);
    free(ci);
}

/* Eq. (1): r = real(F^-1{ F{f} conj(F{g}) / (|F{f}| |F{g}|) }) for two W x W
 * real windows (terms with a zero magnitude are dropped), scaled by 1/W^2. */
void orc_phase_corr(const double *f, const double *g, int W, double *r)
{
    const long n = (long)W * W;
    double *fr = (double *)calloc(n, sizeof(double)), *fi = (double *)calloc(n, sizeof(double));
    double *gr = (double *)calloc(n, sizeof(double)), *gi = (double *)calloc(n, sizeof(double));
    memcpy(fr, f, sizeof(double) * n);
    memcpy(gr, g, sizeof(double) * n);
    orc_fft2(fr, fi, W, -1);
    orc_fft2(gr, gi, W, -1);
    for (long k = 0; k < n; ++k) {
        const double cr = fr[k] * gr[k] + fi[k] * gi[k];   /* F conj(G) */
        const double ci = fi[k] * gr[k] - fr[k] * gi[k];
        const double mag = hypot(fr[k], fi[k]) * hypot(gr[k], gi[k]);
        fr[k] = mag > 0.0 ? cr / mag : 0.0;
        fi[k] = mag > 0.0 ? ci / mag : 0.0;
    }
    orc_fft2(fr, fi, W, +1);
    for (long k = 0; k < n; ++k) r[k] = fr[k] / (double)n;
    free(fr); free(fi); free(gr); free(gi);
}

/* Peak of a W x W map as the signed index q in [-W/2, W/2)^2 (ties as above);
 * *margin receives the peak minus the largest value elsewhere. */
void orc_map_peak(const double *r, int W, int *qx, int *qy, double *margin)
{
    int bx = 0, by = 0, found = 0;
    double best = 0.0, second = -INFINITY;
    for (int y = 0; y < W; ++y)
        for (int x = 0; x < W; ++x) {
            const double v = r[(long)y * W + x];
            const int sx = x < W / 2 ? x : x - W, sy = y < W / 2 ? y : y - W;
            int better = !found || v > best;
            if (found && v == best) {
                const long d2 = (long)sx * sx + (long)sy * sy, b2 = (long)bx * bx + (long)by * by;
                better = d2 < b2 || (d2 == b2 && (sy < by || (sy == by && sx < bx)));
            }
            if (better) {
                if (found) second = fmax(second, best);
                found = 1; best = v; bx = sx; by = sy;
            } else {
                second = fmax(second, v);
            }
        }
    *qx = bx;
    *qy = by;
    if (margin) *margin = best - second;
}

/* Sub-pixel offset of a peak from its neighbours a (at -1), b (peak), c (+1). */
double orc_gauss3(double a, double b, double c)
{
    double e;
    if (a > 0.0 && b > 0.0 && c > 0.0) {
        const double la = log(a), lb = log(b), lc = log(c);
        const double den = 2.0 * (la - 2.0 * lb + lc);
        e = den != 0.0 ? (la - lc) / den : 0.0;
    } else {
        const double den = 2.0 * (a - 2.0 * b + c);
        e = den != 0.0 ? (a - c) / den : 0.0;
    }
    return (fabs(e) <= 0.5) ? e : 0.0;
}

/* Window sizes: regular levels into sizes[], their count returned; *wf receives
 * the node-level size (0 if the image cannot hold it). */
int orc_mw_levels(int max_disp, int N, int imgW, int imgH, int *sizes, int *wf)
{
    int f = 1;
    while (f < N) f <<= 1;
    const int side = imgW < imgH ? imgW : imgH;
    *wf = f <= side ? f : 0;
    int w1 = 1;
    while (w1 <= max_disp) w1 <<= 1;
    while (w1 > side) w1 >>= 1;
    int n = 0;
    for (int w = w1; w > f; w >>= 1) sizes[n++] = w;
    return n;
}

/* round(num / den) half away from zero, den > 0 */
static long round_div(long num, long den)
{
    return num >= 0 ? (2 * num + den) / (2 * den) : -((-2 * num + den) / (2 * den));
}

typedef struct {
    int W, S, nx, ny; /* window size, grid spacing, grid shape; centres W/2 + j S */
    int *u, *v;       /* integer displacements [ny][nx] */
} orc_level;

/* The previous level's integer field interpolated bilinearly at (cx, cy),
 * exactly (numerators over S^2 in integers), clamped to the grid's extent. */
static void guess_from(const orc_level *L, int cx, int cy, int *gu, int *gv)
{
    const int S = L->S, o = L->W / 2;
    int i0 = (cx - o) >= 0 ? (cx - o) / S : 0, j0 = (cy - o) >= 0 ? (cy - o) / S : 0;
    if (i0 > L->nx - 1) i0 = L->nx - 1;
    if (j0 > L->ny - 1) j0 = L->ny - 1;
    const int i1 = i0 + 1 < L->nx ? i0 + 1 : i0, j1 = j0 + 1 < L->ny ? j0 + 1 : j0;
    long a = (long)cx - o - (long)i0 * S, b = (long)cy - o - (long)j0 * S;
    if (a < 0) a = 0;
    if (b < 0) b = 0;
    if (a > S || i1 == i0) a = i1 == i0 ? 0 : S;
    if (b > S || j1 == j0) b = j1 == j0 ? 0 : S;
    const long w00 = (S - a) * (S - b), w10 = a * (S - b), w01 = (S - a) * b, w11 = a * b;
    const long den = (long)S * S;
    const long nu = w00 * L->u[j0 * L->nx + i0] + w10 * L->u[j0 * L->nx + i1] + w01 * L->u[j1 * L->nx + i0] +
                    w11 * L->u[j1 * L->nx + i1];
    const long nv = w00 * L->v[j0 * L->nx + i0] + w10 * L->v[j0 * L->nx + i1] + w01 * L->v[j1 * L->nx + i0] +
                    w11 * L->v[j1 * L->nx + i1];
    *gu = (int)round_div(nu, den);
    *gv = (int)round_div(nv, den);
}

static int cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static double median(double *a, int n)
{
    qsort(a, n, sizeof(double), cmp_double);
    return n & 1 ? a[n / 2] : 0.5 * (a[n / 2 - 1] + a[n / 2]);
}

/* One MAD pass over an integer grid field (ok: entries that take part; NULL =
 * all); rep (may be NULL) marks the replaced entries.  Returns their number. */
long orc_mad_filter(int *u, int *v, const uint8_t *ok, int nx, int ny, double thr, uint8_t *rep)
{
    const long n = (long)nx * ny;
    int *ou = (int *)malloc(sizeof(int) * n), *ov = (int *)malloc(sizeof(int) * n);
    memcpy(ou, u, sizeof(int) * n);
    memcpy(ov, v, sizeof(int) * n);
    long replaced = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const long c = (long)j * nx + i;
            if (rep) rep[c] = 0;
            if (ok && !ok[c]) continue;
            double nu[8], nv[8], du[8], dv[8];
            int m = 0;
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di, jj = j + dj;
                    if ((di == 0 && dj == 0) || ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
                    const long q = (long)jj * nx + ii;
                    if (ok && !ok[q]) continue;
                    nu[m] = ou[q];
                    nv[m] = ov[q];
                    ++m;
                }
            if (m < 3) continue;
            const double mu = median(nu, m), mv = median(nv, m);
            for (int k = 0; k < m; ++k) { du[k] = fabs(nu[k] - mu); dv[k] = fabs(nv[k] - mv); }
            const double madu = median(du, m), madv = median(dv, m);
            if (fabs(ou[c] - mu) > thr * (madu + 1.0) || fabs(ov[c] - mv) > thr * (madv + 1.0)) {
                u[c] = (int)round_div((long)(2.0 * mu), 2);   /* medians are multiples of 1/2 */
                v[c] = (int)round_div((long)(2.0 * mv), 2);
                if (rep) rep[c] = 1;
                ++replaced;
            }
        }
    free(ou);
    free(ov);
    return replaced;
}

/* Phase-correlation estimate of one window pair: reference top-left (rx, ry),
 * integer shift (sx, sy); result in (*du, *dv) = shift - peak, sub-pixel fit in
 * (*fu, *fv) if asked.  A shifted window outside the image returns the shift. */
static void window_estimate(const double *ref, const double *def, int imgW, int imgH, int Wn, int rx, int ry,
                            int sx, int sy, int subpixel, double *rbuf, double *fbuf, double *gbuf, int *du, int *dv,
                            double *fu, double *fv, double *margin)
{
    const int gx = rx + sx, gy = ry + sy;
    if (gx < 0 || gy < 0 || gx > imgW - Wn || gy > imgH - Wn) {
        *du = sx;
        *dv = sy;
        *fu = sx;
        *fv = sy;
        *margin = 0.0;
        return;
    }
    for (int y = 0; y < Wn; ++y) {
        const double sy = sin(M_PI * y / Wn);
        for (int x = 0; x < Wn; ++x) {
            const double sx = sin(M_PI * x / Wn), w = sx * sx * sy * sy;
            fbuf[(long)y * Wn + x] = w * ref[(long)(ry + y) * imgW + rx + x];
            gbuf[(long)y * Wn + x] = w * def[(long)(gy + y) * imgW + gx + x];
        }
    }
    orc_phase_corr(fbuf, gbuf, Wn, rbuf);
    int qx, qy;
    orc_map_peak(rbuf, Wn, &qx, &qy, margin);
    *du = (gx - rx) - qx;
    *dv = (gy - ry) - qy;
    *fu = *du;
    *fv = *dv;
    if (subpixel) {
        const int px = (qx + Wn) % Wn, py = (qy + Wn) % Wn;
        const double b = rbuf[(long)py * Wn + px];
        const double ex = orc_gauss3(rbuf[(long)py * Wn + (px + Wn - 1) % Wn], b, rbuf[(long)py * Wn + (px + 1) % Wn]);
        const double ey = orc_gauss3(rbuf[(long)((py + Wn - 1) % Wn) * Wn + px], b, rbuf[(long)((py + 1) % Wn) * Wn + px]);
        *fu = (gx - rx) - (qx + ex);
        *fv = (gy - ry) - (qy + ey);
    }
}

/*
 * Multi-window FFT estimate at every node of the subset grid (N, step) of a
 * raw pair [H][W] (doubles).  roi: [H][W] 0/1 or NULL; a node is computed iff
 * all N^2 of its pixels are inside.  Outputs [ny][nx]: u, v (integers unless
 * subpixel), valid (1 computed, 0 not), margin (the peak's lead over the
 * map's next value).  levels_out (may be NULL) receives the sizes used, the
 * node level last; returns their count, or -1 if the image cannot hold a
 * node-level window.
 */
int orc_multiwindow(const double *ref, const double *def, int W, int H, const uint8_t *roi, int N, int step,
                    int max_disp, int subpixel, double mad_thr, double *u_out, double *v_out, int32_t *valid_out,
                    double *margin_out, int32_t *levels_out)
{
    int sizes[32], wf = 0;
    const int nlev = orc_mw_levels(max_disp, N, W, H, sizes, &wf);
    if (wf == 0) return -1;
    const int h = (N - 1) / 2;
    const int nx = W >= N ? (W - N) / step + 1 : 0, ny = H >= N ? (H - N) / step + 1 : 0;
    const int wmax = nlev > 0 ? sizes[0] : wf;
    double *rbuf = (double *)malloc(sizeof(double) * wmax * wmax);
    double *fbuf = (double *)malloc(sizeof(double) * wmax * wmax);
    double *gbuf = (double *)malloc(sizeof(double) * wmax * wmax);
    orc_level prev;
    memset(&prev, 0, sizeof(prev));
    for (int l = 0; l < nlev; ++l) {
        orc_level L;
        L.W = sizes[l];
        L.S = L.W / 2;
        L.nx = (W - L.W) / L.S + 1;
        L.ny = (H - L.W) / L.S + 1;
        L.u = (int *)malloc(sizeof(int) * L.nx * L.ny);
        L.v = (int *)malloc(sizeof(int) * L.nx * L.ny);
        for (int j = 0; j < L.ny; ++j)
            for (int i = 0; i < L.nx; ++i) {
                const int cx = L.W / 2 + i * L.S, cy = L.W / 2 + j * L.S;
                int gu = 0, gv = 0;
                if (l > 0) guess_from(&prev, cx, cy, &gu, &gv);
                double fu, fv, mg;
                window_estimate(ref, def, W, H, L.W, cx - L.W / 2, cy - L.W / 2, gu, gv, 0, rbuf, fbuf, gbuf,
                                &L.u[j * L.nx + i], &L.v[j * L.nx + i], &fu, &fv, &mg);
            }
        if (mad_thr > 0.0) orc_mad_filter(L.u, L.v, NULL, L.nx, L.ny, mad_thr, NULL);
        if (l > 0) { free(prev.u); free(prev.v); }
        prev = L;
        if (levels_out) levels_out[l] = L.W;
    }
    /* node level */
    const long nn = (long)nx * ny;
    int *nu = (int *)calloc(nn + 1, sizeof(int)), *nv = (int *)calloc(nn + 1, sizeof(int));
    uint8_t *ok = (uint8_t *)calloc(nn + 1, 1);
    double *fu = (double *)calloc(nn + 1, sizeof(double)), *fv = (double *)calloc(nn + 1, sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const long c = (long)j * nx + i;
            const int xc = h + i * step, yc = h + j * step;
            int act = 1;
            if (roi)
                for (int dy = -h; dy <= h && act; ++dy)
                    for (int dx = -h; dx <= h; ++dx)
                        if (!roi[(long)(yc + dy) * W + xc + dx]) { act = 0; break; }
            ok[c] = (uint8_t)act;
            margin_out[c] = 0.0;
            if (!act) continue;
            int gu = 0, gv = 0;
            if (nlev > 0) guess_from(&prev, xc, yc, &gu, &gv);
            int rx = xc - wf / 2, ry = yc - wf / 2;
            if (rx < 0) rx = 0;
            if (ry < 0) ry = 0;
            if (rx > W - wf) rx = W - wf;
            if (ry > H - wf) ry = H - wf;
            window_estimate(ref, def, W, H, wf, rx, ry, gu, gv, subpixel, rbuf, fbuf, gbuf, &nu[c], &nv[c], &fu[c],
                            &fv[c], &margin_out[c]);
        }
    /* the MAD test runs on the integer peaks; a replaced node takes the
     * neighbours' integer medians, the others keep their (sub-pixel) estimate */
    uint8_t *rp = (uint8_t *)calloc(nn + 1, 1);
    if (mad_thr > 0.0) orc_mad_filter(nu, nv, ok, nx, ny, mad_thr, rp);
    for (long c = 0; c < nn; ++c) {
        valid_out[c] = ok[c];
        u_out[c] = ok[c] ? (rp[c] ? (double)nu[c] : fu[c]) : 0.0;
        v_out[c] = ok[c] ? (rp[c] ? (double)nv[c] : fv[c]) : 0.0;
    }
    free(rp);
    if (levels_out) levels_out[nlev] = wf;
    if (nlev > 0) { free(prev.u); free(prev.v); }
    free(nu); free(nv); free(ok); free(fu); free(fv);
    free(rbuf); free(fbuf); free(gbuf);
    return nlev + 1;
}
