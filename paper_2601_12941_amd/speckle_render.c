/*
 * Gaussian-blob speckle renderer for large synthetic images (input generation
 * only; none of the correlation method's arithmetic).
 *
 * img[y][x] += A_k exp(-((x - X_k)^2 + (y - Y_k)^2) / (2 s_k^2)) for every blob k
 * with (x - X_k)^2 + (y - Y_k)^2 <= 25 s_k^2, at integer pixel centres.
 * The image is split into horizontal bands, one OpenMP thread per band; a band
 * visits the blobs whose vertical extent meets it, in the order of `order`
 * (blob indices sorted by Y), so every pixel sums its blobs in the same order
 * whatever the thread count.
 *
 * Build: gcc -O3 -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>

static long lower_bound(const double *ys, const int64_t *order, long n, double v)
{
    long lo = 0, hi = n;
    while (lo < hi) {
        long mid = lo + (hi - lo) / 2;
        if (ys[order[mid]] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

void speckle_render(float *img, long W, long H, const double *X, const double *Y, const double *S, const double *A,
                    const int64_t *order, long n, double smax, long band)
{
    const double R = ceil(5.0 * smax);
    const long nb = (H + band - 1) / band;
#pragma omp parallel for schedule(dynamic, 1)
    for (long b = 0; b < nb; ++b) {
        const long y0 = b * band, y1 = y0 + band < H ? y0 + band : H;
        for (long i = y0 * W; i < y1 * W; ++i) img[i] = 0.0f;
        long first = lower_bound(Y, order, n, (double)y0 - R - 1.0);
        for (long q = first; q < n; ++q) {
            const long k = order[q];
            const double yk = Y[k];
            if (yk > (double)y1 + R + 1.0) break;
            const double xk = X[k], sk = S[k], ak = A[k];
            const double r2max = 25.0 * sk * sk, inv = 1.0 / (2.0 * sk * sk);
            const long rr = (long)ceil(5.0 * sk);
            const long cx = (long)floor(xk), cy = (long)floor(yk);
            long ya = cy - rr, yb = cy + rr;
            if (ya < y0) ya = y0;
            if (yb > y1 - 1) yb = y1 - 1;
            long xa = cx - rr, xb = cx + rr;
            if (xa < 0) xa = 0;
            if (xb > W - 1) xb = W - 1;
            for (long y = ya; y <= yb; ++y) {
                const double dy2 = ((double)y - yk) * ((double)y - yk);
                float *row = img + y * W;
                for (long x = xa; x <= xb; ++x) {
                    const double r2 = ((double)x - xk) * ((double)x - xk) + dy2;
                    if (r2 <= r2max) row[x] += (float)(ak * exp(-r2 * inv));
                }
            }
        }
    }
}
