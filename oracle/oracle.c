/*
 * CPU oracle of every job's stage chain -- TEST INFRASTRUCTURE, NOT THE PRODUCT.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header, table or constant with the HIP
 * path: the GPU side derives everything it needs on its own.
 *
 * Plain, slow, sequential loops; floating point is evaluated in double.
 *
 * What "correct" means here.  The method (SET, Sections 4.1-4.2) is a
 * scheduler: it must deliver, for every job, exactly the result of that job's
 * own chain (H2D -> stage kernels -> D2H, Section 3.2's three-step job
 * abstraction) applied to that job's own input, whatever stream, buffer slot,
 * steal or interleaving it ran with (per-job ordering and memory safety,
 * Section 1; worker isolation and stolen-job retargeting, Section 4.2).  So
 * the oracle is each chain written out for a single job.  The stage chains
 * themselves are this implementation's synthetic workloads, standing in for
 * the paper's Sobel-style image pipeline and small-kernel workloads
 * (Section 5.1); readings the paper leaves open are fixed as:
 *   box/histogram : 3x3 sum with zero padding, divisor always 9, 256 bins;
 *   Gaussian/Sobel: 5 taps exp(-k^2/2)/sum rounded to float32, replicate
 *                   borders, horizontal then vertical, unnormalised Sobel,
 *                   L2 magnitude, strict mag > 1 threshold, sum over all pixels;
 *   vector job    : z = a*x + y, t = tanh(z), S = sum t;
 *   scan          : inclusive prefix sum of int32 into int64;
 *   thermal grid  : explicit five-point heat update with power input and an
 *                   ambient loss term, zero-flux borders (see below).
 *
 * parity pinned: every function here is pinned by tests against brute force,
 * closed forms and invariants (see the oracle tests).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* ------------------------------------------------------------------ box / histogram */
/*
 * S[y][x] = sum over the 3x3 neighbourhood of I, pixels outside the image
 * count as 0; Q = floor(S / 9); H[v] = number of pixels with Q == v.
 * Any of S, Q may be NULL.  h*w == 0 gives an all-zero histogram.
 */
int oracle_box_hist_u8(const uint8_t *img, int64_t h, int64_t w,
                       uint16_t *S, uint8_t *Q, uint32_t *H)
{
    if (h < 0 || w < 0 || H == NULL || (h * w > 0 && img == NULL))
        return ORACLE_EINVAL;
    for (int v = 0; v < 256; ++v)
        H[v] = 0;
    for (int64_t y = 0; y < h; ++y) {
        for (int64_t x = 0; x < w; ++x) {
            unsigned s = 0;
            for (int64_t dy = -1; dy <= 1; ++dy) {
                for (int64_t dx = -1; dx <= 1; ++dx) {
                    int64_t yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= h || xx < 0 || xx >= w)
                        continue; /* zero padding */
                    s += img[yy * w + xx];
                }
            }
            unsigned q = s / 9u;
            if (S) S[y * w + x] = (uint16_t)s;
            if (Q) Q[y * w + x] = (uint8_t)q;
            H[q] += 1;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ Gaussian / Sobel */
/* Sampled Gaussian of radius 2, sigma 1, normalised in double, rounded to float32. */
void oracle_gauss_taps(double g[5])
{
    double e[5], s = 0.0;
    for (int k = -2; k <= 2; ++k) {
        e[k + 2] = exp(-(double)(k * k) / 2.0);
        s += e[k + 2];
    }
    for (int i = 0; i < 5; ++i)
        g[i] = (double)(float)(e[i] / s);
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/*
 * blur = separable 5x5 Gaussian of img with replicated borders (the 2-D sum
 * of g[i]*g[j]*img[clamp(y+i-2)][clamp(x+j-2)], evaluated horizontally then
 * vertically in double);
 * gx, gy = Sobel derivatives of blur with replicated borders,
 *   gx = sum_{dy,dx} Kx[dy][dx] * blur[clamp(y+dy)][clamp(x+dx)],
 *   Kx = [[-1,0,1],[-2,0,2],[-1,0,1]], Ky = transpose(Kx);
 * mag = sqrt(gx^2 + gy^2); mask = mag > 1; count = sum mask; sum = sum mag;
 * band = number of pixels with |mag - 1| <= band_eps (pixels whose mask a
 * float32 evaluation may legitimately flip).
 * blur, mag, mask may be NULL.
 */
int oracle_gauss_sobel_f32(const float *img, int64_t h, int64_t w, double band_eps,
                           double *blur, double *mag, uint8_t *mask,
                           uint32_t *count, double *sum, uint32_t *band)
{
    if (h < 0 || w < 0 || count == NULL || sum == NULL || band == NULL ||
        (h * w > 0 && img == NULL))
        return ORACLE_EINVAL;
    *count = 0;
    *sum = 0.0;
    *band = 0;
    if (h * w == 0)
        return ORACLE_OK;
    double g[5];
    oracle_gauss_taps(g);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(h * w));
    double *b = blur ? blur : (double *)malloc(sizeof(double) * (size_t)(h * w));
    if (tmp == NULL || b == NULL) {
        free(tmp);
        if (!blur) free(b);
        return ORACLE_ENOMEM;
    }
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            double acc = 0.0;
            for (int j = -2; j <= 2; ++j)
                acc += g[j + 2] * (double)img[y * w + clampi(x + j, 0, w - 1)];
            tmp[y * w + x] = acc;
        }
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            double acc = 0.0;
            for (int i = -2; i <= 2; ++i)
                acc += g[i + 2] * tmp[clampi(y + i, 0, h - 1) * w + x];
            b[y * w + x] = acc;
        }
    static const int kx[3][3] = {{-1, 0, 1}, {-2, 0, 2}, {-1, 0, 1}};
    uint32_t cnt = 0, bnd = 0;
    double s = 0.0;
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            double gx = 0.0, gy = 0.0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    double v = b[clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1)];
                    gx += kx[dy + 1][dx + 1] * v;
                    gy += kx[dx + 1][dy + 1] * v; /* transpose */
                }
            double m = sqrt(gx * gx + gy * gy);
            int on = m > 1.0;
            if (mag) mag[y * w + x] = m;
            if (mask) mask[y * w + x] = (uint8_t)on;
            cnt += (uint32_t)on;
            s += m;
            if (fabs(m - 1.0) <= band_eps)
                bnd += 1;
        }
    *count = cnt;
    *sum = s;
    *band = bnd;
    free(tmp);
    if (!blur) free(b);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ vector job */
/*
 * z_i = a*x_i + y_i, t_i = tanh(z_i), S = sum_i t_i, all in double.
 * E = 2^-24 * ((ceil(log2 n) + 4) * sum|t_i| + sum|z_i|) is the a-priori
 * error allowance of a float32 evaluation (reduction depth, a few-ulp tanh,
 * rounded z); E may be NULL.  n == 0 gives S = 0.
 */
int oracle_saxpy_tanh_sum_f32(const float *x, const float *y, int64_t n, float a,
                              double *S, double *E)
{
    if (n < 0 || S == NULL || (n > 0 && (x == NULL || y == NULL)))
        return ORACLE_EINVAL;
    double s = 0.0, st = 0.0, sz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double z = (double)a * (double)x[i] + (double)y[i];
        double t = tanh(z);
        s += t;
        st += fabs(t);
        sz += fabs(z);
    }
    *S = s;
    if (E) {
        int depth = 0;
        while (depth < 63 && ((int64_t)1 << depth) < n)
            ++depth; /* ceil(log2 n) */
        *E = ldexp((depth + 4) * st + sz, -24);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ scan */
/* out[i] = sum_{j <= i} in[j], accumulated in int64 (exact for |in| < 2^31, n < 2^32). */
int oracle_scan_i32_i64(const int32_t *in, int64_t n, int64_t *out)
{
    if (n < 0 || (n > 0 && (in == NULL || out == NULL)))
        return ORACLE_EINVAL;
    int64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) {
        acc += (int64_t)in[i];
        out[i] = acc;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ thermal grid (iterative stencil) */
/*
 * The memory-bound iterative workload standing in for the paper's Hotspot
 * (Section 5.1): a chip's temperature grid T advanced by explicit steps of
 * the two-dimensional heat equation with a power-density source and a
 * leakage to ambient.  One step, for every cell, with N, S, W, E its four
 * neighbours (a neighbour outside the grid is the cell itself: no heat
 * crosses the border):
 *
 *   T' = T + CP*P + CY*(N + S - 2T) + CX*(W + E - 2T) + CZ*(T_AMB - T)
 *
 * iterated `iters` times from T0.  The coefficients are the workload's
 * (CX = CY = 0.1, CZ = 1/640, CP = 0.5, T_AMB = 300); 1 - 2CX - 2CY - CZ > 0,
 * so every step is a convex combination plus source and the scheme is
 * monotone.  Evaluated in double from the float32 inputs.
 */
#define HS_CX 0.1
#define HS_CY 0.1
#define HS_CZ (1.0 / 640.0)
#define HS_CP 0.5
#define HS_TAMB 300.0

int oracle_hotspot_f32(const float *T0, const float *P, int64_t h, int64_t w, int iters, double *out)
{
    if (h < 1 || w < 1 || iters < 0 || T0 == NULL || P == NULL || out == NULL)
        return ORACLE_EINVAL;
    const int64_t n = h * w;
    double *a = (double *)malloc((size_t)n * sizeof(double));
    double *b = (double *)malloc((size_t)n * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i)
        a[i] = (double)T0[i];
    for (int k = 0; k < iters; ++k) {
        for (int64_t y = 0; y < h; ++y) {
            for (int64_t x = 0; x < w; ++x) {
                const double t = a[y * w + x];
                const double nn = a[clampi(y - 1, 0, h - 1) * w + x];
                const double ss = a[clampi(y + 1, 0, h - 1) * w + x];
                const double ww = a[y * w + clampi(x - 1, 0, w - 1)];
                const double ee = a[y * w + clampi(x + 1, 0, w - 1)];
                b[y * w + x] = t + HS_CP * (double)P[y * w + x] + HS_CY * (nn + ss - 2.0 * t) +
                               HS_CX * (ww + ee - 2.0 * t) + HS_CZ * (HS_TAMB - t);
            }
        }
        double *tmp = a;
        a = b;
        b = tmp;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    free(a);
    free(b);
    return ORACLE_OK;
}
