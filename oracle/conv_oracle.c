/*
 * FP64 CPU oracle of the PSF surrogate's convolution layers.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  The surrogate is this library's
 * own learned component (the paper has none); its layers are plain 3-D
 * cross-correlations with zero padding and strides, evaluated here by direct
 * loops in double precision on whatever (for instance bf16-rounded) operands
 * the caller passes:
 *
 *   y[n][co][z][y][x] = b[co] + sum_{ci,a,b,c} w[co][ci][a][b][c]
 *                        * x[n][ci][z sd + a - pd][y sh + b - ph][x sw + c - pw]
 *   (optionally ReLU), and its exact gradients
 *   dx = sum over (co, a, b, c) of w * dy at the output positions reading x,
 *   dw = sum over (n, z, y, x) of dy * x,  db = sum over (n, z, y, x) of dy.
 * Layouts: x [N][Ci][D][H][W], w [Co][Ci][kd][kh][kw], y [N][Co][Do][Ho][Wo],
 * Do = (D + 2 pd - kd) / sd + 1 (likewise Ho, Wo).
 */
#include <stdlib.h>
#include <string.h>

#define CONV_ERR_ARG (-1)

static int out_size(int n, int k, int s, int p) { return (n + 2 * p - k) / s + 1; }

static int check(int N, int Ci, int D, int H, int W, int Co, int kd, int kh, int kw, int sd,
                 int sh, int sw, int pd, int ph, int pw) {
    if (N < 1 || Ci < 1 || D < 1 || H < 1 || W < 1 || Co < 1 || kd < 1 || kh < 1 || kw < 1 ||
        sd < 1 || sh < 1 || sw < 1 || pd < 0 || ph < 0 || pw < 0)
        return CONV_ERR_ARG;
    if (out_size(D, kd, sd, pd) < 1 || out_size(H, kh, sh, ph) < 1 || out_size(W, kw, sw, pw) < 1)
        return CONV_ERR_ARG;
    return 0;
}

int oracle_conv3d_forward(const double *x, const double *w, const double *b, double *y, int N,
                          int Ci, int D, int H, int W, int Co, int kd, int kh, int kw, int sd,
                          int sh, int sw, int pd, int ph, int pw, int relu) {
    if (!x || !w || !y || check(N, Ci, D, H, W, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw))
        return CONV_ERR_ARG;
    const int Do = out_size(D, kd, sd, pd), Ho = out_size(H, kh, sh, ph), Wo = out_size(W, kw, sw, pw);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int n = 0; n < N; n++)
        for (int co = 0; co < Co; co++)
            for (int z = 0; z < Do; z++)
                for (int yy = 0; yy < Ho; yy++)
                    for (int xx = 0; xx < Wo; xx++) {
                        double acc = b ? b[co] : 0.0;
                        for (int ci = 0; ci < Ci; ci++)
                            for (int a = 0; a < kd; a++) {
                                const int iz = z * sd + a - pd;
                                if (iz < 0 || iz >= D) continue;
                                for (int bb = 0; bb < kh; bb++) {
                                    const int iy = yy * sh + bb - ph;
                                    if (iy < 0 || iy >= H) continue;
                                    for (int c = 0; c < kw; c++) {
                                        const int ix = xx * sw + c - pw;
                                        if (ix < 0 || ix >= W) continue;
                                        acc += w[((((long)co * Ci + ci) * kd + a) * kh + bb) * kw + c] *
                                               x[((((long)n * Ci + ci) * D + iz) * H + iy) * W + ix];
                                    }
                                }
                            }
                        if (relu && acc < 0) acc = 0;
                        y[((((long)n * Co + co) * Do + z) * Ho + yy) * Wo + xx] = acc;
                    }
    return 0;
}

int oracle_conv3d_backward(const double *x, const double *w, const double *dy, double *dx,
                           double *dw, double *db, int N, int Ci, int D, int H, int W, int Co,
                           int kd, int kh, int kw, int sd, int sh, int sw, int pd, int ph, int pw) {
    if (!x || !w || !dy || check(N, Ci, D, H, W, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw))
        return CONV_ERR_ARG;
    const int Do = out_size(D, kd, sd, pd), Ho = out_size(H, kh, sh, ph), Wo = out_size(W, kw, sw, pw);
    if (dx) memset(dx, 0, sizeof(double) * (size_t)N * Ci * D * H * W);
    if (dw) memset(dw, 0, sizeof(double) * (size_t)Co * Ci * kd * kh * kw);
    if (db) memset(db, 0, sizeof(double) * (size_t)Co);
    for (int n = 0; n < N; n++)
        for (int co = 0; co < Co; co++)
            for (int z = 0; z < Do; z++)
                for (int yy = 0; yy < Ho; yy++)
                    for (int xx = 0; xx < Wo; xx++) {
                        const double g = dy[((((long)n * Co + co) * Do + z) * Ho + yy) * Wo + xx];
                        if (db) db[co] += g;
                        for (int ci = 0; ci < Ci; ci++)
                            for (int a = 0; a < kd; a++) {
                                const int iz = z * sd + a - pd;
                                if (iz < 0 || iz >= D) continue;
                                for (int bb = 0; bb < kh; bb++) {
                                    const int iy = yy * sh + bb - ph;
                                    if (iy < 0 || iy >= H) continue;
                                    for (int c = 0; c < kw; c++) {
                                        const int ix = xx * sw + c - pw;
                                        if (ix < 0 || ix >= W) continue;
                                        const long wi = ((((long)co * Ci + ci) * kd + a) * kh + bb) * kw + c;
                                        const long xi = ((((long)n * Ci + ci) * D + iz) * H + iy) * W + ix;
                                        if (dx) dx[xi] += w[wi] * g;
                                        if (dw) dw[wi] += x[xi] * g;
                                    }
                                }
                            }
                    }
    return 0;
}
