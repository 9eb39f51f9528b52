/*
 * FP64 CPU oracle for the split-step beam-propagation march.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) links, loads or calls this file; only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
 * with the GPU path: its own radix-2 FFT, its own propagator, its own loops.
 *
 * What it computes (Weigert, Myers & Kreysing, arXiv 1706.02261, main text,
 * the paragraph on the beam-propagation model: BPM after refs. [20-22] with
 * the exact, non-paraxial propagator, and the multiplexed field of the same
 * paragraph).  The paper prints no step equations; the recursion below is the
 * textbook split-step scheme in the order "propagate, then phase screen":
 *
 *   k0 = 2 pi / lambda,  k = n0 k0,
 *   kx = 2 pi m~ / (Nx dx),  ky = 2 pi l~ / (Ny dx),   m~, l~ signed indices,
 *   H[l][m] = exp(i dz sqrt(k^2 - kx^2 - ky^2))  if kx^2 + ky^2 <= k^2, else 0,
 *   for j = 0 .. steps-1:
 *       v       = IDFT2( H * DFT2(u_j) )
 *       u_{j+1} = exp(i k0 dz dn[j]) * v
 *       I[j]    = |u_{j+1}|^2
 *
 * DFT: X[k] = sum_n x[n] exp(-2 pi i n k / N); IDFT carries exp(+...) and 1/N.
 * The propagating test is done on integers (see prop_mask) so it cannot
 * disagree with another implementation by rounding.
 *
 * The adjoint (gradients in PyTorch's convention g = dL/dRe + i dL/dIm) runs
 * the same recursion backwards, storing every forward field:
 *
 *   g_N = grad_u_out (or 0)
 *   for j = N-1 .. 0:
 *       g_{j+1} += 2 gI[j] u_{j+1}
 *       grad_dn[j] = k0 dz Im(g_{j+1} conj(u_{j+1}))
 *       w   = conj(S_j) g_{j+1}
 *       g_j = IDFT2( conj(H) * DFT2(w) )
 *   grad_u0 = g_0,  grad_spectrum0 = DFT2(g_0) / (Nx Ny)
 *
 * Arrays: complex values are interleaved (re, im) doubles; fields [ny][nx],
 * volumes [steps][ny][nx], x fastest.  Every entry point returns 0 on success
 * and a negative value for invalid arguments.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_MEM (-2)

static const double PI = 3.14159265358979323846264338327950288;

static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

/* ------------------------------------------------------------------------ */
/* radix-2 FFT                                                              */

/* twiddle table w[t] = exp(sign 2 pi i t / n), t < n/2, from cos/sin in double */
static cplx *twiddles(int n, int sign) {
    int half = n / 2 > 0 ? n / 2 : 1;
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)half);
    if (!w) return NULL;
    for (int t = 0; t < half; t++) {
        double a = sign * 2.0 * PI * (double)t / (double)n;
        w[t] = cos(a) + I * sin(a);
    }
    return w;
}

/* In-place iterative Cooley-Tukey, decimation in time: bit-reversal
 * permutation, then log2(n) butterfly stages.  a[i*stride], i < n. */
static void fft1d(cplx *a, int n, long stride, const cplx *w) {
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = a[i * stride];
            a[i * stride] = a[j * stride];
            a[j * stride] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int s = 0; s < n; s += len) {
            for (int k = 0; k < half; k++) {
                cplx x = a[(s + k) * stride];
                cplx y = a[(s + k + half) * stride] * w[k * step];
                a[(s + k) * stride] = x + y;
                a[(s + k + half) * stride] = x - y;
            }
        }
    }
}

/* unnormalised 2-D transform of u[ny][nx]: rows, then columns */
static int fft2d(cplx *u, int nx, int ny, int sign) {
    cplx *wx = twiddles(nx, sign), *wy = twiddles(ny, sign);
    if (!wx || !wy) { free(wx); free(wy); return ORACLE_ERR_MEM; }
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++) fft1d(u + (long)y * nx, nx, 1, wx);
    #pragma omp parallel
    {
        cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
        #pragma omp for schedule(static)
        for (int x = 0; x < nx; x++) {
            for (int y = 0; y < ny; y++) col[y] = u[(long)y * nx + x];
            fft1d(col, ny, 1, wy);
            for (int y = 0; y < ny; y++) u[(long)y * nx + x] = col[y];
        }
        free(col);
    }
    free(wx); free(wy);
    return 0;
}

int oracle_fft1d(double *data, int n, int sign) {
    if (!data || !is_pow2(n) || (sign != 1 && sign != -1)) return ORACLE_ERR_ARG;
    cplx *w = twiddles(n, sign);
    if (!w) return ORACLE_ERR_MEM;
    fft1d((cplx *)data, n, 1, w);
    free(w);
    return 0;
}

int oracle_fft2d(double *data, int nx, int ny, int sign) {
    if (!data || !is_pow2(nx) || !is_pow2(ny) || (sign != 1 && sign != -1)) return ORACLE_ERR_ARG;
    return fft2d((cplx *)data, nx, ny, sign);
}

/* ------------------------------------------------------------------------ */
/* propagator                                                               */

static long signed_index(long i, long n) { return i < n / 2 ? i : i - n; }

/* kx^2 + ky^2 <= k^2  <=>  (m~ Ny)^2 + (l~ Nx)^2 <= (Nx Ny n0 dx / lambda)^2.
 * The left side is an exact integer (< 2^44 for sizes up to 2048). */
static int prop_mask(long m, long l, int nx, int ny, double thr) {
    long a = signed_index(m, nx) * ny, b = signed_index(l, ny) * nx;
    return (double)(a * a + b * b) <= thr;
}

static double mask_threshold(int nx, int ny, double dx, double lam, double n0) {
    double t = (double)nx * (double)ny * n0 * dx / lam;
    return t * t;
}

/* H[l][m] (no 1/(Nx Ny) folded in) */
int oracle_propagator(int nx, int ny, double dx, double dz, double lam, double n0, double *h) {
    if (!h || !is_pow2(nx) || !is_pow2(ny) || !(dx > 0) || !(lam > 0) || !(n0 > 0)) return ORACLE_ERR_ARG;
    cplx *H = (cplx *)h;
    double k0 = 2.0 * PI / lam, k = n0 * k0, thr = mask_threshold(nx, ny, dx, lam, n0);
    for (int l = 0; l < ny; l++) {
        double ky = 2.0 * PI * (double)signed_index(l, ny) / (ny * dx);
        for (int m = 0; m < nx; m++) {
            double kx = 2.0 * PI * (double)signed_index(m, nx) / (nx * dx);
            cplx v = 0.0;
            if (prop_mask(m, l, nx, ny, thr)) {
                double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
                v = cos(dz * kz) + I * sin(dz * kz);
            }
            H[(long)l * nx + m] = v;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* forward march                                                            */

static int check_geom(int nx, int ny, int steps, double dx, double dz, double lam, double n0) {
    if (!is_pow2(nx) || !is_pow2(ny) || steps < 0) return ORACLE_ERR_ARG;
    if (!(dx > 0) || !isfinite(dz) || !(lam > 0) || !(n0 > 0)) return ORACLE_ERR_ARG;
    return 0;
}

/* one step u <- S_j * IDFT2(H * DFT2(u)) */
/* one step; the screen uses dn[j] - ref (ref = 0 in the plain march) */
static int step_forward_ref(cplx *u, const cplx *H, const double *dn_j, double ref, int nx, int ny,
                            double k0dz) {
    long n = (long)nx * ny;
    int rc = fft2d(u, nx, ny, -1);
    if (rc) return rc;
    for (long i = 0; i < n; i++) u[i] *= H[i];
    rc = fft2d(u, nx, ny, +1);
    if (rc) return rc;
    double inv = 1.0 / (double)n;
    for (long i = 0; i < n; i++) {
        double ph = k0dz * (dn_j[i] - ref);
        u[i] *= inv * (cos(ph) + I * sin(ph));
    }
    return 0;
}

static int step_forward(cplx *u, const cplx *H, const double *dn_j, int nx, int ny, double k0dz) {
    return step_forward_ref(u, H, dn_j, 0.0, nx, ny, k0dz);
}

int oracle_bpm_forward(const double *u0, const double *dn, int nx, int ny, int steps,
                       double dx, double dz, double lam, double n0,
                       double *u_out, double *intensity_out) {
    int rc = check_geom(nx, ny, steps, dx, dz, lam, n0);
    if (rc) return rc;
    if (!u0 || !u_out || (steps > 0 && !dn)) return ORACLE_ERR_ARG;
    long n = (long)nx * ny;
    cplx *H = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!H || !u) { free(H); free(u); return ORACLE_ERR_MEM; }
    oracle_propagator(nx, ny, dx, dz, lam, n0, (double *)H);
    memcpy(u, u0, sizeof(cplx) * (size_t)n);
    double k0dz = 2.0 * PI / lam * dz;
    for (int j = 0; j < steps && rc == 0; j++) {
        rc = step_forward(u, H, dn + (long)j * n, nx, ny, k0dz);
        if (intensity_out)
            for (long i = 0; i < n; i++) {
                double re = creal(u[i]), im = cimag(u[i]);
                intensity_out[(long)j * n + i] = re * re + im * im;
            }
    }
    if (rc == 0) memcpy(u_out, u, sizeof(cplx) * (size_t)n);
    free(H); free(u);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* adjoint march                                                            */

/*
 * Locally adapted expansion of the refractive index (main text, paragraph on
 * the beam-propagation model: the exact propagator is used "together with a
 * locally adapted expansion of refractive indices"; the details sit in
 * supplementary notes that are not part of the text).  Reading used here:
 * slice j is expanded about its own reference index nr_j = n0 + dn_ref[j]
 * instead of n0.  The step propagates with the exact propagator of a
 * homogeneous medium of index nr_j, evanescent modes cut at kt^2 <= (nr_j k0)^2
 * (integer test as prop_mask with nr_j in place of n0), and the screen carries
 * only the remainder:
 *
 *   v       = IDFT2( H_j * DFT2(u_j) ),  H_j = exp(i dz sqrt((nr_j k0)^2 - kt^2))
 *   u_{j+1} = exp(i k0 dz (dn[j] - dn_ref[j])) * v
 *   I[j]    = |u_{j+1}|^2
 *
 * A slice that is homogeneous at nr_j is then propagated exactly; with
 * dn_ref = 0 this is oracle_bpm_forward.
 */
int oracle_bpm_forward_adapted(const double *u0, const double *dn, const double *dn_ref, int nx,
                               int ny, int steps, double dx, double dz, double lam, double n0,
                               double *u_out, double *intensity_out) {
    int rc = check_geom(nx, ny, steps, dx, dz, lam, n0);
    if (rc) return rc;
    if (!u0 || !u_out || (steps > 0 && (!dn || !dn_ref))) return ORACLE_ERR_ARG;
    for (int j = 0; j < steps; j++)
        if (!(n0 + dn_ref[j] > 0)) return ORACLE_ERR_ARG;
    long n = (long)nx * ny;
    cplx *H = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!H || !u) { free(H); free(u); return ORACLE_ERR_MEM; }
    memcpy(u, u0, sizeof(cplx) * (size_t)n);
    double k0dz = 2.0 * PI / lam * dz;
    for (int j = 0; j < steps && rc == 0; j++) {
        oracle_propagator(nx, ny, dx, dz, lam, n0 + dn_ref[j], (double *)H);
        rc = step_forward_ref(u, H, dn + (long)j * n, dn_ref[j], nx, ny, k0dz);
        if (intensity_out)
            for (long i = 0; i < n; i++) {
                double re = creal(u[i]), im = cimag(u[i]);
                intensity_out[(long)j * n + i] = re * re + im * im;
            }
    }
    if (rc == 0) memcpy(u_out, u, sizeof(cplx) * (size_t)n);
    free(H); free(u);
    return rc;
}

int oracle_bpm_adjoint(const double *u0, const double *dn, int nx, int ny, int steps,
                       double dx, double dz, double lam, double n0,
                       const double *grad_u_out, const double *grad_intensity,
                       double *grad_u0, double *grad_spectrum0, double *grad_dn) {
    int rc = check_geom(nx, ny, steps, dx, dz, lam, n0);
    if (rc) return rc;
    if (!u0 || (steps > 0 && !dn)) return ORACLE_ERR_ARG;
    long n = (long)nx * ny;
    cplx *H = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *us = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(steps + 1));
    cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!H || !us || !g) { free(H); free(us); free(g); return ORACLE_ERR_MEM; }
    oracle_propagator(nx, ny, dx, dz, lam, n0, (double *)H);
    double k0dz = 2.0 * PI / lam * dz;

    /* forward, keeping u_0 .. u_N */
    memcpy(us, u0, sizeof(cplx) * (size_t)n);
    for (int j = 0; j < steps && rc == 0; j++) {
        memcpy(us + (long)(j + 1) * n, us + (long)j * n, sizeof(cplx) * (size_t)n);
        rc = step_forward(us + (long)(j + 1) * n, H, dn + (long)j * n, nx, ny, k0dz);
    }

    /* backward */
    if (grad_u_out) memcpy(g, grad_u_out, sizeof(cplx) * (size_t)n);
    else for (long i = 0; i < n; i++) g[i] = 0.0;
    double inv = 1.0 / (double)n;
    for (int j = steps - 1; j >= 0 && rc == 0; j--) {
        const cplx *u = us + (long)(j + 1) * n;
        const double *dnj = dn + (long)j * n;
        if (grad_intensity)
            for (long i = 0; i < n; i++) g[i] += 2.0 * grad_intensity[(long)j * n + i] * u[i];
        if (grad_dn)
            for (long i = 0; i < n; i++) grad_dn[(long)j * n + i] = k0dz * cimag(g[i] * conj(u[i]));
        for (long i = 0; i < n; i++) {
            double ph = k0dz * dnj[i];
            g[i] *= cos(ph) - I * sin(ph);
        }
        rc = fft2d(g, nx, ny, -1);
        if (rc) break;
        for (long i = 0; i < n; i++) g[i] *= conj(H[i]);
        rc = fft2d(g, nx, ny, +1);
        for (long i = 0; i < n; i++) g[i] *= inv;
    }
    if (rc == 0) {
        if (grad_u0) memcpy(grad_u0, g, sizeof(cplx) * (size_t)n);
        if (grad_spectrum0) {
            rc = fft2d(g, nx, ny, -1);
            for (long i = 0; i < n; i++) g[i] *= inv;
            memcpy(grad_spectrum0, g, sizeof(cplx) * (size_t)n);
        }
    }
    free(H); free(us); free(g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* threading of the OpenMP loops (n <= 0: leave the runtime default)         */

int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* PSF readout of a multiplexed run                                          */
/*
 * The detection path images the source plane through an idealised lens
 * (main-text paragraph on the light-sheet simulation: light of the
 * multiplexed point sources propagated through the sample and a refocusing
 * lens to the camera).  From the exit field u of a march that started at the
 * source plane `back_steps` slices earlier:
 *
 *   S    = DFT2(u) . P . exp(-i kz back_steps dz),  P = [kx^2 + ky^2 <= (k0 NA)^2]
 *   (P evaluated on integers like the propagating test:
 *    (m~ ny)^2 + (l~ nx)^2 <= (nx ny NA dx / lambda)^2)
 *   E_m  = IDFT2( S . exp(i kz m dz) ),   m = -planes/2 .. planes/2 - 1
 *   psf[i][m + planes/2][y][x] = scale |E_m(sy_i - crop/2 + y, sx_i - crop/2 + x)|^2
 *
 * (periodic indices; kz = sqrt(k^2 - kx^2 - ky^2), k = n0 k0).  src holds
 * (sy, sx) pixel pairs.  psf_out: [n_src][planes][crop][crop].
 */
int oracle_psf_readout(const double *exit_field, int nx, int ny, double dx, double dz,
                       double lam, double n0, double na, int back_steps, const int *src,
                       int n_src, int planes, int crop, double scale, double *psf_out) {
    if (!exit_field || !src || !psf_out || !is_pow2(nx) || !is_pow2(ny) || planes < 1 ||
        crop < 1 || n_src < 0 || !(dx > 0) || !(lam > 0) || !(n0 > 0) || !(na > 0))
        return ORACLE_ERR_ARG;
    long n = (long)nx * ny;
    cplx *S = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *E = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!S || !E) { free(S); free(E); return ORACLE_ERR_MEM; }
    memcpy(S, exit_field, sizeof(cplx) * (size_t)n);
    int rc = fft2d(S, nx, ny, -1);
    double k0 = 2.0 * PI / lam, k = n0 * k0;
    double pthr = (double)nx * (double)ny * na * dx / lam;
    pthr *= pthr;
    for (int l = 0; l < ny && rc == 0; l++) {
        double ky = 2.0 * PI * (double)signed_index(l, ny) / (ny * dx);
        for (int m = 0; m < nx; m++) {
            double kx = 2.0 * PI * (double)signed_index(m, nx) / (nx * dx);
            double kt2 = kx * kx + ky * ky;
            long i = (long)l * nx + m;
            if (prop_mask(m, l, nx, ny, pthr)) {
                double kz = sqrt(fmax(k * k - kt2, 0.0));
                double ph = -kz * back_steps * dz;
                S[i] *= cos(ph) + I * sin(ph);
            } else {
                S[i] = 0.0;
            }
        }
    }
    for (int p = 0; p < planes && rc == 0; p++) {
        int mz = p - planes / 2;
        for (int l = 0; l < ny; l++) {
            double ky = 2.0 * PI * (double)signed_index(l, ny) / (ny * dx);
            for (int m = 0; m < nx; m++) {
                double kx = 2.0 * PI * (double)signed_index(m, nx) / (nx * dx);
                double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
                double ph = kz * mz * dz;
                long i = (long)l * nx + m;
                E[i] = S[i] * (cos(ph) + I * sin(ph));
            }
        }
        rc = fft2d(E, nx, ny, +1);
        for (int s = 0; s < n_src && rc == 0; s++) {
            int sy = src[2 * s], sx = src[2 * s + 1];
            for (int y = 0; y < crop; y++) {
                int gy = ((sy - crop / 2 + y) % ny + ny) % ny;
                for (int x = 0; x < crop; x++) {
                    int gx = ((sx - crop / 2 + x) % nx + nx) % nx;
                    cplx e = E[(long)gy * nx + gx] / (double)n;
                    double v = creal(e) * creal(e) + cimag(e) * cimag(e);
                    psf_out[(((long)s * planes + p) * crop + y) * crop + x] = scale * v;
                }
            }
        }
    }
    free(S); free(E);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* multiplexed point-source input field                                     */
/*
 * Diffraction-limited point sources (main-text paragraphs on the detection
 * PSFs and on multiplexing).  One source is the Gaussian-apodised,
 * NA-limited angular spectrum
 *
 *   S(k) = exp(-(kt / (k0 NA))^2) [kt <= k0 NA] exp(-i kz z_d)
 *
 * (pupil by the integer test of the readout, kz = sqrt(k^2 - kt^2)), brought to
 * real space by the inverse DFT and scaled to unit L2 norm:
 * u_src = IDFT2(S) / ||IDFT2(S)||.  The multiplexed field is the weighted sum
 * of its integer circular shifts, evaluated here by the direct double loop
 *
 *   u0[y][x] = sum_i exp(i phase_i) u_src[(y - py_i) mod ny][(x - px_i) mod nx].
 *
 * pos: (py, px) pixel pairs; phases may be NULL (all zero); out: [ny][nx].
 */
int oracle_point_sources(const int *pos, const double *phases, int n_src, int nx, int ny,
                         double dx, double lam, double n0, double na, double z_d, double *out) {
    if (!out || (n_src > 0 && !pos) || n_src < 0 || !is_pow2(nx) || !is_pow2(ny) || !(dx > 0) ||
        !(lam > 0) || !(n0 > 0) || !(na > 0))
        return ORACLE_ERR_ARG;
    long n = (long)nx * ny;
    cplx *src = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!src) return ORACLE_ERR_MEM;
    double k0 = 2.0 * PI / lam, k = n0 * k0, kmax = k0 * na;
    double pthr = (double)nx * (double)ny * na * dx / lam;
    pthr *= pthr;
    for (int l = 0; l < ny; l++) {
        double ky = 2.0 * PI * (double)signed_index(l, ny) / (ny * dx);
        for (int m = 0; m < nx; m++) {
            double kx = 2.0 * PI * (double)signed_index(m, nx) / (nx * dx);
            double kt2 = kx * kx + ky * ky;
            cplx v = 0.0;
            if (prop_mask(m, l, nx, ny, pthr)) {
                double kz = sqrt(fmax(k * k - kt2, 0.0));
                v = exp(-kt2 / (kmax * kmax)) * (cos(kz * z_d) - I * sin(kz * z_d));
            }
            src[(long)l * nx + m] = v;
        }
    }
    int rc = fft2d(src, nx, ny, +1);
    if (rc) { free(src); return rc; }
    double norm2 = 0.0;
    for (long i = 0; i < n; i++) norm2 += creal(src[i]) * creal(src[i]) + cimag(src[i]) * cimag(src[i]);
    double scale = 1.0 / sqrt(norm2);  /* the 1/(nx ny) of the IDFT cancels here */
    cplx *u = (cplx *)out;
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++) {
        for (int x = 0; x < nx; x++) {
            cplx acc = 0.0;
            for (int s = 0; s < n_src; s++) {
                int sy = ((y - pos[2 * s]) % ny + ny) % ny;
                int sx = ((x - pos[2 * s + 1]) % nx + nx) % nx;
                double ph = phases ? phases[s] : 0.0;
                acc += (cos(ph) + I * sin(ph)) * src[(long)sy * nx + sx];
            }
            u[(long)y * nx + x] = acc * scale;
        }
    }
    free(src);
    return 0;
}
