// PSF readout of a multiplexed run: the idealised refocusing lens of the
// detection path.  The exit field of a march that started at the source plane
// `back` slices earlier is brought back to the source plane in free space,
// cut by the detection pupil (NA), refocused to `planes` planes around it,
// and every source's crop x crop window is cut out of each plane's intensity:
//
//   S    = DFT2(u) . P . exp(-i kz back dz)
//   E_m  = IDFT2( S . exp(i kz m dz) ),  m = -planes/2 .. planes/2 - 1
//   psf[s][m + planes/2][y][x] = scale |E_m(sy - crop/2 + y, sx - crop/2 + x)|^2
//
// Launches: the natural-order DFT of u (fft2), one launch over (column tile,
// plane) for the pupil, the refocus phase and the column IDFT, one over
// (row unit, plane) for the row IDFT and |.|^2, and the crop gather.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "passes.hpp"

namespace bpm {

template <int NY>
__global__ __launch_bounds__(kBlock) void readout_cols_kernel(
    const float2* __restrict__ S, float2* __restrict__ T, int nx, int ny, double dx, double dz,
    double k, double pthr, int back, int planes, const float2* __restrict__ tw,
    const int* __restrict__ permy) {
    constexpr int T_ = NY / kR, W = units_per_block<NY>();
    extern __shared__ float2 smem[];
    const double kPi = 3.14159265358979323846;
    const int w = threadIdx.x % W, t = threadIdx.x / W;
    const int c = blockIdx.x * W + w;
    const int plane = blockIdx.y;
    const bool on = c < nx;
    const int col = on ? c : 0;
    const int mz = plane - planes / 2;
    Twiddles<NY, kR> twy;
    twy.load(tw, t);
    const long ms = col < nx / 2 ? col : col - nx;
    const double kx = 2.0 * kPi * (double)ms / (nx * dx);
    float2 v[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) {
        const int l = i * T_ + t;
        const long ls = l < ny / 2 ? l : l - ny;
        const long a = ms * ny, b = ls * nx;
        float2 z = make_float2(0.f, 0.f);
        if ((double)(a * a + b * b) <= pthr) {
            const double ky = 2.0 * kPi * (double)ls / (ny * dx);
            const double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
            double sv, cv;
            sincos(kz * (double)(mz - back) * dz, &sv, &cv);
            const float2 s = S[(size_t)l * nx + col];
            z = c_mul(s, make_float2((float)cv, (float)sv));
        }
        v[i] = c_conj(z);  // inverse DFT as conj(DFT(conj))
    }
    fft_forward<NY, kR, W>(v, smem + w, t, twy, BlockSync());
    if (on) {
        float2* Tp = T + (size_t)plane * nx * ny;
#pragma unroll
        for (int r = 0; r < kR; ++r) Tp[(size_t)permy[r * T_ + t] * nx + col] = c_conj(v[r]);
    }
}

template <int NX>
__global__ __launch_bounds__(kBlock) void readout_rows_kernel(const float2* __restrict__ T,
                                                              float* __restrict__ I, int ny,
                                                              float scale,
                                                              const float2* __restrict__ tw,
                                                              const int* __restrict__ permx) {
    constexpr int T_ = NX / kR, B = units_per_block<NX>();
    extern __shared__ float2 smem[];
    const int sub = threadIdx.x / T_, tau = threadIdx.x % T_;
    const int row = blockIdx.x * B + sub;
    const bool on = row < ny;
    const size_t plane_off = (size_t)blockIdx.y * NX * ny;
    const size_t rowoff = plane_off + (size_t)(on ? row : 0) * NX;
    Twiddles<NX, kR> twx;
    twx.load(tw, tau);
    float2 v[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = c_conj(T[rowoff + i * T_ + tau]);
    fft_forward<NX, kR, 1>(v, smem + sub * lds_size<NX>(), tau, twx, BlockSync());
    if (on) {
#pragma unroll
        for (int r = 0; r < kR; ++r) I[rowoff + permx[r * T_ + tau]] = scale * c_abs2(v[r]);
    }
}

// psf[s][p][y][x] = I[p][(sy - crop/2 + y) mod ny][(sx - crop/2 + x) mod nx]
__global__ void readout_crop_kernel(const float* __restrict__ I, const int* __restrict__ src,
                                    int n_src, int nx, int ny, int planes, int crop,
                                    float* __restrict__ psf) {
    const long per = (long)planes * crop * crop;
    const long total = per * n_src;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / per);
        const long r = e % per;
        const int p = (int)(r / (crop * crop));
        const int y = (int)(r / crop % crop), x = (int)(r % crop);
        const int gy = ((src[2 * s] - crop / 2 + y) % ny + ny) % ny;
        const int gx = ((src[2 * s + 1] - crop / 2 + x) % nx + nx) % nx;
        psf[e] = I[((size_t)p * ny + gy) * nx + gx];
    }
}

size_t readout_bytes(int nx, int ny, int planes) {
    const size_t n = (size_t)nx * ny;
    return plan_bytes(nx, ny) + align_up(sizeof(float2) * n) +
           align_up(sizeof(float2) * n * planes) + align_up(sizeof(float) * n * planes);
}

hipError_t launch_readout(const ReadoutArgs& r, void* ws, hipStream_t s) {
    const size_t n = (size_t)r.nx * r.ny;
    char* b = static_cast<char*>(ws);
    const Plan p = plan_carve(b, r.nx, r.ny);
    b += plan_bytes(r.nx, r.ny);
    float2* S = (float2*)b;
    b += align_up(sizeof(float2) * n);
    float2* T = (float2*)b;
    b += align_up(sizeof(float2) * n * r.planes);
    float* I = (float*)b;
    const Geom g{r.nx, r.ny, 0, r.dx, r.dz, r.wavelength, r.n0};
    hipError_t e = launch_plan(g, p, false, s);
    if (e == hipSuccess) e = launch_fft2(r.exit_field, S, r.nx, r.ny, false, 1.0f, p, s);
    if (e != hipSuccess) return e;
    const double kPi = 3.14159265358979323846;
    const double k = 2.0 * kPi * r.n0 / r.wavelength;
    double pthr = (double)r.nx * (double)r.ny * r.na * r.dx / r.wavelength;
    pthr *= pthr;
    const double nn = (double)r.nx * r.ny;
    const float scale = (float)(r.scale / (nn * nn));
    auto cols = [&](auto yc) -> hipError_t {
        constexpr int NY = decltype(yc)::value, W = units_per_block<NY>();
        readout_cols_kernel<NY><<<dim3((r.nx + W - 1) / W, r.planes), kBlock,
                                  sizeof(float2) * W * lds_size<NY>(), s>>>(
            S, T, r.nx, r.ny, r.dx, r.dz, k, pthr, r.back_steps, r.planes,
            (const float2*)p.twy, (const int*)p.permy);
        return hipGetLastError();
    };
    auto rows = [&](auto xc) -> hipError_t {
        constexpr int NX = decltype(xc)::value, B = units_per_block<NX>();
        readout_rows_kernel<NX><<<dim3((r.ny + B - 1) / B, r.planes), kBlock,
                                  sizeof(float2) * B * lds_size<NX>(), s>>>(
            T, I, r.ny, scale, (const float2*)p.twx, (const int*)p.permx);
        return hipGetLastError();
    };
    e = dispatch_size(r.ny, cols);
    if (e == hipSuccess) e = dispatch_size(r.nx, rows);
    if (e != hipSuccess || r.n_src == 0) return e;
    const long total = (long)r.n_src * r.planes * r.crop * r.crop;
    const long blocks = (total + 255) / 256;
    readout_crop_kernel<<<(unsigned)(blocks < 65535 ? blocks : 65535), 256, 0, s>>>(
        I, r.sources, r.n_src, r.nx, r.ny, r.planes, r.crop, r.psf_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pupil fields and Zernike fits of the sample-induced aberrations.
//
//   E0     = IDFT2( DFT2(u) . P . exp(-i kz back dz) )       (complex, 1 / (nx ny))
//   X_s    = DFT2 of the crop x crop window of E0 whose centre (index crop/2)
//            is source s
//   fit    : on the disc D of the window's DFT grid, Y = X (-1)^(l+m); tilt
//            t_x = arg sum Y(l, m+1) conj Y(l, m), t_y likewise, piston p0;
//            T = t_x m' + t_y l' + p0, W = wrap(arg Y - T) + T; c = P W then
//            twice c += P wrap(W - Z c); rms = sqrt(mean_D wrap(W - Z c)^2),
//            Z the Noll-normalised Zernike polynomials on D, P = (Z^T Z)^-1 Z^T.

// complex row IDFT of the column pass output: E = scale * IDFT_rows(T)
template <int NX>
__global__ __launch_bounds__(kBlock) void refocus_rows_kernel(const float2* __restrict__ T,
                                                              float2* __restrict__ E, int ny,
                                                              float scale,
                                                              const float2* __restrict__ tw,
                                                              const int* __restrict__ permx) {
    constexpr int T_ = NX / kR, B = units_per_block<NX>();
    extern __shared__ float2 smem[];
    const int sub = threadIdx.x / T_, tau = threadIdx.x % T_;
    const int row = blockIdx.x * B + sub;
    const bool on = row < ny;
    const size_t rowoff = (size_t)(on ? row : 0) * NX;
    Twiddles<NX, kR> twx;
    twx.load(tw, tau);
    float2 v[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = c_conj(T[rowoff + i * T_ + tau]);
    fft_forward<NX, kR, 1>(v, smem + sub * lds_size<NX>(), tau, twx, BlockSync());
    if (on) {
#pragma unroll
        for (int r = 0; r < kR; ++r)
            E[rowoff + permx[r * T_ + tau]] = make_float2(scale * v[r].x, -scale * v[r].y);
    }
}

constexpr int kAbBlock = 256;

// z + a b
__device__ __forceinline__ float2 c_fma(float2 a, float2 b, float2 z) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, z.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, z.y)));
}

// X_s: gather the C x C window of E around source s, then its 2-D DFT
// (row and column DFTs as direct sums over an LDS-resident window).
template <int C>
__global__ __launch_bounds__(kAbBlock) void pupil_crop_kernel(const float2* __restrict__ E,
                                                              const int* __restrict__ src,
                                                              int nx, int ny,
                                                              float2* __restrict__ out) {
    constexpr int CC = C * C, PER = (CC + kAbBlock - 1) / kAbBlock, LD = C + 1;
    __shared__ float2 a[C * LD];
    __shared__ float2 tw[C];
    const int s = blockIdx.x;
    const int sy = src[2 * s], sx = src[2 * s + 1];
    for (int i = threadIdx.x; i < C; i += kAbBlock) {
        double sv, cv;
        sincospi(-2.0 * i / C, &sv, &cv);
        tw[i] = make_float2((float)cv, (float)sv);
    }
    for (int e = threadIdx.x; e < CC; e += kAbBlock) {
        const int y = e / C, x = e % C;
        const int gy = ((sy - C / 2 + y) % ny + ny) % ny;
        const int gx = ((sx - C / 2 + x) % nx + nx) % nx;
        a[y * LD + x] = E[(size_t)gy * nx + gx];
    }
    __syncthreads();
    float2 acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        float2 z = make_float2(0.f, 0.f);
        if (e < CC) {
            const int y = e / C, m = e % C;
            for (int x = 0; x < C; ++x) z = c_fma(a[y * LD + x], tw[(m * x) & (C - 1)], z);
        }
        acc[q] = z;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        if (e < CC) a[(e / C) * LD + e % C] = acc[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        if (e < CC) {
            const int l = e / C, m = e % C;
            float2 z = make_float2(0.f, 0.f);
            for (int y = 0; y < C; ++y) z = c_fma(a[y * LD + m], tw[(l * y) & (C - 1)], z);
            out[(size_t)s * CC + e] = z;
        }
    }
}

// Noll index j >= 1 -> (n, m), m < 0 for the sine terms (odd j)
__device__ inline void noll_nm(int j, int& n, int& m) {
    int nn = 0;
    while ((nn + 1) * (nn + 2) / 2 < j) ++nn;
    const int k = j - nn * (nn + 1) / 2 - 1;
    int mm = nn % 2 + 2 * ((k + 1 - nn % 2) / 2);
    if (mm != 0 && (j & 1)) mm = -mm;
    n = nn;
    m = mm;
}

__device__ inline double factorial_d(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// Noll-normalised Zernike polynomials Z_1 .. Z_J at one point, into z[]
// (radial powers by repeated multiplication; n <= 6 for J <= 28)
__device__ void zernike_all(int J, double rho, double theta, double* z) {
    double rp[7];
    rp[0] = 1.0;
    for (int k = 1; k < 7; ++k) rp[k] = rp[k - 1] * rho;
    for (int j = 0; j < J; ++j) {
        int n, m;
        noll_nm(j + 1, n, m);
        const int am = m < 0 ? -m : m;
        double r = 0.0;
        for (int s = 0; s <= (n - am) / 2; ++s)
            r += ((s & 1) ? -1.0 : 1.0) * factorial_d(n - s) /
                 (factorial_d(s) * factorial_d((n + am) / 2 - s) * factorial_d((n - am) / 2 - s)) *
                 rp[n - 2 * s];
        z[j] = m == 0 ? sqrt((double)(n + 1)) * r
                      : sqrt(2.0 * (n + 1)) * r * (m > 0 ? cos(am * theta) : sin(am * theta));
    }
}

// One workgroup: the basis Z [J][C*C] on the disc (zero outside) and the
// least-squares operator P = (Z^T Z)^-1 Z^T [J][C*C], both float; Zd is a
// double scratch [J][C*C].  R = NA C dx / lambda.  The Gram matrix is summed
// over chunks of kAbBlock samples staged in LDS (one sample per thread) and
// inverted by the whole workgroup (Gauss-Jordan, one pivot per round).
template <int C>
__global__ __launch_bounds__(kAbBlock) void zernike_basis_kernel(int J, double R,
                                                                 double* __restrict__ Zd,
                                                                 float* __restrict__ Zf,
                                                                 float* __restrict__ Pf,
                                                                 int* __restrict__ ok) {
    constexpr int CC = C * C;
    constexpr int W2 = 2 * kMaxZernike;
    __shared__ double A[kMaxZernike * W2];  // [G | I] -> [I | G^-1] by Gauss-Jordan
    __shared__ double zs[kAbBlock * kMaxZernike];
    __shared__ int s_bad;
    const int npairs = J * (J + 1) / 2;
    double gacc[2] = {0.0, 0.0};  // pairs threadIdx.x and threadIdx.x + kAbBlock
    int pa[2], pb[2];
    for (int q = 0; q < 2; ++q) {
        int p = threadIdx.x + q * kAbBlock, a = 0;
        while (p > a) {  // pair p = (a, b), b <= a, in row-major lower-triangle order
            p -= a + 1;
            ++a;
        }
        pa[q] = a;
        pb[q] = p;
    }
    for (int c0 = 0; c0 < CC; c0 += kAbBlock) {
        const int i = c0 + threadIdx.x;
        double z[kMaxZernike];
        const int l = i / C, m = i % C;
        const int ls = l < C / 2 ? l : l - C, ms = m < C / 2 ? m : m - C;
        const bool in = i < CC && (double)(ls * ls + ms * ms) <= R * R;
        if (in)
            zernike_all(J, sqrt((double)(ls * ls + ms * ms)) / R, atan2((double)ls, (double)ms), z);
        for (int j = 0; j < J; ++j) {
            const double v = in ? z[j] : 0.0;
            zs[threadIdx.x * kMaxZernike + j] = v;
            if (i < CC) {
                Zd[(size_t)j * CC + i] = v;
                Zf[(size_t)j * CC + i] = (float)v;
            }
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            if (threadIdx.x + q * kAbBlock < npairs) {
                double acc = gacc[q];
                for (int t = 0; t < kAbBlock; ++t)
                    acc += zs[t * kMaxZernike + pa[q]] * zs[t * kMaxZernike + pb[q]];
                gacc[q] = acc;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < J * W2; e += kAbBlock) {
        const int r = e / W2, c = e % W2;
        A[r * W2 + c] = c >= J ? (c - J == r ? 1.0 : 0.0) : 0.0;
    }
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
        if (threadIdx.x + q * kAbBlock < npairs) {
            A[pa[q] * W2 + pb[q]] = gacc[q];
            A[pb[q] * W2 + pa[q]] = gacc[q];
        }
    }
    // Gauss-Jordan on [G | I]: G is symmetric positive definite, so the
    // pivots of the unpivoted elimination are positive exactly when the
    // basis is not singular on the disc
    constexpr int PER = (kMaxZernike * W2 + kAbBlock - 1) / kAbBlock;
    for (int k = 0; k < J; ++k) {
        __syncthreads();
        const double piv = A[k * W2 + k];
        if (!(piv > 0.0)) {
            if (threadIdx.x == 0) s_bad = 1;
            break;
        }
        double ark[PER], akc[PER], arc[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * kAbBlock;
            if (e < J * W2) {
                const int r = e / W2, c = e % W2;
                ark[q] = A[r * W2 + k];
                akc[q] = A[k * W2 + c];
                arc[q] = A[r * W2 + c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * kAbBlock;
            if (e < J * W2) {
                const int r = e / W2, c = e % W2;
                const double t = akc[q] / piv;
                A[r * W2 + c] = r == k ? t : arc[q] - ark[q] * t;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *ok = s_bad ? 0 : 1;
    for (int i = threadIdx.x; i < CC; i += kAbBlock) {
        double z[kMaxZernike];
        for (int k = 0; k < J; ++k) z[k] = Zd[(size_t)k * CC + i];
        for (int j = 0; j < J; ++j) {
            double acc = 0.0;
            for (int k = 0; k < J; ++k) acc += A[j * W2 + J + k] * z[k];
            Pf[(size_t)j * CC + i] = (float)acc;
        }
    }
}

// sum of K values over the workgroup; every thread gets the totals in out
template <int K>
__device__ inline void block_sum(float (&v)[K], float* red, float* out) {
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) red[wave * K + k] = x;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        float t = 0.f;
        for (int w = 0; w < kAbBlock / 64; ++w) t += red[w * K + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

__device__ inline float wrap_pi(float p) {
    const float kPi = 3.14159265358979f;
    return p - 2.f * kPi * floorf((p + kPi) / (2.f * kPi));
}

// one workgroup per source
template <int C>
__global__ __launch_bounds__(kAbBlock) void zernike_fit_kernel(const float2* __restrict__ X,
                                                               int J, double R, int disc_n,
                                                               const float* __restrict__ Zf,
                                                               const float* __restrict__ Pf,
                                                               float* __restrict__ coeffs,
                                                               float* __restrict__ rms) {
    constexpr int CC = C * C, PER = (CC + kAbBlock - 1) / kAbBlock;
    __shared__ float red[(kAbBlock / 64) * kMaxZernike];
    __shared__ float tot[kMaxZernike];
    const int s = blockIdx.x;
    const float2* Xs = X + (size_t)s * CC;
    auto inside = [&](int l, int m) {
        const int ls = l < C / 2 ? l : l - C, ms = m < C / 2 ? m : m - C;
        return (double)(ls * ls + ms * ms) <= R * R;
    };
    auto Yat = [&](int l, int m) {
        const float2 x = Xs[l * C + m];
        return ((l + m) & 1) ? make_float2(-x.x, -x.y) : x;
    };
    float W[PER];
    bool in[PER];
    // tilt
    float t4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        in[q] = false;
        if (e < CC) {
            const int l = e / C, m = e % C;
            in[q] = inside(l, m);
            if (in[q]) {
                const float2 y = Yat(l, m);
                const int m1 = (m + 1) & (C - 1), l1 = (l + 1) & (C - 1);
                if (inside(l, m1)) {
                    const float2 z = c_mul(Yat(l, m1), c_conj(y));
                    t4[0] += z.x;
                    t4[1] += z.y;
                }
                if (inside(l1, m)) {
                    const float2 z = c_mul(Yat(l1, m), c_conj(y));
                    t4[2] += z.x;
                    t4[3] += z.y;
                }
            }
        }
    }
    block_sum<4>(t4, red, tot);
    const float tx = atan2f(tot[1], tot[0]), ty = atan2f(tot[3], tot[2]);
    // piston
    float p2[2] = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        if (in[q]) {
            const int l = e / C, m = e % C;
            const int ls = l < C / 2 ? l : l - C, ms = m < C / 2 ? m : m - C;
            float sv, cv;
            sincosf(-(tx * ms + ty * ls), &sv, &cv);
            const float2 z = c_mul(Yat(l, m), make_float2(cv, sv));
            p2[0] += z.x;
            p2[1] += z.y;
        }
    }
    block_sum<2>(p2, red, tot);
    const float p0 = atan2f(tot[1], tot[0]);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        W[q] = 0.f;
        if (in[q]) {
            const int l = e / C, m = e % C;
            const int ls = l < C / 2 ? l : l - C, ms = m < C / 2 ? m : m - C;
            const float T = tx * ms + ty * ls + p0;
            const float2 y = Yat(l, m);
            W[q] = wrap_pi(atan2f(y.y, y.x) - T) + T;
        }
    }
    // c = P W, then two passes c += P wrap(W - Z c)
    float c[kMaxZernike];
    for (int j = 0; j < kMaxZernike; ++j) c[j] = 0.f;
    for (int pass = 0; pass < 3; ++pass) {
        float part[kMaxZernike];
        for (int j = 0; j < kMaxZernike; ++j) part[j] = 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * kAbBlock;
            if (in[q]) {
                float r = W[q];
                if (pass > 0) {
                    float zc = 0.f;
                    for (int j = 0; j < J; ++j) zc += Zf[(size_t)j * CC + e] * c[j];
                    r = wrap_pi(W[q] - zc);
                }
                for (int j = 0; j < J; ++j) part[j] += Pf[(size_t)j * CC + e] * r;
            }
        }
        block_sum<kMaxZernike>(part, red, tot);
        for (int j = 0; j < J; ++j) c[j] += tot[j];
    }
    float e2[1] = {0.f};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * kAbBlock;
        if (in[q]) {
            float zc = 0.f;
            for (int j = 0; j < J; ++j) zc += Zf[(size_t)j * CC + e] * c[j];
            const float r = wrap_pi(W[q] - zc);
            e2[0] += r * r;
        }
    }
    block_sum<1>(e2, red, tot);
    if (threadIdx.x < J) coeffs[(size_t)s * J + threadIdx.x] = c[threadIdx.x];
    if (threadIdx.x == 0 && rms) rms[s] = sqrtf(tot[0] / (float)disc_n);
}

size_t pupil_fields_bytes(int nx, int ny) {
    const size_t n = (size_t)nx * ny;
    return plan_bytes(nx, ny) + 2 * align_up(sizeof(float2) * n);
}

hipError_t launch_pupil_fields(const PupilFieldArgs& r, void* ws, hipStream_t s) {
    const size_t n = (size_t)r.nx * r.ny;
    char* b = static_cast<char*>(ws);
    const Plan p = plan_carve(b, r.nx, r.ny);
    b += plan_bytes(r.nx, r.ny);
    float2* S = (float2*)b;
    b += align_up(sizeof(float2) * n);
    float2* T = (float2*)b;
    const Geom g{r.nx, r.ny, 0, r.dx, r.dz, r.wavelength, r.n0};
    hipError_t e = launch_plan(g, p, false, s);
    if (e == hipSuccess) e = launch_fft2(r.exit_field, S, r.nx, r.ny, false, 1.0f, p, s);
    if (e != hipSuccess) return e;
    const double kPi = 3.14159265358979323846;
    const double k = 2.0 * kPi * r.n0 / r.wavelength;
    double pthr = (double)r.nx * (double)r.ny * r.na * r.dx / r.wavelength;
    pthr *= pthr;
    const float scale = (float)(1.0 / ((double)r.nx * r.ny));
    auto cols = [&](auto yc) -> hipError_t {
        constexpr int NY = decltype(yc)::value, W = units_per_block<NY>();
        readout_cols_kernel<NY><<<dim3((r.nx + W - 1) / W, 1), kBlock,
                                  sizeof(float2) * W * lds_size<NY>(), s>>>(
            S, T, r.nx, r.ny, r.dx, r.dz, k, pthr, r.back_steps, 1, (const float2*)p.twy,
            (const int*)p.permy);
        return hipGetLastError();
    };
    // E overwrites S (the spectrum is no longer needed after the column pass)
    auto rows = [&](auto xc) -> hipError_t {
        constexpr int NX = decltype(xc)::value, B = units_per_block<NX>();
        refocus_rows_kernel<NX><<<(r.ny + B - 1) / B, kBlock, sizeof(float2) * B * lds_size<NX>(),
                                  s>>>(T, S, r.ny, scale, (const float2*)p.twx,
                                       (const int*)p.permx);
        return hipGetLastError();
    };
    e = dispatch_size(r.ny, cols);
    if (e == hipSuccess) e = dispatch_size(r.nx, rows);
    if (e != hipSuccess || r.n_src == 0) return e;
    switch (r.crop) {
        case 16:
            pupil_crop_kernel<16><<<r.n_src, kAbBlock, 0, s>>>(S, r.sources, r.nx, r.ny,
                                                               (float2*)r.pupil_out);
            break;
        case 32:
            pupil_crop_kernel<32><<<r.n_src, kAbBlock, 0, s>>>(S, r.sources, r.nx, r.ny,
                                                               (float2*)r.pupil_out);
            break;
        case 64:
            pupil_crop_kernel<64><<<r.n_src, kAbBlock, 0, s>>>(S, r.sources, r.nx, r.ny,
                                                               (float2*)r.pupil_out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t zernike_bytes(int crop, int n_modes) {
    const size_t cc = (size_t)crop * crop * n_modes;
    return align_up(sizeof(double) * cc) + 2 * align_up(sizeof(float) * cc) + 256;
}

hipError_t launch_zernike_fit(const ZernikeArgs& a, void* ws, int* host_ok, hipStream_t s) {
    const size_t cc = (size_t)a.crop * a.crop * a.n_modes;
    char* b = static_cast<char*>(ws);
    double* Zd = (double*)b;
    b += align_up(sizeof(double) * cc);
    float* Zf = (float*)b;
    b += align_up(sizeof(float) * cc);
    float* Pf = (float*)b;
    b += align_up(sizeof(float) * cc);
    int* ok = (int*)b;
    const double R = a.na * a.crop * a.dx / a.wavelength;
    auto run = [&](auto cc_) -> hipError_t {
        constexpr int C = decltype(cc_)::value;
        zernike_basis_kernel<C><<<1, kAbBlock, 0, s>>>(a.n_modes, R, Zd, Zf, Pf, ok);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (a.n_src > 0)
            zernike_fit_kernel<C><<<a.n_src, kAbBlock, 0, s>>>(
                (const float2*)a.pupil, a.n_modes, R, a.disc_n, Zf, Pf, a.coeffs_out, a.rms_out);
        e = hipGetLastError();
        if (e == hipSuccess && host_ok) {
            e = hipMemcpyAsync(host_ok, ok, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        return e;
    };
    switch (a.crop) {
        case 16: return run(std::integral_constant<int, 16>{});
        case 32: return run(std::integral_constant<int, 32>{});
        case 64: return run(std::integral_constant<int, 64>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bpm
