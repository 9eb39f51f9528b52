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

}  // namespace bpm
