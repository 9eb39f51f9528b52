// Forward split-step march: plan builder, fused row pass, fused column pass.
//
// One step j of the march (propagate, then phase screen) is split into two
// passes over the field, each reading and writing it once:
//
//   column pass j : forward column FFTs  ->  x H (exact propagator, evanescent
//                   modes zero, 1/(nx ny) folded in)  ->  inverse column FFTs
//   row pass j    : inverse row FFTs  ->  x exp(i k0 dz dn[j])  ->  I[j] = |u|^2
//                   ->  forward row FFTs (first half of step j+1's DFT2)
//
// plus a head row pass (forward row FFTs of u_0) and a tail row pass (no
// forward FFT; natural-order u_steps written out).  Between passes the field
// lives in the caller's output buffer with its x axis in the FFT's storage
// order (see fft.hpp); the y axis never leaves a column pass permuted.
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "internal.hpp"
#include "mathx.hpp"

namespace bpm {

constexpr int kR = 16;  // complex values per thread

template <int N>
constexpr int rows_per_block() {
    constexpr int t = N / kR, b = 256 / t;
    return b < 1 ? 1 : (b > 32 ? 32 : b);
}
template <int N>
constexpr int cols_per_block() { return rows_per_block<N>(); }

// ---------------------------------------------------------------------------
// plan

size_t plan_bytes(int nx, int ny) {
    return align_up(sizeof(float2) * (size_t)nx * ny) + align_up(sizeof(float2) * nx) +
           align_up(sizeof(float2) * ny);
}

Plan plan_carve(void* ws, int nx, int ny) {
    char* b = static_cast<char*>(ws);
    Plan p;
    p.H = b;
    b += align_up(sizeof(float2) * (size_t)nx * ny);
    p.twx = b;
    b += align_up(sizeof(float2) * nx);
    p.twy = b;
    return p;
}

__global__ void plan_kernel(float2* __restrict__ H, float2* __restrict__ twx,
                            float2* __restrict__ twy, int nx, int ny, double dx, double dz,
                            double lam, double n0) {
    const double kPi = 3.14159265358979323846;
    const long total = (long)nx * ny + nx + ny;
    const double k0 = 2.0 * kPi / lam, k = n0 * k0;
    const double thr_sqrt = (double)nx * (double)ny * n0 * dx / lam;
    const double thr = thr_sqrt * thr_sqrt;
    const double scale = 1.0 / ((double)nx * (double)ny);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        if (e < (long)nx * ny) {
            const int py = (int)(e / nx), px = (int)(e % nx);
            // storage slot -> frequency index on each axis
            const int m = fft_freq_of_store(nx, kR, px);
            const int l = fft_freq_of_store(ny, kR, py);
            const long ms = m < nx / 2 ? m : m - nx, ls = l < ny / 2 ? l : l - ny;
            const long a = ms * ny, b = ls * nx;
            float2 h = make_float2(0.f, 0.f);
            if ((double)(a * a + b * b) <= thr) {
                const double kx = 2.0 * kPi * (double)ms / (nx * dx);
                const double ky = 2.0 * kPi * (double)ls / (ny * dx);
                const double kz = sqrt(fmax(k * k - kx * kx - ky * ky, 0.0));
                double sv, cv;
                sincos(dz * kz, &sv, &cv);
                h = make_float2((float)(cv * scale), (float)(sv * scale));
            }
            H[e] = h;
        } else {
            const long t = e - (long)nx * ny;
            const int n = t < nx ? nx : ny;
            const long i = t < nx ? t : t - nx;
            double sv, cv;
            sincos(-2.0 * kPi * (double)i / n, &sv, &cv);
            (t < nx ? twx : twy)[i] = make_float2((float)cv, (float)sv);
        }
    }
}

hipError_t launch_plan(const Geom& g, const Plan& p, hipStream_t s) {
    const long total = (long)g.nx * g.ny + g.nx + g.ny;
    const int threads = 256;
    const long blocks = (total + threads - 1) / threads;
    plan_kernel<<<(unsigned)(blocks < 4096 ? blocks : 4096), threads, 0, s>>>(
        (float2*)p.H, (float2*)p.twx, (float2*)p.twy, g.nx, g.ny, g.dx, g.dz, g.wavelength,
        g.n0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// row pass

enum RowMode { kHead = 0, kMid = 1, kTail = 2 };

template <int NX, int MODE>
__global__ __launch_bounds__(256) void row_pass(const float2* src, float2* dst,
                                                const float* __restrict__ dn,
                                                float* __restrict__ inten,
                                                const float2* __restrict__ twx, float k0dz) {
    constexpr int T = NX / kR, B = rows_per_block<NX>();
    extern __shared__ float2 smem[];
    const int sub = threadIdx.x / T, tau = threadIdx.x % T;
    const size_t rowoff = (size_t)(blockIdx.x * B + sub) * NX;
    float2* lds = smem + sub * lds_size<NX>();
    auto sync = [] { __syncthreads(); };
    float2 v[kR];
    if constexpr (MODE == kHead) {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = src[rowoff + i * T + tau];
    } else {
#pragma unroll
        for (int r = 0; r < kR; ++r) v[r] = src[rowoff + r * T + tau];
        fft_inverse<NX, kR, 1>(v, lds, tau, twx, sync);
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            const size_t x = rowoff + i * T + tau;
            v[i] = c_mul(v[i], expi(k0dz * dn[x]));
            if (inten) inten[x] = c_abs2(v[i]);
        }
    }
    if constexpr (MODE == kTail) {
#pragma unroll
        for (int i = 0; i < kR; ++i) dst[rowoff + i * T + tau] = v[i];
    } else {
        fft_forward<NX, kR, 1>(v, lds, tau, twx, sync);
#pragma unroll
        for (int r = 0; r < kR; ++r) dst[rowoff + r * T + tau] = v[r];
    }
}

// ---------------------------------------------------------------------------
// column pass

template <int NY, bool CONJ>
__global__ __launch_bounds__(256) void col_pass(float2* work, const float2* __restrict__ H,
                                                const float2* __restrict__ twy, int nx) {
    constexpr int T = NY / kR, W = cols_per_block<NY>();
    extern __shared__ float2 smem[];
    const int w = threadIdx.x % W, t = threadIdx.x / W;
    // XCD-aware tile order: consecutive tiles (sharing cache lines) on one XCD
    const int tiles = nx / W, b = blockIdx.x;
    const int tile = (tiles % 8 == 0) ? (b % 8) * (tiles / 8) + b / 8 : b;
    const size_t col = (size_t)tile * W + w;
    float2* lds = smem + w;
    auto sync = [] { __syncthreads(); };
    float2 v[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = work[(size_t)(i * T + t) * nx + col];
    fft_forward<NY, kR, W>(v, lds, t, twy, sync);
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const float2 h = H[(size_t)(r * T + t) * nx + col];
        v[r] = CONJ ? c_mulc(v[r], h) : c_mul(v[r], h);
    }
    fft_inverse<NY, kR, W>(v, lds, t, twy, sync);
#pragma unroll
    for (int i = 0; i < kR; ++i) work[(size_t)(i * T + t) * nx + col] = v[i];
}

// ---------------------------------------------------------------------------
// launchers

template <int NX, int MODE>
static void launch_row_n(const float2* src, float2* dst, const float* dn, float* inten,
                         const float2* twx, float k0dz, int ny, hipStream_t s) {
    constexpr int T = NX / kR, B = rows_per_block<NX>();
    const size_t lds = sizeof(float2) * B * lds_size<NX>();
    row_pass<NX, MODE><<<ny / B, B * T, lds, s>>>(src, dst, dn, inten, twx, k0dz);
}

template <int MODE>
static hipError_t launch_row(int nx, const float2* src, float2* dst, const float* dn,
                             float* inten, const float2* twx, float k0dz, int ny,
                             hipStream_t s) {
    switch (nx) {
        case 32: launch_row_n<32, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        case 64: launch_row_n<64, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        case 128: launch_row_n<128, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        case 256: launch_row_n<256, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        case 512: launch_row_n<512, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        case 1024: launch_row_n<1024, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        case 2048: launch_row_n<2048, MODE>(src, dst, dn, inten, twx, k0dz, ny, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

template <int NY, bool CONJ>
static void launch_col_n(float2* work, const float2* H, const float2* twy, int nx,
                         hipStream_t s) {
    constexpr int T = NY / kR, W = cols_per_block<NY>();
    const size_t lds = sizeof(float2) * W * lds_size<NY>();
    col_pass<NY, CONJ><<<nx / W, W * T, lds, s>>>(work, H, twy, nx);
}

template <bool CONJ>
static hipError_t launch_col(int ny, float2* work, const float2* H, const float2* twy, int nx,
                             hipStream_t s) {
    switch (ny) {
        case 32: launch_col_n<32, CONJ>(work, H, twy, nx, s); break;
        case 64: launch_col_n<64, CONJ>(work, H, twy, nx, s); break;
        case 128: launch_col_n<128, CONJ>(work, H, twy, nx, s); break;
        case 256: launch_col_n<256, CONJ>(work, H, twy, nx, s); break;
        case 512: launch_col_n<512, CONJ>(work, H, twy, nx, s); break;
        case 1024: launch_col_n<1024, CONJ>(work, H, twy, nx, s); break;
        case 2048: launch_col_n<2048, CONJ>(work, H, twy, nx, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

hipError_t launch_forward(const Geom& g, const Plan& p, const MarchIO& io, hipStream_t s) {
    const size_t plane = (size_t)g.nx * g.ny;
    const float k0dz = (float)(2.0 * 3.14159265358979323846 / g.wavelength * g.dz);
    const float2* twx = (const float2*)p.twx;
    const float2* twy = (const float2*)p.twy;
    const float2* H = (const float2*)p.H;
    float2* work = (float2*)io.field_out;
    if (g.steps == 0) {
        if (io.field_out != io.field_in)
            return hipMemcpyAsync(io.field_out, io.field_in, plane * sizeof(float2),
                                  hipMemcpyDeviceToDevice, s);
        return hipSuccess;
    }
    hipError_t e = launch_row<kHead>(g.nx, (const float2*)io.field_in, work, nullptr, nullptr,
                                     twx, k0dz, g.ny, s);
    for (int j = 0; j < g.steps && e == hipSuccess; ++j) {
        e = launch_col<false>(g.ny, work, H, twy, g.nx, s);
        if (e != hipSuccess) break;
        const float* dnj = io.dn + j * plane;
        float* ij = io.intensity ? io.intensity + j * plane : nullptr;
        if (j + 1 < g.steps)
            e = launch_row<kMid>(g.nx, work, work, dnj, ij, twx, k0dz, g.ny, s);
        else
            e = launch_row<kTail>(g.nx, work, work, dnj, ij, twx, k0dz, g.ny, s);
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace bpm
