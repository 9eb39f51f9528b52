// Multiplexed point-source input field built on the device:
//
//   u0 = sum_i exp(i phi_i) shift(u_src, p_i),
//   u_src = IDFT2(S) / ||IDFT2(S)||,
//   S(k) = exp(-(kt / (k0 NA))^2) [kt <= k0 NA] exp(-i kz z_d)
//
// (Gaussian-apodised, NA-limited point source focusing z_d after the input
// plane; integer circular shifts).  The shifted sum is a circular convolution
// of the source with a comb of weighted deltas, so it is formed in the
// frequency domain: u0 = IDFT2(DFT2(comb) . S) / ||u_src||, with
// ||u_src||^2 = sum_k |S(k)|^2 / (nx ny) by Parseval.  The pupil test is the
// integer one of the readout: (m ny)^2 + (l nx)^2 <= (nx ny NA dx / lambda)^2.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace bpm {

__global__ void comb_zero_kernel(float2* c, long n) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x)
        c[e] = make_float2(0.f, 0.f);
}

__global__ void comb_scatter_kernel(const int* __restrict__ pos, const float* __restrict__ phase,
                                    int n_src, int nx, int ny, float* comb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_src) return;
    const int y = ((pos[2 * i] % ny) + ny) % ny, x = ((pos[2 * i + 1] % nx) + nx) % nx;
    float s = 0.f, c = 1.f;
    if (phase) sincosf(phase[i], &s, &c);
    float* p = comb + 2 * ((size_t)y * nx + x);
    atomicAdd(p, c);
    atomicAdd(p + 1, s);
}

struct SourceSpec {
    int nx, ny;
    double dx, k0, k, kmax2, pthr, z_d;
};

__device__ __forceinline__ bool source_mode(const SourceSpec& q, long e, double* amp,
                                            double* kz) {
    const int m = (int)(e % q.nx), l = (int)(e / q.nx);
    const long ms = m < q.nx / 2 ? m : m - q.nx, ls = l < q.ny / 2 ? l : l - q.ny;
    const long a = ms * q.ny, b = ls * q.nx;
    if ((double)(a * a + b * b) > q.pthr) return false;
    const double kPi = 3.14159265358979323846;
    const double kx = 2.0 * kPi * (double)ms / (q.nx * q.dx);
    const double ky = 2.0 * kPi * (double)ls / (q.ny * q.dx);
    const double kt2 = kx * kx + ky * ky;
    *amp = exp(-kt2 / q.kmax2);
    *kz = sqrt(fmax(q.k * q.k - kt2, 0.0));
    return true;
}

// sum_k |S(k)|^2 in double: kNormBlocks partial sums, then one block adds
// them in a fixed order (deterministic)
constexpr int kNormBlocks = 256;

__global__ void source_norm_partial_kernel(SourceSpec q, double* __restrict__ part) {
    __shared__ double red[256];
    const long n = (long)q.nx * q.ny;
    double s = 0.0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x) {
        double amp, kz;
        if (source_mode(q, e, &amp, &kz)) s += amp * amp;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void source_norm_final_kernel(const double* __restrict__ part, double* out) {
    __shared__ double red[kNormBlocks];
    red[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int st = kNormBlocks / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// C[k] <- C[k] S(k) / ||u_src||
__global__ void source_apply_kernel(SourceSpec q, const double* __restrict__ norm2, float2* C) {
    const long n = (long)q.nx * q.ny;
    const double inv = 1.0 / sqrt(norm2[0] / (double)n);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
         e += (long)gridDim.x * blockDim.x) {
        double amp, kz;
        float2 r = make_float2(0.f, 0.f);
        if (source_mode(q, e, &amp, &kz)) {
            double sv, cv;
            sincos(-kz * q.z_d, &sv, &cv);
            const double wr = amp * inv * cv, wi = amp * inv * sv;
            const float2 c = C[e];
            r = make_float2((float)(c.x * wr - c.y * wi), (float)(c.x * wi + c.y * wr));
        }
        C[e] = r;
    }
}

size_t sources_bytes(int nx, int ny) {
    return plan_bytes(nx, ny) + align_up(sizeof(float2) * (size_t)nx * ny) + kAlign +
           align_up(sizeof(double) * kNormBlocks);
}

hipError_t launch_point_sources(const SourceArgs& a, void* ws, hipStream_t s) {
    const long n = (long)a.nx * a.ny;
    char* b = static_cast<char*>(ws);
    const Plan p = plan_carve(b, a.nx, a.ny);
    b += plan_bytes(a.nx, a.ny);
    float2* comb = (float2*)b;
    b += align_up(sizeof(float2) * n);
    double* norm2 = (double*)b;
    b += kAlign;
    double* partial = (double*)b;
    const Geom g{a.nx, a.ny, 0, a.dx, 0.0, a.wavelength, a.n0};
    hipError_t e = launch_plan(g, p, false, s);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    comb_zero_kernel<<<blocks, 256, 0, s>>>(comb, n);
    if (a.n_src > 0)
        comb_scatter_kernel<<<(a.n_src + 255) / 256, 256, 0, s>>>(a.positions, a.phases, a.n_src,
                                                                  a.nx, a.ny, (float*)comb);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_fft2(comb, comb, a.nx, a.ny, false, 1.0f, p, s);
    if (e != hipSuccess) return e;
    const double kPi = 3.14159265358979323846;
    SourceSpec q{};
    q.nx = a.nx;
    q.ny = a.ny;
    q.dx = a.dx;
    q.k0 = 2.0 * kPi / a.wavelength;
    q.k = a.n0 * q.k0;
    q.kmax2 = (q.k0 * a.na) * (q.k0 * a.na);
    q.pthr = (double)a.nx * (double)a.ny * a.na * a.dx / a.wavelength;
    q.pthr *= q.pthr;
    q.z_d = a.z_d;
    source_norm_partial_kernel<<<kNormBlocks, 256, 0, s>>>(q, partial);
    source_norm_final_kernel<<<1, kNormBlocks, 0, s>>>(partial, norm2);
    source_apply_kernel<<<blocks, 256, 0, s>>>(q, norm2, comb);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = launch_fft2(comb, a.field_out, a.nx, a.ny, true, (float)(1.0 / (double)n), p, s);
    return e;
}

}  // namespace bpm
