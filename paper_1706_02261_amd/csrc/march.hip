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

constexpr int kR = 16;         // complex values per thread
constexpr int kBarWords = 1024;  // grid-barrier words (4 KiB) in the plan

// The field travels between the passes of the persistent march through
// global memory while the kernel runs.  The L2 caches of the eight XCDs are
// not coherent with each other, so every access to that buffer is an
// agent-scope relaxed atomic (a load that does not hit a stale L2 line, a
// store that writes through to the device coherence point).  Read-only data
// (propagator, twiddles, dn) keeps ordinary cached loads.
__device__ __forceinline__ float2 ld_shared_field(const float2* p) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, v);
}
__device__ __forceinline__ void st_shared_field(float2* p, float2 v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                       __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// plan

size_t plan_bytes(int nx, int ny) {
    return align_up(sizeof(float2) * (size_t)nx * ny) + align_up(sizeof(float2) * nx) +
           align_up(sizeof(float2) * ny) + sizeof(unsigned) * kBarWords;
}

Plan plan_carve(void* ws, int nx, int ny) {
    char* b = static_cast<char*>(ws);
    Plan p;
    p.H = b;
    b += align_up(sizeof(float2) * (size_t)nx * ny);
    p.twx = b;
    b += align_up(sizeof(float2) * nx);
    p.twy = b;
    b += align_up(sizeof(float2) * ny);
    p.counter = b;
    return p;
}

__global__ void plan_kernel(float2* __restrict__ H, float2* __restrict__ twx,
                            float2* __restrict__ twy, unsigned* __restrict__ counter, int nx,
                            int ny, double dx, double dz, double lam, double n0) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kBarWords; i += blockDim.x) counter[i] = 0u;
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
        (float2*)p.H, (float2*)p.twx, (float2*)p.twy, (unsigned*)p.counter, g.nx, g.ny, g.dx,
        g.dz, g.wavelength, g.n0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass bodies
//
// Every workgroup has 256 threads.  A row unit is B = 256 / (nx/16) rows, a
// column unit W = 256 / (ny/16) columns; units past the field's edge idle but
// still take part in the workgroup barriers.

enum RowMode { kHead = 0, kMid = 1, kTail = 2 };
constexpr int kBlock = 256;

template <int N>
constexpr int units_per_block() { return kBlock / (N / kR); }

// workgroup-wide and wavefront-wide LDS ordering points
struct BlockSync {
    __device__ __forceinline__ void operator()() const { __syncthreads(); }
};
struct WaveSync {
    __device__ __forceinline__ void operator()() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// row FFTs of at most one wavefront only need wavefront-wide LDS ordering
template <int N>
using RowSync = typename std::conditional<(N / kR <= 64), WaveSync, BlockSync>::type;

// screen: v[i] *= exp(i ph[i]); when every phase of the wavefront lies in
// [-pi/4, pi/4] (the usual case: k0 dz dn is a fraction of a radian) the
// range reduction is skipped.
__device__ __forceinline__ void apply_screen(float2 (&v)[kR], const float (&ph)[kR]) {
    bool small = true;
#pragma unroll
    for (int i = 0; i < kR; ++i) small &= fabsf(ph[i]) <= kQuarterPi;
    if (__all(small)) {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = c_mul(v[i], cos_sin_quarter(ph[i]));
    } else {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = c_mul(v[i], expi(ph[i]));
    }
}

// dn of this thread's row unit, fetched ahead of the row pass
template <int NX>
__device__ __forceinline__ void load_dn(float (&d)[kR], int unit, int ny,
                                        const float* __restrict__ dn) {
    constexpr int T = NX / kR, B = units_per_block<NX>();
    const int row = unit * B + threadIdx.x / T, tau = threadIdx.x % T;
    const size_t rowoff = (size_t)(row < ny ? row : 0) * NX;
#pragma unroll
    for (int i = 0; i < kR; ++i) d[i] = dn[rowoff + i * T + tau];
}

template <int NX, int MODE>
__device__ __forceinline__ void row_unit(int unit, int ny, const float2* src, float2* dst,
                                         const float (&d)[kR], float* __restrict__ inten,
                                         const Twiddles<NX, kR>& twx, float k0dz,
                                         float2* smem) {
    constexpr int T = NX / kR, B = units_per_block<NX>();
    const int sub = threadIdx.x / T, tau = threadIdx.x % T;
    const int row = unit * B + sub;
    const bool on = row < ny;  // rows past the edge compute on row 0 and store nothing
    const size_t rowoff = (size_t)(on ? row : 0) * NX;
    float2* lds = smem + sub * lds_size<NX>();
    const RowSync<NX> sync;
    float2 v[kR];
    if constexpr (MODE == kHead) {
#pragma unroll
        for (int i = 0; i < kR; ++i) v[i] = src[rowoff + i * T + tau];
    } else {
#pragma unroll
        for (int r = 0; r < kR; ++r) v[r] = ld_shared_field(src + rowoff + r * T + tau);
        fft_inverse<NX, kR, 1>(v, lds, tau, twx, sync);
        float ph[kR];
#pragma unroll
        for (int i = 0; i < kR; ++i) ph[i] = k0dz * d[i];
        apply_screen(v, ph);
        if (inten && on) {
#pragma unroll
            for (int i = 0; i < kR; ++i) inten[rowoff + i * T + tau] = c_abs2(v[i]);
        }
    }
    if constexpr (MODE == kTail) {
        if (on) {
#pragma unroll
            for (int i = 0; i < kR; ++i) dst[rowoff + i * T + tau] = v[i];
        }
    } else {
        fft_forward<NX, kR, 1>(v, lds, tau, twx, sync);
        if (on) {
#pragma unroll
            for (int r = 0; r < kR; ++r) st_shared_field(dst + rowoff + r * T + tau, v[r]);
        }
    }
}

template <int NY, bool CONJ>
__device__ __forceinline__ void col_unit(int unit, int nx, float2* work,
                                         const float2* __restrict__ H,
                                         const Twiddles<NY, kR>& twy, float2* smem) {
    constexpr int T = NY / kR, W = units_per_block<NY>();
    const int w = threadIdx.x % W, t = threadIdx.x / W;
    const int c = unit * W + w;
    const bool on = c < nx;  // columns past the edge compute on column 0 and store nothing
    const size_t col = on ? (size_t)c : 0;
    float2* lds = smem + w;
    const BlockSync sync;
    float2 v[kR], h[kR];
#pragma unroll
    for (int i = 0; i < kR; ++i) v[i] = ld_shared_field(work + (size_t)(i * T + t) * nx + col);
#pragma unroll
    for (int r = 0; r < kR; ++r) h[r] = H[(size_t)(r * T + t) * nx + col];
    fft_forward<NY, kR, W>(v, lds, t, twy, sync);
#pragma unroll
    for (int r = 0; r < kR; ++r) v[r] = CONJ ? c_mulc(v[r], h[r]) : c_mul(v[r], h[r]);
    fft_inverse<NY, kR, W>(v, lds, t, twy, sync);
    if (on) {
#pragma unroll
        for (int i = 0; i < kR; ++i) st_shared_field(work + (size_t)(i * T + t) * nx + col, v[i]);
    }
}

// ---------------------------------------------------------------------------
// grid barrier of the persistent march
//
// Two levels, no cache maintenance.  Workgroup b belongs to group b % 8 (the
// XCD the hardware deals it to).  Each arrival bumps its group's counter; the
// last arrival of a group bumps the global counter; the last group's closer
// publishes the barrier's generation to eight per-group flags, which the
// groups poll.  Every counter and flag sits in its own 128-byte line.  All of
// a wave's stores are complete (s_waitcnt) before its workgroup arrives, and
// the shared field is only accessed with agent-coherent operations, so no L2
// write-back or invalidation is needed.
//
// Every workgroup is resident (cooperative launch), so the wait ends; as a
// guard against a launch that is not, the spin is bounded and a time-out is
// recorded in the error word and ends all further waiting, so the kernel
// always exits.
//
// Barrier words (unsigned, zeroed by the plan kernel before every march):
//   [32 * g]        arrivals of group g        (g < 8)
//   [256 + 32 * g]  released generation of g
//   [512]           closed groups
//   [544]           time-out flag

constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ void grid_sync(unsigned* bar, unsigned gen, bool& abort) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned G = gridDim.x, g = blockIdx.x & 7u;
        const unsigned groups = G < 8u ? G : 8u;
        const unsigned members = (G - g + 7u) / 8u;
        const unsigned old = __hip_atomic_fetch_add(bar + 32 * g, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == gen * members) {
            const unsigned o2 = __hip_atomic_fetch_add(bar + 512, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (o2 + 1u == gen * groups)
                for (unsigned k = 0; k < groups; ++k)
                    __hip_atomic_store(bar + 256 + 32 * k, gen, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        unsigned spins = 0;
        while (!abort && __hip_atomic_load(bar + 256 + 32 * g, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) < gen) {
            if (++spins > kSpinLimit) {
                __hip_atomic_store(bar + 544, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                abort = true;
            }
        }
    }
    __syncthreads();
}

struct MarchArgs {
    const float2* field_in;
    float2* work;
    const float* dn;
    float* inten;
    const float2* H;
    const float2* twx;
    const float2* twy;
    unsigned* counter;
    int nx, ny, steps;
    float k0dz;
};

template <int NX, int NY>
__global__ __launch_bounds__(kBlock) void march_kernel(MarchArgs a) {
    extern __shared__ float2 smem[];
    const int G = gridDim.x, b = blockIdx.x;
    // XCD-aware order: workgroups are dealt round-robin over the 8 XCDs, so
    // give each XCD a contiguous range of units (neighbouring columns share
    // cache lines)
    const int v = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    const int rows_u = (a.ny + units_per_block<NX>() - 1) / units_per_block<NX>();
    const int cols_u = (a.nx + units_per_block<NY>() - 1) / units_per_block<NY>();
    const size_t plane = (size_t)a.nx * a.ny;
    unsigned nbar = 0;
    bool abort = false;
    Twiddles<NX, kR> twx;
    Twiddles<NY, kR> twy;
    twx.load(a.twx, threadIdx.x % (NX / kR));
    twy.load(a.twy, threadIdx.x / units_per_block<NY>());
    float d[kR];
    for (int i = 0; i < kR; ++i) d[i] = 0.f;
    for (int u = v; u < rows_u; u += G)
        row_unit<NX, kHead>(u, a.ny, a.field_in, a.work, d, nullptr, twx, a.k0dz, smem);
    // a workgroup with a single row unit fetches its dn slice during the column pass
    const bool one_row_unit = rows_u <= G;
    for (int j = 0; j < a.steps; ++j) {
        const float* dnj = a.dn + j * plane;
        float* ij = a.inten ? a.inten + j * plane : nullptr;
        if (one_row_unit) load_dn<NX>(d, v < rows_u ? v : 0, a.ny, dnj);
        grid_sync(a.counter, ++nbar, abort);
        for (int u = v; u < cols_u; u += G) col_unit<NY, false>(u, a.nx, a.work, a.H, twy, smem);
        grid_sync(a.counter, ++nbar, abort);
        for (int u = v; u < rows_u; u += G) {
            if (!one_row_unit) load_dn<NX>(d, u, a.ny, dnj);
            if (j + 1 < a.steps)
                row_unit<NX, kMid>(u, a.ny, a.work, a.work, d, ij, twx, a.k0dz, smem);
            else
                row_unit<NX, kTail>(u, a.ny, a.work, a.work, d, ij, twx, a.k0dz, smem);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
    }
    return cus;
}

template <int NX, int NY>
static hipError_t launch_march_n(MarchArgs a, hipStream_t s) {
    constexpr int BX = units_per_block<NX>(), WY = units_per_block<NY>();
    const int rows_u = (a.ny + BX - 1) / BX, cols_u = (a.nx + WY - 1) / WY;
    const int cus = device_cus();
    if (cus <= 0) return hipErrorNoDevice;
    int grid = rows_u > cols_u ? rows_u : cols_u;
    if (grid > cus) grid = cus;
    const size_t lds_r = sizeof(float2) * BX * lds_size<NX>();
    const size_t lds_c = sizeof(float2) * WY * lds_size<NY>();
    const size_t lds = lds_r > lds_c ? lds_r : lds_c;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&march_kernel<NX, NY>),
                                      dim3(grid), dim3(kBlock), args, (unsigned)lds, s);
}

template <int NX>
static hipError_t launch_march_x(MarchArgs a, hipStream_t s) {
    switch (a.ny) {
        case 32: return launch_march_n<NX, 32>(a, s);
        case 64: return launch_march_n<NX, 64>(a, s);
        case 128: return launch_march_n<NX, 128>(a, s);
        case 256: return launch_march_n<NX, 256>(a, s);
        case 512: return launch_march_n<NX, 512>(a, s);
        case 1024: return launch_march_n<NX, 1024>(a, s);
        case 2048: return launch_march_n<NX, 2048>(a, s);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_march(MarchArgs a, hipStream_t s) {
    switch (a.nx) {
        case 32: return launch_march_x<32>(a, s);
        case 64: return launch_march_x<64>(a, s);
        case 128: return launch_march_x<128>(a, s);
        case 256: return launch_march_x<256>(a, s);
        case 512: return launch_march_x<512>(a, s);
        case 1024: return launch_march_x<1024>(a, s);
        case 2048: return launch_march_x<2048>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(const Geom& g, const Plan& p, const MarchIO& io, hipStream_t s) {
    const size_t plane = (size_t)g.nx * g.ny;
    if (g.steps == 0) {
        if (io.field_out != io.field_in)
            return hipMemcpyAsync(io.field_out, io.field_in, plane * sizeof(float2),
                                  hipMemcpyDeviceToDevice, s);
        return hipSuccess;
    }
    MarchArgs a;
    a.field_in = (const float2*)io.field_in;
    a.work = (float2*)io.field_out;
    a.dn = io.dn;
    a.inten = io.intensity;
    a.H = (const float2*)p.H;
    a.twx = (const float2*)p.twx;
    a.twy = (const float2*)p.twy;
    a.counter = (unsigned*)p.counter;
    a.nx = g.nx;
    a.ny = g.ny;
    a.steps = g.steps;
    a.k0dz = (float)(2.0 * 3.14159265358979323846 / g.wavelength * g.dz);
    return launch_march(a, s);
}

}  // namespace bpm
